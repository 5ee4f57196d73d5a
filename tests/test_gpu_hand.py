"""GPU parity of the articulated-hand calls (link frames, self-contact and
the contact reward) against the FP64 oracle: contact, ids and reward counts
bit-exact, displacements within TOL_U, pose gradients of objects and links
within the adjoint bars."""
import numpy as np
import pytest

import oracle
import scenes
from scenes import articulated as art
from tests.gpu_util import TOL_U, DevModel, DevScene, log, make_plan, max_err, to_dev, torch_dev
from tests.test_gpu_backward import _close

pytestmark = pytest.mark.gpu

OMEGA = 0.5


class DevHand:
    """A plan with the hand attached, and the device copies of one workload."""

    def __init__(self, h, mesh, scene, links, model, backward=False):
        from paper_2604_20295_amd import _native
        torch, dev = torch_dev()
        self.plan = make_plan(mesh, scene.n_envs, scene.max_obj, backward=backward)
        self.plan.set_hand(h)
        self.ds, self.dm = DevScene(scene), DevModel(model)
        self.lrot = to_dev(links.rot.astype(np.float32))
        self.ltr = to_dev(links.trans.astype(np.float32))
        self.E, self.O, self.N, self.K = scene.n_envs, scene.max_obj, mesh.n_nodes, mesh.n_patches
        self.L = h.n_links
        self._n = _native

    def structs(self):
        return self.ds.struct(self.plan), self.plan.links_struct(self.lrot, self.ltr)

    def reward(self):
        torch, dev = torch_dev()
        out = dict(n_touch=torch.full((self.E, self.K), -3, dtype=torch.int32, device=dev),
                   n_a=torch.full((self.E,), -3, dtype=torch.int32, device=dev),
                   link_mask=torch.full((self.E,), -3, dtype=torch.int32, device=dev),
                   r_contact=torch.full((self.E,), float("nan"), device=dev))
        return out, self.plan.reward_struct(self.E, OMEGA, **out)

    def contact(self):
        torch, dev = torch_dev()
        sc, lk = self.structs()
        cobj = torch.full((self.E, self.N), 99, dtype=torch.int8, device=dev)
        uhat = torch.full((3, self.E, self.N), float("nan"), device=dev)
        na = torch.full((self.E, self.K), -7, dtype=torch.int32, device=dev)
        rw, rs = self.reward()
        self._n.etac_hand_contact(self.plan, sc, lk, cobj, uhat, na, rs)
        torch.cuda.synchronize()
        return dict(contact_obj=cobj.cpu().numpy(), uhat=uhat.cpu().numpy(), n_active=na.cpu().numpy(),
                    **{k: v.cpu().numpy() for k, v in rw.items()})

    def step(self, mode=None, saved=None):
        torch, dev = torch_dev()
        sc, lk = self.structs()
        u = torch.full((3, self.E, self.N), float("nan"), device=dev)
        cobj = torch.full((self.E, self.N), 99, dtype=torch.int8, device=dev)
        na = torch.full((self.E, self.K), -7, dtype=torch.int32, device=dev)
        rw, rs = self.reward()
        self._n.etac_hand_step(self.plan, sc, lk, self.dm.struct(self.plan, mode), u, cobj, na, rs, saved=saved)
        torch.cuda.synchronize()
        return dict(u=u.cpu().numpy(), contact_obj=cobj.cpu().numpy(), n_active=na.cpu().numpy(),
                    **{k: v.cpu().numpy() for k, v in rw.items()})

    def backward(self, grad_u, saved=None):
        torch, dev = torch_dev()
        sc, lk = self.structs()
        g = dict(grad_rot=torch.empty((self.E, self.O, 9), device=dev),
                 grad_trans=torch.empty((self.E, self.O, 3), device=dev),
                 grad_link_rot=torch.empty((self.E, self.L, 9), device=dev),
                 grad_link_trans=torch.empty((self.E, self.L, 3), device=dev),
                 grad_alpha=torch.empty((self.K,), device=dev),
                 grad_phi=torch.empty((scenes.PHI_SIZE,), device=dev))
        self._n.etac_hand_step_backward(self.plan, sc, lk, self.dm.struct(self.plan), to_dev(grad_u.astype(np.float32)),
                                        g["grad_rot"], g["grad_trans"], g["grad_link_rot"], g["grad_link_trans"],
                                        g["grad_alpha"], g["grad_phi"], saved=saved)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in g.items()}


def _check_contact(got, ref, O):
    assert np.array_equal(got["contact_obj"], ref["contact_obj"])
    assert np.array_equal(got["n_active"], ref["n_active"])
    assert np.array_equal(got["n_touch"], ref["n_touch"])
    assert np.array_equal(got["n_a"], ref["n_a"])
    assert np.array_equal(got["link_mask"].view(np.uint32), ref["link_mask"])
    assert np.allclose(got["r_contact"], ref["r_contact"], rtol=1e-6, atol=1e-7)
    n_self = int((ref["contact_obj"] >= O).sum())
    n_obj = int(((ref["contact_obj"] >= 0) & (ref["contact_obj"] < O)).sum())
    return n_self, n_obj


def test_hand_contact_and_reward_match_oracle(oracle_lib):
    h, mesh, scene, links, model = art.config_hand(n_envs=96, seed=2)
    d = DevHand(h, mesh, scene, links, model)
    log("[gpu] hand contact: 96 envs of the 16-link hand")
    got = d.contact()
    ref = oracle.hand_forward(mesh, h, scene, links, model, omega_a=OMEGA)
    n_self, n_obj = _check_contact(got, ref, scene.max_obj)
    assert n_self > 0 and n_obj > 0
    assert max_err(got["uhat"], ref["uhat"]) <= TOL_U
    log(f"[gpu]   {n_obj} object-contact and {n_self} self-contact nodes, max|du_hat| "
        f"{max_err(got['uhat'], ref['uhat']):.3e} mm")


@pytest.mark.parametrize("mode", [scenes.MODE_FULL, scenes.MODE_DECAY_ONLY, scenes.MODE_RESIDUAL_ONLY])
def test_hand_step_matches_oracle(oracle_lib, mode):
    h, mesh, scene, links, model = art.config_hand(n_envs=64, seed=3, mode=mode)
    d = DevHand(h, mesh, scene, links, model)
    log(f"[gpu] hand step: 64 envs, mode {mode}")
    got = d.step()
    ref = oracle.hand_forward(mesh, h, scene, links, model, omega_a=OMEGA)
    _check_contact(got, ref, scene.max_obj)
    err = max_err(got["u"], ref["u"])
    log(f"[gpu]   max|dU| {err:.3e} mm of max|U| {np.abs(ref['u']).max():.3e}")
    assert err <= TOL_U


def test_hand_with_identity_links_equals_the_plain_step(oracle_lib):
    # every link at the identity and no self-contact pairs: the rows hold the
    # env's objects unchanged, so the hand step reproduces etac_step bit for bit
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=48)
    K = mesh.n_patches
    h = art.Hand(K, np.full(K, -1, np.int32), np.arange(K, dtype=np.int32), np.zeros(K, np.uint32),
                 np.full(K, art.NONE, np.int32), np.zeros((K, 4), np.float32),
                 np.tile(np.eye(3, dtype=np.float32).ravel(), (K, 1)), np.zeros((K, 3), np.float32),
                 np.zeros((K, 3)), np.tile(np.eye(3), (K, 1, 1)))
    d = DevHand(h, mesh, scene, art.identity_links(h, scene.n_envs), model)
    log("[gpu] hand step with identity links vs etac_step: 48-env hand")
    got = d.step()
    u = torch.empty((3, d.E, d.N), device=dev)
    cobj = torch.empty((d.E, d.N), dtype=torch.int8, device=dev)
    na = torch.empty((d.E, d.K), dtype=torch.int32, device=dev)
    _native.etac_step(d.plan, d.ds.struct(d.plan), d.dm.struct(d.plan), u, cobj, na)
    torch.cuda.synchronize()
    assert np.array_equal(got["u"], u.cpu().numpy())
    assert np.array_equal(got["contact_obj"], cobj.cpu().numpy())
    assert np.array_equal(got["n_active"], na.cpu().numpy())
    assert np.array_equal(got["n_touch"], got["n_active"])


def _item_mask(ref, mesh, mode):
    """dL/dU weights kept on the items whose network decisions clear the margin
    (all items for decay-only); zero elsewhere, which makes those items'
    contributions vanish identically whatever branch FP32 takes."""
    keep = (ref["margin"] > 5e-6) if mode != scenes.MODE_DECAY_ONLY else np.ones_like(ref["margin"], bool)
    node_keep = np.repeat(keep, np.diff(mesh.patch_offset), axis=1)    # [E][N]
    return keep, node_keep


@pytest.mark.parametrize("mode", [scenes.MODE_DECAY_ONLY, scenes.MODE_FULL])
def test_hand_adjoint_matches_oracle(oracle_lib, mode):
    h, mesh, scene, links, model = art.config_hand(n_envs=64, seed=5, mode=mode)
    ref = oracle.hand_forward(mesh, h, scene, links, model, with_margin=True)
    keep, node_keep = _item_mask(ref, mesh, mode)
    contacted = ref["n_active"] > 0
    assert (keep & contacted).sum() >= 64, (keep & contacted).sum()
    w = np.random.default_rng(7).standard_normal((3, scene.n_envs, mesh.n_nodes))
    w *= node_keep[None]
    d = DevHand(h, mesh, scene, links, model, backward=True)
    log(f"[gpu] hand adjoint: mode {mode}, dL/dU on {(keep & contacted).sum()} of {contacted.sum()} contacted items")
    got = d.backward(w)
    g = oracle.hand_backward(mesh, h, scene, links, model, w.astype(np.float32).astype(np.float64))
    for key in ("grad_trans", "grad_rot", "grad_link_trans", "grad_link_rot", "grad_alpha"):
        _close(got[key], g[key], key)
    if mode == scenes.MODE_FULL:
        _close(got["grad_phi"], g["grad_phi"], "grad_phi")
    # envs whose contacted items all carry no dL/dU have exactly zero pose gradients
    silent = ~(keep & contacted).any(axis=1)
    for key in ("grad_trans", "grad_rot", "grad_link_trans", "grad_link_rot"):
        assert not np.any(got[key][silent]), key


def test_hand_adjoint_with_the_pooling_record(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    h, mesh, scene, links, model = art.config_hand(n_envs=32, seed=6)
    d = DevHand(h, mesh, scene, links, model, backward=True)
    w = np.random.default_rng(8).standard_normal((3, scene.n_envs, mesh.n_nodes))
    rec = _native.saved_buffer(d.plan, scene.n_envs)
    d.step(saved=rec)
    log("[gpu] hand adjoint from the pooling record vs recomputed: 32 envs")
    a = d.backward(w, saved=rec)
    b = d.backward(w)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_hand_full_size_contact_and_sampled_displacements(oracle_lib):
    # the 4096-env hand workload in the launch shape the benchmark uses:
    # contact and reward of every env, U of sampled envs
    h, mesh, scene, links, model = art.config_hand(n_envs=4096)
    d = DevHand(h, mesh, scene, links, model, backward=True)
    d.plan.set_launch(2, 4, 4, 3, 2)
    log("[gpu] hand full size: 4096 envs, contact of every env, U of 64 sampled envs")
    got = d.step()
    ref = oracle.hand_forward(mesh, h, scene, links, model.with_mode(scenes.MODE_DECAY_ONLY), omega_a=OMEGA)
    _check_contact(got, ref, scene.max_obj)
    envs = np.random.default_rng(3).choice(scene.n_envs, 64, replace=False)
    sub = oracle.hand_forward(mesh, h, scene.select(envs), links.select(envs), model, omega_a=OMEGA)
    err = max_err(got["u"][:, envs], sub["u"])
    log(f"[gpu]   max|dU| {err:.3e} mm on the sampled envs")
    assert err <= TOL_U


def test_hand_step_graph_replays(oracle_lib):
    # the pre-pass, the fused step and the reward kernel captured in one HIP
    # graph; replays with eager work in between reproduce the eager result
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    h, mesh, scene, links, model = art.config_hand(n_envs=64, seed=9)
    d = DevHand(h, mesh, scene, links, model)
    eager = d.step()
    sc, lk = d.structs()
    md = d.dm.struct(d.plan)
    u = torch.empty((3, d.E, d.N), device=dev)
    cobj = torch.empty((d.E, d.N), dtype=torch.int8, device=dev)
    na = torch.empty((d.E, d.K), dtype=torch.int32, device=dev)
    rw, rs = d.reward()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _native.etac_hand_step(d.plan, sc, lk, md, u, cobj, na, rs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _native.etac_hand_step(d.plan, sc, lk, md, u, cobj, na, rs)
    log("[gpu] hand step graph: 3 replays")
    for r in range(3):
        u.fill_(float("nan"))
        rw["r_contact"].fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), eager["u"]), r
        assert np.array_equal(cobj.cpu().numpy(), eager["contact_obj"]), r
        assert np.array_equal(rw["r_contact"].cpu().numpy(), eager["r_contact"]), r
        d.contact()      # eager work between replays


def test_hand_autograd_binding(oracle_lib):
    # ETacHandStep: U and r_contact as etac_hand_step gives them, gradients of
    # sum(w * U) as etac_hand_step_backward gives them (same kernels)
    from paper_2604_20295_amd.autograd import etac_hand_step
    torch, dev = torch_dev()
    h, mesh, scene, links, model = art.config_hand(n_envs=16, seed=12, mode=scenes.MODE_DECAY_ONLY)
    d = DevHand(h, mesh, scene, links, model, backward=True)
    leaves = [x.clone().requires_grad_(True) for x in (d.ds.rot, d.ds.trans, d.lrot, d.ltr, d.dm.alpha)]
    log("[gpu] hand autograd binding: 16 envs, decay-only")
    u, cobj, na, r = etac_hand_step(d.plan, d.ds.n_obj, d.ds.type, d.ds.shape, *leaves, d.dm.phi,
                                    scenes.MODE_DECAY_ONLY, OMEGA)
    w = np.random.default_rng(3).standard_normal((3, d.E, d.N)).astype(np.float32)
    (u * to_dev(w)).sum().backward()
    torch.cuda.synchronize()
    ref = d.step()
    assert np.array_equal(u.detach().cpu().numpy(), ref["u"])
    assert np.array_equal(r.cpu().numpy(), ref["r_contact"])
    g = d.backward(w)
    for leaf, key in zip(leaves, ("grad_rot", "grad_trans", "grad_link_rot", "grad_link_trans", "grad_alpha")):
        assert np.array_equal(leaf.grad.cpu().numpy(), g[key]), key
