"""GPU parity on the benchmark configurations, at their full sizes where the
benchmark runs them.

* Differentiable step on the 8 pads: full model, GPU gradients of the pose
  (6-DoF), alpha and sampled Phi entries of every layer against FP64 central
  differences of the oracle, and the whole Phi gradient against its adjoint.
* The 4096-env hand in the benchmark's launch configuration: alpha and Phi
  gradients of 64 sampled envs against the oracle (dL/dU zero elsewhere).
* High-resolution pads (4096 envs x 4 x 128^2 nodes): the full-model adjoint
  of sampled items, with a network whose decisions are far from their
  boundaries (see below).
* The graph-captured rollout (16384 envs x 200 steps): U and contact of 64
  sampled envs at steps 0, 99 and 199 against the oracle.

The model is only piecewise smooth (ReLU gates, max-pool arg-max): an item
whose decision lies within FP32 rounding of its boundary may take the other
branch on the GPU, so gradients are compared on items whose oracle decision
margin clears MARGIN, with dL/dU zero on every other item (their
contributions then vanish identically).
"""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL
from tests.gpu_util import DevModel, DevScene, TOL_U, log, make_plan, max_err, to_dev, torch_dev
from tests.test_gpu_backward import MARGIN, _close, gpu_step_backward

pytestmark = pytest.mark.gpu

PHI_BLOCKS = (("W1", 576), ("b1", 64), ("W2", 4096), ("b2", 64), ("W3", 4096), ("b3", 64), ("W4", 8192),
              ("b4", 64), ("W5", 192), ("b5", 3))


def clean_pad_seeds(oracle_lib, n=8, search=3000):
    """The first n pad seeds (config-1 geometry) whose env clears MARGIN under
    the model shared by the differentiable-step envs (config 1's model of
    seed 0)."""
    mesh, scene, model, _ = scenes.config3(seeds=range(search), model_seed=0)
    out = oracle_lib.forward(mesh, scene, model, with_sig=True)
    seeds = [int(s) for s in np.nonzero(out["margin"] > MARGIN)[0][:n]]
    assert len(seeds) == n
    return seeds


def test_config3_full_model_vs_central_fd(oracle_lib):
    seeds = clean_pad_seeds(oracle_lib)
    mesh, scene, model, w = scenes.config3(seeds=seeds, model_seed=0)
    out = oracle_lib.forward(mesh, scene, model, with_sig=True)
    assert np.all(out["margin"] > MARGIN)
    log(f"[gpu] config 3, full model, pad seeds {seeds}: 8 of 8 envs clear the margin")
    off = scenes.phi_offsets()
    rng = np.random.default_rng(5)
    plan = make_plan(mesh, 1, 1, backward=True)
    n_phi = 0
    per_block = {b: 0 for b, _ in PHI_BLOCKS}
    for e in range(8):
        sc, we = scene.select([e]), w[:, e:e + 1]
        g = gpu_step_backward(plan, sc, model, we)
        ref = oracle_lib.backward(mesh, sc, model, we)
        _close(g["grad_phi"], ref["grad_phi"], f"env {e} grad_phi vs adjoint")
        # Phi entries of every block whose adjoint gradient is not negligible
        idx = []
        for b, size in PHI_BLOCKS:
            gb = np.abs(ref["grad_phi"][off[b]:off[b] + size])
            cand = np.nonzero(gb > 1e-2 * gb.max())[0]
            idx += [int(off[b] + i) for i in rng.choice(cand, size=min(4, len(cand)), replace=False)]
        fd, _ = oracle_lib.fd_gradients(mesh, sc, model, we, phi_idx=idx, shrink=(1e-5, 1e-6, 1e-7, 1e-8))
        ok = fd["ok_each"]
        assert ok["trans"].all() and ok["twist"].all() and ok["alpha"].all(), e
        # pose (translation and twist), alpha
        tw = oracle_lib.twist_from_grad_rot(g["grad_rot"][0, 0], sc.rot[0, 0])
        scale = max(np.abs(fd["trans"]).max(), np.abs(fd["twist"]).max(), 1e-3)
        assert np.max(np.abs(g["grad_trans"][0, 0] - fd["trans"])) <= 1e-4 * scale + 1e-6, e
        assert np.max(np.abs(tw - fd["twist"])) <= 1e-4 * scale + 1e-6, e
        assert np.max(np.abs(g["grad_alpha"] - fd["alpha"])) <= 1e-4 * np.abs(fd["alpha"]).max() + 1e-6, e
        # Phi entries: GPU against FD, bounded by the env's largest Phi gradient
        pb = 1e-4 * np.abs(ref["grad_phi"]).max() + 1e-6
        sel = np.array(idx)[ok["phi"]]
        err = np.abs(g["grad_phi"][sel] - fd["phi"][ok["phi"]])
        log(f"[gpu]   env {e}: pose, alpha and {len(sel)} Phi entries vs FD, max Phi err {err.max():.3e} "
            f"(bound {pb:.3e})")
        assert np.all(err <= pb), e
        n_phi += len(sel)
        for i in sel:
            b = [bb for bb, size in PHI_BLOCKS if off[bb] <= i < off[bb] + size][0]
            per_block[b] += 1
    log(f"[gpu]   Phi entries checked per block {per_block}")
    assert n_phi >= 64
    assert all(v > 0 for v in per_block.values())


def test_config2_full_size_alpha_phi_sampled(oracle_lib):
    # the benchmark's 4096-env hand and launch configuration (forward with the
    # pooling record, adjoint given it), dL/dU ~ N(0,1) on 64 sampled envs
    # that clear the margin and zero elsewhere
    mesh, scene, model = scenes.config2(n_envs=4096)
    rng = np.random.default_rng(13)
    perm = rng.permutation(4096)
    envs = []
    for c0 in range(0, 4096, 256):
        cand = np.sort(perm[c0:c0 + 256])
        out = oracle_lib.forward(mesh, scene.select(cand), model, with_sig=True)
        ok = (out["margin"] > MARGIN) & (out["n_active"].sum(axis=1) > 0)
        envs += [int(e) for e in cand[ok]]
        if len(envs) >= 64:
            break
    envs = np.sort(np.array(envs[:64]))
    assert len(envs) == 64
    w = np.zeros((3, 4096, mesh.n_nodes), np.float32)
    w[:, envs] = np.random.default_rng(21).standard_normal((3, 64, mesh.n_nodes))
    plan = make_plan(mesh, 4096, scene.max_obj, backward=True)
    log(f"[gpu] hand E=4096, full model: gradients of 64 sampled envs vs the oracle")
    g = gpu_step_backward(plan, scene, model, w, saved=True)
    ref = oracle_lib.backward(mesh, scene.select(envs), model, w[:, envs].astype(np.float64))
    _close(g["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    _close(g["grad_phi"], ref["grad_phi"], "grad_phi")
    _close(g["grad_trans"][envs], ref["grad_trans"], "grad_trans")
    _close(g["grad_rot"][envs], ref["grad_rot"], "grad_rot")
    others = np.setdiff1d(np.arange(4096), envs)
    assert np.all(g["grad_trans"][others] == 0.0) and np.all(g["grad_rot"][others] == 0.0)


def separated_phi(model, X):
    """The seeded weights with biases that keep every ReLU input at least one
    unit away from zero: b_j = +-(2 B + 1) with B a bound of |W x| over the
    layer's inputs (X bounds every node input), alternating signs, so half
    the units are always on and half always off.  W3 and W4[:, 64:] are zero,
    so the pooled feature and its arg-max enter neither U nor any gradient.
    Used where a patch has so many nodes that some seeded pre-activation, or
    some max-pool runner-up, always lies within FP32 rounding of its
    boundary; the max-pool routing is checked on the smaller configurations."""
    off = scenes.phi_offsets()
    p = model.phi.astype(np.float64).copy()
    sign = np.where(np.arange(64) % 2 == 0, 1.0, -1.0)

    def block(name, o, i):
        return p[off[name]:off[name] + o * i].reshape(o, i)

    W1, W2, W4 = block("W1", 64, 9), block("W2", 64, 64), block("W4", 64, 128)
    block("W3", 64, 64)[:] = 0.0
    W4[:, 64:] = 0.0
    n1, n2, n4 = (np.abs(W).sum(1).max() for W in (W1, W2, W4))
    b1 = 2 * n1 * X + 1
    h1 = n1 * X + b1                       # bound of the live h1
    b2 = 2 * n2 * h1 + 1
    f = n2 * h1 + b2
    b4 = 2 * n4 * f + 1
    for name, b in (("b1", b1), ("b2", b2), ("b4", b4)):
        p[off[name]:off[name] + 64] = sign * b
    return p.astype(np.float32)


def test_hires_full_model_adjoint_sampled(oracle_lib):
    # every contacted item of 6 sampled envs, decisions certain by
    # construction (separated_phi); U of those envs relative to max |U|
    # (the residuals are large with these biases)
    mesh, scene, model = scenes.config4(n_envs=4096, mode=MODE_FULL)
    reach = np.abs(mesh.pos - np.repeat(mesh.origin.T, np.diff(mesh.patch_offset), axis=1)).max()
    X = float(reach) + float(scene.shape[..., :3].max())        # |p - o|, |n| <= 1, |u_hat| <= object size
    m = scenes.Model(MODE_FULL, model.alpha, separated_phi(model, X))
    envs = np.sort(np.random.default_rng(4).choice(4096, size=6, replace=False))
    w = np.zeros((3, 4096, mesh.n_nodes), np.float32)
    w[:, envs] = np.random.default_rng(12).standard_normal((3, len(envs), mesh.n_nodes))
    plan = make_plan(mesh, 4096, 4, backward=True)
    from tests.gpu_util import gpu_step
    u, cobj, _ = gpu_step(plan, scene, m)
    ref_f = oracle_lib.forward(mesh, scene.select(envs), m)
    assert np.array_equal(cobj[envs], ref_f["contact_obj"])
    err = max_err(u[:, envs], ref_f["u"])
    mx = float(np.abs(ref_f["u"]).max())
    log(f"[gpu] hires E=4096, full model (separated decisions): {int((ref_f['n_active'] > 0).sum())} contacted "
        f"items in {len(envs)} sampled envs, max|dU| {err:.3e} of max|U| {mx:.3e}")
    assert err <= 2e-5 * mx
    g = gpu_step_backward(plan, scene, m, w, saved=True)
    ref = oracle_lib.backward(mesh, scene.select(envs), m, w[:, envs].astype(np.float64))
    _close(g["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    _close(g["grad_phi"], ref["grad_phi"], "grad_phi")
    _close(g["grad_trans"][envs], ref["grad_trans"], "grad_trans")
    _close(g["grad_rot"][envs], ref["grad_rot"], "grad_rot")


def test_rollout_spot_checks(oracle_lib):
    # 16384 envs of the hand, 200 steps of smooth object motion, the step
    # replayed from one HIP graph with the poses selected by a device step
    # counter (the benchmark's rollout); 64 sampled envs at steps 0, 99, 199
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh = scenes.hand_mesh(0)
    E, T = 16384, 200
    scene = scenes.hand_scene(mesh, E, 1)
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_FULL)
    traj_rot, traj_trans = scenes.trajectory(scene, T, seed=5)
    O, N, K = scene.max_obj, mesh.n_nodes, mesh.n_patches
    plan = make_plan(mesh, E, O)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    trot, ttr = to_dev(traj_rot), to_dev(traj_trans)
    step_idx = torch.zeros(1, dtype=torch.long, device=dev)
    u = torch.empty((3, E, N), device=dev)
    cobj = torch.empty((E, N), dtype=torch.int8, device=dev)
    na = torch.empty((E, K), dtype=torch.int32, device=dev)

    def body():
        ds.rot.copy_(torch.index_select(trot, 0, step_idx)[0])
        ds.trans.copy_(torch.index_select(ttr, 0, step_idx)[0])
        _native.etac_step(plan, sc, md, u, cobj, na)
        step_idx.add_(1).remainder_(T)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    step_idx.zero_()
    envs = np.sort(np.random.default_rng(8).choice(E, size=64, replace=False))
    ie = torch.from_numpy(envs).to(dev)
    got = {}
    log(f"[gpu] rollout E={E}, {T} steps from one graph")
    for s in range(T):
        g.replay()
        if s in (0, 99, 199):
            torch.cuda.synchronize()
            got[s] = (u.index_select(1, ie).cpu().numpy(), cobj.index_select(0, ie).cpu().numpy(),
                      na.index_select(0, ie).cpu().numpy())
    torch.cuda.synchronize()
    assert int(step_idx.item()) == 0
    for s, (us, cs, ns) in got.items():
        sub = scene.select(envs)
        sub.rot, sub.trans = traj_rot[s][envs], traj_trans[s][envs]
        ref = oracle_lib.forward(mesh, sub, model)
        err = max_err(us, ref["u"])
        log(f"[gpu]   step {s}: active nodes {int(ref['n_active'].sum())}, max|dU| {err:.3e} mm")
        assert np.array_equal(cs, ref["contact_obj"]), s
        assert np.array_equal(ns, ref["n_active"]), s
        assert err <= TOL_U, s
