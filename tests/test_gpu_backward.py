"""GPU parity of the adjoint (etac_step_backward, etac_propagate_backward,
etac_contact_backward) against the FP64 oracle's adjoint and against FP64
central finite differences of the oracle.

The model is piecewise smooth: ReLU gates and the max-pool arg-max are
discrete decisions.  FP32 pre-activations differ from FP64 by up to ~2e-6 on
these workloads, so where a decision lies within that distance of its boundary
both branches are valid and the FP32 and FP64 gradients may legitimately take
different ones.  The oracle reports, per env, the smallest distance of any
such decision from its boundary; envs below MARGIN are left out (their objects
are removed, so their items carry no gradient) and the rest must match to
|dG| <= 1e-4 max|G| + 1e-6 per gradient block.  Decay-only mode has no such
decisions and is compared on every env.  Contact decisions are bit-exact and
never excluded."""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY
from tests.gpu_util import DevModel, DevScene, log, make_plan, to_dev, torch_dev

pytestmark = pytest.mark.gpu

MARGIN = 5e-6
SMALL = dict(sizes=(64, 128, 256), scale=0.2, placement="press")   # small-patch hand: many envs clear the margin


def _close(gpu, ref, name, rel=1e-4, atol=1e-6):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = float(np.max(np.abs(gpu - ref))) if ref.size else 0.0
    mx = float(np.max(np.abs(ref))) if ref.size else 0.0
    bound = rel * mx + atol
    log(f"[gpu]   {name}: max err {err:.3e}  bound {bound:.3e}  max|ref| {mx:.3e}")
    assert np.all(np.isfinite(gpu)), name
    assert err <= bound, name


def gpu_step_backward(plan, scene, model, grad_u, saved=False):
    """etac_step_backward; with saved=True the forward's pooling record is
    taken first (etac_step with a saved buffer) and handed to the adjoint."""
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    ds, dm = DevScene(scene), DevModel(model)
    E, O = ds.E, ds.O
    rec = None
    if saved:
        rec = torch.full((E * plan.K, _native.ETAC_SAVED_WORDS), -1, dtype=torch.int32, device=dev)
        u = torch.empty((3, E, plan.N), device=dev)
        cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
        na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
        _native.etac_step(plan, ds.struct(plan), dm.struct(plan), u, cobj, na, saved=rec)
    gu = to_dev(grad_u.astype(np.float32))
    grot = torch.full((E, O, 9), float("nan"), device=dev)
    gt = torch.full((E, O, 3), float("nan"), device=dev)
    ga = torch.full((plan.K,), float("nan"), device=dev)
    gp = torch.full((17411,), float("nan"), device=dev)
    _native.etac_step_backward(plan, ds.struct(plan), dm.struct(plan), gu, grot, gt, ga, gp, saved=rec)
    torch.cuda.synchronize()
    return dict(grad_rot=grot.cpu().numpy(), grad_trans=gt.cpu().numpy(), grad_alpha=ga.cpu().numpy(),
                grad_phi=gp.cpu().numpy())


def clean_scene(oracle_lib, mesh, scene, model):
    """Scene restricted to envs whose decisions all clear MARGIN."""
    if model.mode == MODE_DECAY_ONLY:
        return scene, scene.n_envs
    out = oracle_lib.forward(mesh, scene, model, with_sig=True)
    keep = out["margin"] > MARGIN
    s = scene.copy()
    s.n_obj[~keep] = 0
    hit = keep & (out["n_active"].sum(axis=1) > 0)
    return s, int(hit.sum())


def _compare_all(g, ref, mode):
    _close(g["grad_trans"], ref["grad_trans"], "grad_trans")
    _close(g["grad_rot"], ref["grad_rot"], "grad_rot")
    if mode != MODE_RESIDUAL_ONLY:
        _close(g["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    else:
        assert np.all(g["grad_alpha"] == 0.0)
    if mode != MODE_DECAY_ONLY:
        _close(g["grad_phi"], ref["grad_phi"], "grad_phi")
    else:
        assert np.all(g["grad_phi"] == 0.0)


@pytest.mark.parametrize("mode", [MODE_DECAY_ONLY, MODE_FULL])
def test_step_backward_pads(oracle_lib, mode):
    # 8 envs of the 32x32 pad (config-3 geometry), loss weights N(0,1)
    mesh, scene, model, w = scenes.config3()
    model = model.with_mode(mode)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    log(f"[gpu] step backward pads mode={mode} envs compared {n_clean}/8")
    assert n_clean >= 1
    plan = make_plan(mesh, 8, 1, backward=True)
    g = gpu_step_backward(plan, sc, model, w)
    _compare_all(g, oracle_lib.backward(mesh, sc, model, w), mode)


@pytest.mark.parametrize("mode", [MODE_DECAY_ONLY, MODE_FULL])
def test_step_backward_hand(oracle_lib, mode):
    mesh, scene, model = scenes.config2(n_envs=48, mode=mode)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    log(f"[gpu] step backward hand mode={mode} envs compared {n_clean}/48")
    assert n_clean >= 8
    w = np.random.default_rng(9).standard_normal((3, 48, mesh.n_nodes))
    plan = make_plan(mesh, 48, 3, backward=True)
    g = gpu_step_backward(plan, sc, model, w)
    _compare_all(g, oracle_lib.backward(mesh, sc, model, w), mode)


@pytest.mark.parametrize("mode", [MODE_FULL, MODE_RESIDUAL_ONLY])
def test_step_backward_small_hand(oracle_lib, mode):
    mesh, scene, model = scenes.config2(n_envs=96, mode=mode, **SMALL)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    log(f"[gpu] step backward small hand mode={mode} envs compared {n_clean}/96")
    assert n_clean >= 20
    w = np.random.default_rng(4).standard_normal((3, 96, mesh.n_nodes))
    plan = make_plan(mesh, 96, 3, backward=True)
    g = gpu_step_backward(plan, sc, model, w)
    _compare_all(g, oracle_lib.backward(mesh, sc, model, w), mode)


def test_propagate_and_contact_backward(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=32, **SMALL)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    log(f"[gpu] propagate/contact backward envs compared {n_clean}/32")
    rc, ru, _ = oracle_lib.contact(mesh, sc)
    ru32 = ru.astype(np.float32)
    w = np.random.default_rng(5).standard_normal((3, 32, mesh.n_nodes))
    plan = make_plan(mesh, 32, 3, backward=True)
    dm = DevModel(model)
    guh = torch.full((3, 32, mesh.n_nodes), float("nan"), device=dev)
    ga = torch.zeros(plan.K, device=dev)
    gp = torch.zeros(17411, device=dev)
    _native.etac_propagate_backward(plan, dm.struct(plan), 32, to_dev(rc), to_dev(ru32), to_dev(w.astype(np.float32)),
                                    guh, ga, gp)
    torch.cuda.synchronize()
    ref = oracle_lib.propagate_backward(mesh, model, rc, ru32.astype(np.float64), w)
    _close(guh.cpu().numpy(), ref["grad_uhat"], "grad_uhat")
    _close(ga.cpu().numpy(), ref["grad_alpha"], "grad_alpha")
    _close(gp.cpu().numpy(), ref["grad_phi"], "grad_phi")
    # contact adjoint from the oracle's dL/du_hat (same FP32 values on both sides)
    g_uh = ref["grad_uhat"].astype(np.float32)
    ds = DevScene(sc)
    grot = torch.full((32, 3, 9), float("nan"), device=dev)
    gt = torch.full((32, 3, 3), float("nan"), device=dev)
    _native.etac_contact_backward(plan, ds.struct(plan), to_dev(g_uh), grot, gt)
    torch.cuda.synchronize()
    refc = oracle_lib.contact_backward(mesh, sc, g_uh.astype(np.float64))
    _close(grot.cpu().numpy(), refc["grad_rot"], "contact grad_rot")
    _close(gt.cpu().numpy(), refc["grad_trans"], "contact grad_trans")


def _fd_vs_gpu(oracle_lib, mesh, sc, model, w, plan, o=0):
    g = gpu_step_backward(plan, sc, model, w)
    fd, ok = oracle_lib.fd_gradients(mesh, sc, model, w, obj=o)
    if not ok:
        return False
    tw = oracle_lib.twist_from_grad_rot(g["grad_rot"][0, o], sc.rot[0, o])
    scale = max(np.abs(fd["trans"]).max(), np.abs(fd["twist"]).max(), 1e-3)
    log(f"[gpu]   fd trans {g['grad_trans'][0, o]} vs {fd['trans']}; twist {tw} vs {fd['twist']}")
    assert np.max(np.abs(g["grad_trans"][0, o] - fd["trans"])) <= 1e-4 * scale + 1e-6
    assert np.max(np.abs(tw - fd["twist"])) <= 1e-4 * scale + 1e-6
    if model.mode != MODE_RESIDUAL_ONLY:
        assert np.max(np.abs(g["grad_alpha"] - fd["alpha"])) <= 1e-4 * np.abs(fd["alpha"]).max() + 1e-6
    return True


def test_step_backward_vs_central_fd_pads(oracle_lib):
    # GPU adjoint against FP64 central differences (h = 1e-4) of the oracle:
    # 6-DoF twist / translation gradients and dL/dalpha, 8 pad envs.
    mesh, scene, model, w = scenes.config3()
    model = model.with_mode(MODE_DECAY_ONLY)
    plan = make_plan(mesh, 1, 1, backward=True)
    checked = 0
    for e in range(8):
        log(f"[gpu] fd pad env {e}")
        checked += _fd_vs_gpu(oracle_lib, mesh, scene.select([e]), model, w[:, e:e + 1], plan)
    assert checked >= 6


def test_step_backward_vs_central_fd_small_hand(oracle_lib):
    mesh, scene, model = scenes.config2(n_envs=64, **SMALL)
    out = oracle_lib.forward(mesh, scene, model, with_sig=True)
    plan = make_plan(mesh, 1, 3, backward=True)
    rng = np.random.default_rng(6)
    checked = 0
    for e in range(64):
        if out["margin"][e] <= MARGIN or out["n_active"][e].sum() == 0 or checked >= 4:
            continue
        o = int(out["contact_obj"][e][out["contact_obj"][e] >= 0][0])
        log(f"[gpu] fd small hand env {e} obj {o}")
        w = rng.standard_normal((3, 1, mesh.n_nodes))
        checked += _fd_vs_gpu(oracle_lib, mesh, scene.select([e]), model, w, plan, o)
    assert checked >= 3


def test_backward_is_deterministic(oracle_lib):
    mesh, scene, model = scenes.config2(n_envs=32)
    w = np.random.default_rng(1).standard_normal((3, 32, mesh.n_nodes))
    plan = make_plan(mesh, 32, 3, backward=True)
    log("[gpu] backward determinism")
    a = gpu_step_backward(plan, scene, model, w)
    b = gpu_step_backward(plan, scene, model, w)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_autograd_function_matches_direct_call(oracle_lib):
    import torch
    from paper_2604_20295_amd.autograd import etac_step, rotation_from_axis_angle
    torch_, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=16)
    plan = make_plan(mesh, 16, 3, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    rot = ds.rot.clone().requires_grad_(True)
    trans = ds.trans.clone().requires_grad_(True)
    alpha = dm.alpha.clone().requires_grad_(True)
    phi = dm.phi.clone().requires_grad_(True)
    w = to_dev(np.random.default_rng(2).standard_normal((3, 16, mesh.n_nodes)).astype(np.float32))
    log("[gpu] autograd ETacStep")
    u, cobj, na = etac_step(plan, ds.n_obj, ds.type, ds.shape, rot, trans, alpha, phi, model.mode)
    (u * w).sum().backward()
    direct = gpu_step_backward(plan, scene, model, w.cpu().numpy())
    for name, t in (("grad_rot", rot), ("grad_trans", trans), ("grad_alpha", alpha), ("grad_phi", phi)):
        assert np.array_equal(t.grad.cpu().numpy(), direct[name]), name
    ref = oracle_lib.forward(mesh, scene, model)
    assert np.array_equal(cobj.cpu().numpy(), ref["contact_obj"])
    # 6-DoF: rotation through a differentiable axis-angle map, chain rule in torch
    w6 = torch.zeros((16, 3, 3), device=dev, dtype=torch.float32, requires_grad=True)
    R0 = ds.rot.reshape(16, 3, 3, 3)
    R = (rotation_from_axis_angle(w6).reshape(16, 3, 3, 3) @ R0).reshape(16, 3, 9).contiguous()
    u2, _, _ = etac_step(plan, ds.n_obj, ds.type, ds.shape, R, ds.trans, dm.alpha, dm.phi, model.mode)
    (u2 * w).sum().backward()
    assert torch.isfinite(w6.grad).all()
    assert float(w6.grad.abs().sum()) > 0.0


def test_hires_pads_backward_full_size_sampled(oracle_lib):
    # decay-only adjoint at full size: pose gradients of sampled envs
    mesh, scene, model = scenes.config4(n_envs=4096, mode=MODE_DECAY_ONLY)
    w = np.random.default_rng(12).standard_normal((3, 4096, mesh.n_nodes)).astype(np.float32)
    plan = make_plan(mesh, 4096, 4, backward=True)
    log("[gpu] hires pads backward E=4096")
    g = gpu_step_backward(plan, scene, model, w)
    envs = np.random.default_rng(2).choice(4096, size=4, replace=False)
    ref = oracle_lib.backward(mesh, scene.select(envs), model, w[:, envs].astype(np.float64))
    _close(g["grad_trans"][envs], ref["grad_trans"], "grad_trans")
    _close(g["grad_rot"][envs], ref["grad_rot"], "grad_rot")


# ---------------------------------------------------------------------------
# the forward's pooling record (ETAC_SAVED_WORDS per (env, patch) item)
# ---------------------------------------------------------------------------

def _pool_f64(mesh, model, cobj, uhat, e, k):
    """Max-pooled encoder features and their arg-max nodes of one item in
    float64 (the independent torch formulation's encoder), plus per channel
    the gap to the runner-up value."""
    import torch
    from tests.torch_ref import unpack_phi
    W = unpack_phi(torch.tensor(model.phi.astype(np.float64)))
    a, b = int(mesh.patch_offset[k]), int(mesh.patch_offset[k + 1])
    P = torch.tensor(mesh.pos[:, a:b].T.astype(np.float64))
    Nn = torch.tensor(mesh.nrm[:, a:b].T.astype(np.float64))
    act = torch.tensor(cobj[e, a:b] >= 0)
    Uh = torch.tensor(np.moveaxis(uhat[:, e, a:b], 0, 1).astype(np.float64))
    Uh = torch.where(act[:, None], Uh, torch.zeros_like(Uh))
    x = torch.cat([P - torch.tensor(mesh.origin[k].astype(np.float64)), Nn, Uh], dim=1)
    f = torch.relu(torch.relu(x @ W["W1"].T + W["b1"]) @ W["W2"].T + W["b2"])
    g = f.amax(dim=0)
    arg = f.argmax(dim=0)              # first maximal node on ties
    top2 = torch.topk(f, min(2, f.shape[0]), dim=0).values
    gap = (top2[0] - top2[-1]) if f.shape[0] > 1 else torch.full_like(g, float("inf"))
    return g.numpy(), arg.numpy(), gap.numpy()


@pytest.mark.parametrize("which", ["pads", "small_hand"])
def test_saved_pool_record_contents(oracle_lib, which):
    # pooled features within FP32 rounding of a float64 evaluation; arg-max
    # nodes equal wherever the runner-up is further than that rounding
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    if which == "pads":
        mesh, scene, model, _ = scenes.config3()
        model = model.with_mode(MODE_FULL)
    else:
        mesh, scene, model = scenes.config2(n_envs=24, mode=MODE_FULL, **SMALL)
    E = scene.n_envs
    plan = make_plan(mesh, E, scene.max_obj, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    rec = torch.full((E * plan.K, _native.ETAC_SAVED_WORDS), -1, dtype=torch.int32, device=dev)
    u = torch.empty((3, E, plan.N), device=dev)
    cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
    na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
    _native.etac_step(plan, ds.struct(plan), dm.struct(plan), u, cobj, na, saved=rec)
    torch.cuda.synchronize()
    rec = rec.cpu().numpy()
    ref = oracle_lib.forward(mesh, scene, model)
    n_items = 0
    for e in range(E):
        for k in range(plan.K):
            item = e * plan.K + k
            if ref["n_active"][e, k] == 0:
                assert np.all(rec[item] == -1), "items without contact are not written"
                continue
            g, arg, gap = _pool_f64(mesh, model, ref["contact_obj"], ref["uhat"], e, k)
            gg = rec[item, :64].view(np.float32).astype(np.float64)
            ga = rec[item, 64:]
            assert np.max(np.abs(gg - g)) <= 1e-5 * max(1.0, np.abs(g).max()), (e, k)
            n = int(mesh.patch_offset[k + 1] - mesh.patch_offset[k])
            assert np.all((ga >= 0) & (ga < n)), (e, k)
            sure = gap > 1e-4
            assert np.array_equal(ga[sure], arg[sure]), (e, k)
            n_items += 1
    log(f"[gpu] pooling records checked: {n_items} items ({which})")
    assert n_items >= 4


@pytest.mark.parametrize("mode", [MODE_FULL, MODE_RESIDUAL_ONLY])
def test_saved_pool_record_gives_identical_gradients(oracle_lib, mode):
    # the adjoint given the forward's record equals the one that recomputes it, bit for bit
    mesh, scene, model = scenes.config2(n_envs=96, mode=mode, **SMALL)
    w = np.random.default_rng(4).standard_normal((3, 96, mesh.n_nodes))
    plan = make_plan(mesh, 96, 3, backward=True)
    log(f"[gpu] saved pooling record vs recompute, small hand mode={mode}")
    g0 = gpu_step_backward(plan, scene, model, w)
    g1 = gpu_step_backward(plan, scene, model, w, saved=True)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k


def test_saved_pool_record_propagate_adjoint(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=32, **SMALL)
    rc, ru, _ = oracle_lib.contact(mesh, scene)
    c, uh = to_dev(rc), to_dev(ru.astype(np.float32))
    gu = to_dev(np.random.default_rng(5).standard_normal((3, 32, mesh.n_nodes)).astype(np.float32))
    plan = make_plan(mesh, 32, 3, backward=True)
    dm = DevModel(model)
    rec = _native.saved_buffer(plan, 32)
    u = torch.empty((3, 32, plan.N), device=dev)
    _native.etac_propagate(plan, dm.struct(plan), 32, c, uh, u, saved=rec)
    out = []
    for r in (None, rec):
        guh = torch.full((3, 32, plan.N), float("nan"), device=dev)
        ga = torch.zeros(plan.K, device=dev)
        gp = torch.zeros(17411, device=dev)
        _native.etac_propagate_backward(plan, dm.struct(plan), 32, c, uh, gu, guh, ga, gp, saved=r)
        torch.cuda.synchronize()
        out.append((guh.cpu().numpy(), ga.cpu().numpy(), gp.cpu().numpy()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_config2_full_size_backward_sampled(oracle_lib):
    # the 4096-env hand, full model, in the launch configuration the benchmark
    # times (forward with the pooling record, then the adjoint given it):
    # gradients identical to the recomputing adjoint, and pose gradients of
    # sampled envs (all decisions clear of the margin) against the oracle
    mesh, scene, model = scenes.config2(n_envs=4096)
    w = np.random.default_rng(21).standard_normal((3, 4096, mesh.n_nodes)).astype(np.float32)
    plan = make_plan(mesh, 4096, scene.max_obj, backward=True)
    log("[gpu] hand backward E=4096 (saved record vs recompute)")
    g1 = gpu_step_backward(plan, scene, model, w, saved=True)
    g0 = gpu_step_backward(plan, scene, model, w)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k
    rng = np.random.default_rng(3)
    envs = []
    for e in rng.permutation(4096):
        sub = scene.select([int(e)])
        out = oracle_lib.forward(mesh, sub, model, with_sig=True)
        if out["margin"][0] > MARGIN and out["n_active"].sum() > 0:
            envs.append(int(e))
        if len(envs) == 6:
            break
    log(f"[gpu]   sampled envs {envs}")
    assert len(envs) == 6
    envs = np.array(envs)
    ref = oracle_lib.backward(mesh, scene.select(envs), model, w[:, envs].astype(np.float64))
    _close(g1["grad_trans"][envs], ref["grad_trans"], "grad_trans")
    _close(g1["grad_rot"][envs], ref["grad_rot"], "grad_rot")
