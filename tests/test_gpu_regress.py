"""GPU parity of the real-sensor regressor (attention-pooled PointNet with a
residual layer, appendix "Modeling Real Sensors") against the FP64 oracle.

Bar: every taxel output within TOL_REG * max(1, max |y|) of the oracle.
E3 and A1 run on FP16 operands (relative rounding 2^-11 at most) with FP32
accumulation, the pooled features are those FP16 operands, and everything
else is FP32-level; a CPU emulation of exactly these roundings on the
16-patch hand lands at 1.1e-4 of max |y|, so 1e-3 leaves a factor of 9.
Inputs are the oracle's own step outputs or seeded synthetic fields, never
values computed by the GPU.
"""
import numpy as np
import pytest

import oracle
import scenes
from scenes import articulated as art
from tests.gpu_util import log, make_plan, max_err, to_dev, torch_dev

pytestmark = pytest.mark.gpu

TOL_REG = 1e-3


def _ragged_mesh(sizes, seed=0, extent=6.0):
    """Patches of the given node counts, random positions within +-extent mm
    of a per-patch origin."""
    rng = np.random.default_rng([seed, 17])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    N, K = int(off[-1]), len(sizes)
    origin = rng.uniform(-30.0, 30.0, size=(K, 3)).astype(np.float32)
    pos = np.empty((3, N), np.float32)
    for k in range(K):
        pos[:, off[k]:off[k + 1]] = origin[k][:, None] + rng.uniform(-extent, extent, size=(3, sizes[k]))
    nrm = np.zeros((3, N), np.float32)
    nrm[2] = 1.0
    return scenes.Mesh(off, pos, nrm, origin, np.ones(K), [])


def _synthetic_field(mesh, E, frac, seed):
    """u [3][E][N] nonzero on a random fraction of the (env, patch) items
    (smooth bumps of a few mm), zero elsewhere; n_active > 0 exactly there."""
    rng = np.random.default_rng([seed, 23])
    K, N = mesh.n_patches, mesh.n_nodes
    off = mesh.patch_offset
    u = np.zeros((3, E, N), np.float32)
    na = np.zeros((E, K), np.int32)
    live = rng.random((E, K)) < frac
    for e, k in zip(*np.nonzero(live)):
        sl = slice(off[k], off[k + 1])
        p = mesh.pos[:, sl].astype(np.float64)
        c = p[:, rng.integers(p.shape[1])]
        d2 = ((p - c[:, None]) ** 2).sum(0)
        amp = rng.uniform(-3.0, 3.0, size=3)
        u[:, e, sl] = (amp[:, None] * np.exp(-d2 / rng.uniform(2.0, 20.0))).astype(np.float32)
        na[e, k] = 1 + int(rng.integers(sl.stop - sl.start))
    return u, na


def _gpu_regress(plan, reg, u, na):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    E = u.shape[1]
    out = torch.full((E, plan.K, 8), float("nan"), device=dev)
    _native.etac_regress(plan, to_dev(reg), to_dev(u), to_dev(na), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(y_gpu, y_ref, what):
    tol = TOL_REG * max(1.0, float(np.abs(y_ref).max()))
    err = max_err(y_gpu, y_ref)
    log(f"{what}: max|y| {np.abs(y_ref).max():.3f}, max err {err:.2e} (bar {tol:.1e})")
    assert np.isfinite(y_gpu).all()
    assert err <= tol, what


def _reg(seed=21):
    return scenes.draw_regressor(np.random.default_rng(seed))


def test_regress_hand_step_outputs():
    """16-patch hand (64 .. 1024 nodes per patch), u and n_active from the
    oracle's own step."""
    mesh, scene, model = scenes.config2(n_envs=12, env_seed=1)
    out = oracle.forward(mesh, scene, model)
    u = out["u"].astype(np.float32)
    na = out["n_active"]
    assert (na > 0).any() and (na == 0).any()
    reg = _reg()
    plan = make_plan(mesh, 12, 3)
    y = _gpu_regress(plan, reg, u, na)
    _check(y, oracle.regress(mesh, reg.astype(np.float64), u.astype(np.float64)), "hand, oracle step")


def test_regress_ragged_patches_and_tails():
    """Patch sizes that leave ragged 16-node tiles, patches of one node and
    patches larger than the eight waves' first pass (more than 128 nodes)."""
    sizes = [1, 5, 16, 17, 127, 129, 300, 1000, 2]
    mesh = _ragged_mesh(sizes, seed=3)
    E = 7
    u, na = _synthetic_field(mesh, E, 0.6, seed=4)
    reg = _reg(5)
    plan = make_plan(mesh, E, 1)
    y = _gpu_regress(plan, reg, u, na)
    _check(y, oracle.regress(mesh, reg.astype(np.float64), u.astype(np.float64)), "ragged")
    # fewer envs than the plan holds
    y3 = _gpu_regress(plan, reg, np.ascontiguousarray(u[:, :3]), np.ascontiguousarray(na[:3]))
    assert np.array_equal(y3, y[:3])


def test_regress_articulated_hand_link_frames():
    """The articulated hand's step output (link frames, self-contact)."""
    h, mesh, scene, links, model = art.config_hand(n_envs=6, seed=11)
    out = oracle.hand_forward(mesh, h, scene, links, model)
    u = out["u"].astype(np.float32)
    na = out["n_active"]
    assert (na > 0).any()
    reg = _reg(8)
    plan = make_plan(mesh, 6, scene.max_obj)
    y = _gpu_regress(plan, reg, u, na)
    _check(y, oracle.regress(mesh, reg.astype(np.float64), u.astype(np.float64)), "articulated hand")


def test_regress_no_contact_and_empty():
    """All items without contact take the rest output of their patch; an
    empty batch is accepted and enqueues nothing."""
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh = _ragged_mesh([33, 64, 7], seed=9)
    E = 5
    u = np.zeros((3, E, mesh.n_nodes), np.float32)
    na = np.zeros((E, 3), np.int32)
    reg = _reg(10)
    plan = make_plan(mesh, E, 1)
    y = _gpu_regress(plan, reg, u, na)
    ref = oracle.regress(mesh, reg.astype(np.float64), u.astype(np.float64))
    _check(y, ref, "no contact")
    for e in range(1, E):
        assert np.array_equal(y[e], y[0])
    empty = torch.full((0, 3, 8), 7.0, device=dev)
    _native.etac_regress(plan, to_dev(reg), torch.zeros((3, 0, mesh.n_nodes), device=dev),
                         torch.zeros((0, 3), dtype=torch.int32, device=dev), empty)
    torch.cuda.synchronize()


def test_regress_largest_patch():
    """One patch of the largest size the plan accepts (65536 nodes, 4096
    tiles over eight waves)."""
    mesh = _ragged_mesh([65536], seed=12, extent=20.0)
    E = 2
    u, na = _synthetic_field(mesh, E, 1.0, seed=13)
    reg = _reg(14)
    plan = make_plan(mesh, E, 1)
    y = _gpu_regress(plan, reg, u, na)
    _check(y, oracle.regress(mesh, reg.astype(np.float64), u.astype(np.float64)), "65536-node patch")


def test_regress_full_size_sampled():
    """The benchmark's shape (16-patch hand, 4096 envs, about 3% of items in
    contact) in one launch; a sample of items checked against the oracle,
    items without contact against the patch's rest output, and a second call
    bit-identical (fixed reduction order)."""
    mesh, _, _ = scenes.config2(n_envs=1, env_seed=1)
    E = 4096
    u, na = _synthetic_field(mesh, E, 0.03, seed=15)
    reg = _reg(16)
    plan = make_plan(mesh, E, 3)
    y = _gpu_regress(plan, reg, u, na)
    y2 = _gpu_regress(plan, reg, u, na)
    assert np.array_equal(y, y2)
    rng = np.random.default_rng(17)
    live = np.unique(np.nonzero(na)[0])
    envs = np.unique(np.concatenate([rng.choice(live, 24, replace=False), rng.choice(E, 8, replace=False)]))
    ref = oracle.regress(mesh, reg.astype(np.float64), np.ascontiguousarray(u[:, envs]).astype(np.float64))
    _check(y[envs], ref, f"4096 envs, {len(envs)} sampled envs")
    rest = oracle.regress(mesh, reg.astype(np.float64), np.zeros((3, 1, mesh.n_nodes)))[0]
    dead = na == 0
    tol = TOL_REG * max(1.0, float(np.abs(rest).max()))
    assert max_err(y[dead], np.broadcast_to(rest, y.shape)[dead]) <= tol


def test_regress_validation():
    from paper_2604_20295_amd import _native
    lib = _native.lib()
    torch, dev = torch_dev()
    mesh = _ragged_mesh([20, 40], seed=18)
    plan = make_plan(mesh, 3, 1)
    reg = to_dev(_reg())
    u = torch.zeros((3, 4, mesh.n_nodes), device=dev)
    na = torch.zeros((4, 2), dtype=torch.int32, device=dev)
    y = torch.zeros((4, 2, 8), device=dev)
    p = _native._ptr
    assert lib.etac_regress(plan.handle, p(reg), 4, p(u), p(na), p(y), None) == -2   # more envs than the plan
    assert lib.etac_regress(plan.handle, p(reg), -1, p(u), p(na), p(y), None) == -2
    assert lib.etac_regress(plan.handle, None, 2, p(u), p(na), p(y), None) == -1
    assert lib.etac_regress(plan.handle, p(reg), 2, p(u), p(na), None, None) == -1
    assert lib.etac_regress(None, p(reg), 2, p(u), p(na), p(y), None) == -1
    assert lib.etac_regress(plan.handle, None, 0, None, None, None, None) == 0


def test_regress_graph_replay():
    """The step and the regressor captured in one HIP graph replay
    bit-identically to eager calls, with eager work between the replays and
    after new poses are written into the captured buffers."""
    from paper_2604_20295_amd import _native
    from tests.gpu_util import DevModel, DevScene
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=32, env_seed=3)
    E, O, N, K = 32, 3, mesh.n_nodes, mesh.n_patches
    plan = make_plan(mesh, E, O)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    reg = to_dev(_reg(19))
    u = torch.empty((3, E, N), device=dev)
    cobj = torch.empty((E, N), dtype=torch.int8, device=dev)
    na = torch.empty((E, K), dtype=torch.int32, device=dev)
    y = torch.empty((E, K, 8), device=dev)

    def step():
        _native.etac_step(plan, sc, md, u, cobj, na)
        _native.etac_regress(plan, reg, u, na, y)

    def snap():
        torch.cuda.synchronize()
        return y.cpu().numpy().copy()

    step()
    eager = snap()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        y.zero_()
        g.replay()
        assert np.array_equal(snap(), eager), rep
        _ = (torch.randn(1000, device=dev) * 2).sum().item()   # eager work between replays
    traj_rot, traj_trans = scenes.trajectory(scene, 2, seed=4)
    ds.rot.copy_(to_dev(traj_rot[1]))
    ds.trans.copy_(to_dev(traj_trans[1]))
    g.replay()
    got = snap()
    step()
    assert np.array_equal(got, snap())
    # and the replayed taxels against the oracle on the oracle's own step at the new poses
    s2 = scene.copy()
    s2.rot, s2.trans = traj_rot[1], traj_trans[1]
    ref = oracle.forward(mesh, s2, model)
    yr = oracle.regress(mesh, _reg(19).astype(np.float64), ref["u"].astype(np.float32).astype(np.float64))
    _check(got, yr, "graph replay at new poses")
