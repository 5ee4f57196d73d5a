"""The step captured in a HIP graph (torch.cuda.CUDAGraph over the C-ABI
calls) replays bit-identically to eager calls, also across several replays
with eager work in between and after the captured pose buffers are updated
in place (the rollout pattern: new poses, same graph); likewise the
mesh-object calls and their adjoints."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import DevModel, DevScene, log, make_plan, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=64)
    E, O, N, K = 64, 3, mesh.n_nodes, mesh.n_patches
    plan = make_plan(mesh, E, O, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    gu = to_dev(np.random.default_rng(3).standard_normal((3, E, N)).astype(np.float32))
    outs = dict(u=torch.empty((3, E, N), device=dev), cobj=torch.empty((E, N), dtype=torch.int8, device=dev),
                na=torch.empty((E, K), dtype=torch.int32, device=dev), grot=torch.empty((E, O, 9), device=dev),
                gt=torch.empty((E, O, 3), device=dev), ga=torch.empty((K,), device=dev),
                gp=torch.empty((17411,), device=dev))

    def step():
        _native.etac_step(plan, sc, md, outs["u"], outs["cobj"], outs["na"])
        _native.etac_step_backward(plan, sc, md, gu, outs["grot"], outs["gt"], outs["ga"], outs["gp"])

    def snap():
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().copy() for k, v in outs.items()}

    log("[gpu] graph capture")
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
        for v in outs.values():
            v.zero_()
        g.replay()
        got = snap()
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)
        _ = (torch.randn(1000, device=dev) * 2).sum().item()   # eager work between replays
    # new poses in the captured buffers: replay equals a fresh eager step
    traj_rot, traj_trans = scenes.trajectory(scene, 3, seed=9)
    for t in (1, 2):
        ds.rot.copy_(to_dev(traj_rot[t]))
        ds.trans.copy_(to_dev(traj_trans[t]))
        g.replay()
        got = snap()
        step()
        ref = snap()
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (t, k)
        s2 = scene.copy()
        s2.rot, s2.trans = traj_rot[t], traj_trans[t]
        assert np.array_equal(got["cobj"], oracle_lib.contact(mesh, s2)[0])


def test_kernel_timer_counts_eager_launches_only(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=32)
    plan = make_plan(mesh, 32, 3, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    E, N, K = 32, mesh.n_nodes, mesh.n_patches
    u = torch.empty((3, E, N), device=dev)
    cobj = torch.empty((E, N), dtype=torch.int8, device=dev)
    na = torch.empty((E, K), dtype=torch.int32, device=dev)
    log("[gpu] kernel timer")
    assert plan.kernel_time(_native.ETAC_TIMER_STEP) == (0, 0.0)     # never turned on
    plan.set_timing(True)
    for _ in range(5):
        _native.etac_step(plan, sc, md, u, cobj, na)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        _native.etac_step(plan, sc, md, u, cobj, na)          # 6th eager launch (side stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        _native.etac_step(plan, sc, md, u, cobj, na)          # captured: not timed
    g.replay()
    n, ms = plan.kernel_time(_native.ETAC_TIMER_STEP)
    assert n == 6 and 0.0 < ms < 1e4
    assert plan.kernel_time(_native.ETAC_TIMER_STEP) == (0, 0.0)    # reading resets
    assert plan.kernel_time(_native.ETAC_TIMER_BACKWARD) == (0, 0.0)
    plan.set_timing(False)
    _native.etac_step(plan, sc, md, u, cobj, na)
    assert plan.kernel_time(_native.ETAC_TIMER_STEP) == (0, 0.0)
    ref = oracle_lib.forward(mesh, scene, model)
    torch.cuda.synchronize()
    assert np.array_equal(cobj.cpu().numpy(), ref["contact_obj"])


def test_autotune_picks_a_candidate_and_keeps_results(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=64)
    E, O, N, K = 64, 3, mesh.n_nodes, mesh.n_patches
    plan = make_plan(mesh, E, O, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    gu = to_dev(np.random.default_rng(4).standard_normal((3, E, N)).astype(np.float32))
    outs = dict(u=torch.empty((3, E, N), device=dev), cobj=torch.empty((E, N), dtype=torch.int8, device=dev),
                na=torch.empty((E, K), dtype=torch.int32, device=dev), grot=torch.empty((E, O, 9), device=dev),
                gt=torch.empty((E, O, 3), device=dev), ga=torch.empty((K,), device=dev),
                gp=torch.empty((17411,), device=dev))

    def step():
        _native.etac_step(plan, sc, md, outs["u"], outs["cobj"], outs["na"])
        _native.etac_step_backward(plan, sc, md, gu, outs["grot"], outs["gt"], outs["ga"], outs["gp"])
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().copy() for k, v in outs.items()}

    log("[gpu] autotune")
    assert plan.launch() == (2, 4, 4, 3, 2)                  # built-in defaults
    ref = step()
    best = _native.etac_plan_autotune(plan, sc, md, outs["u"], outs["cobj"], outs["na"], gu, outs["grot"],
                                      outs["gt"], outs["ga"], outs["gp"], reps=2)
    log(f"[gpu]   chosen launch shape {best}")
    assert best == plan.launch()
    assert best[0] in (1, 2) and best[1] in (1, 2, 4, 8, 16) and best[2] in (2, 4, 8, 16) and best[3] in (2, 3, 4)
    assert best[4] in (1, 2, 4)
    got = step()
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(got["cobj"], oracle_lib.contact(mesh, scene)[0])


def test_mesh_calls_graph_replay_matches_eager(oracle_lib):
    # mesh contact (with its records), propagation and both adjoints captured
    # in one graph: every replay equals the eager results, with eager work in
    # between
    from paper_2604_20295_amd import _native
    from scenes import trimeshes as tm
    from tests.test_gpu_backward import SMALL
    torch, dev = torch_dev()
    mesh = scenes.hand_mesh(0, sizes=SMALL["sizes"])
    ms = tm.object_set(scale=SMALL["scale"])
    scene = tm.hand_mesh_scene(mesh, ms, 32, seed=4, p_mesh=0.7, scale=SMALL["scale"])
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, scenes.MODE_FULL)
    E, O, N, K = 32, 3, mesh.n_nodes, mesh.n_patches
    plan = make_plan(mesh, E, O, backward=True)
    dms = _native.MeshSet.from_set(ms)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    gu = to_dev(np.random.default_rng(8).standard_normal((3, E, N)).astype(np.float32))
    saved = _native.saved_buffer(plan, E)
    outs = dict(cobj=torch.empty((E, N), dtype=torch.int8, device=dev), uhat=torch.empty((3, E, N), device=dev),
                na=torch.empty((E, K), dtype=torch.int32, device=dev),
                hit=torch.empty((E, N), dtype=torch.int32, device=dev), u=torch.empty((3, E, N), device=dev),
                guhat=torch.empty((3, E, N), device=dev), ga=torch.empty((K,), device=dev),
                gp=torch.empty((17411,), device=dev), grot=torch.empty((E, O, 9), device=dev),
                gt=torch.empty((E, O, 3), device=dev))

    def step():
        _native.etac_contact_mesh(plan, dms, sc, outs["cobj"], outs["uhat"], outs["na"], outs["hit"])
        _native.etac_propagate(plan, md, E, outs["cobj"], outs["uhat"], outs["u"], saved=saved)
        _native.etac_propagate_backward(plan, md, E, outs["cobj"], outs["uhat"], gu, outs["guhat"], outs["ga"],
                                        outs["gp"], saved=saved)
        _native.etac_contact_mesh_backward(plan, dms, sc, outs["guhat"], outs["grot"], outs["gt"], outs["cobj"],
                                           outs["hit"])

    def snap():
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().copy() for k, v in outs.items()}

    log("[gpu] graph capture of the mesh-object calls")
    step()
    eager = snap()
    assert (eager["hit"] >= 0).sum() > 100
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
        for v in outs.values():
            v.zero_()
        g.replay()
        got = snap()
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)
        _ = (torch.randn(1000, device=dev) * 2).sum().item()
