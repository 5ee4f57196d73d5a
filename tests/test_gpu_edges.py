"""Edge cases at the limits of the C ABI against the FP64 oracle: eight
objects per env (ETAC_MAX_OBJ), one patch of the largest allowed node count
(ETAC_MAX_PATCH_NODES), and calls with zero envs."""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL, MODE_DECAY_ONLY, SPHERE, BOX
from tests.gpu_util import DevModel, DevScene, gpu_step, log, make_plan, max_err, to_dev, torch_dev
from tests.test_gpu_backward import SMALL, _compare_all, clean_scene, gpu_step_backward

pytestmark = pytest.mark.gpu


def _eight_object_scene(mesh, E, seed):
    """Every env holds eight small primitives placed like the hand's."""
    scene = scenes._empty_scene(E, 8)
    for e in range(E):
        rng = np.random.default_rng([seed, e])
        scene.n_obj[e] = 8
        for o in range(8):
            ptype, shape, R = scenes.draw_primitive(rng, 0.2)
            t = scenes.place_primitive(rng, mesh, ptype, shape, R, (0.4, 2.0))
            scene.type[e, o] = ptype
            scene.shape[e, o] = shape
            scene.rot[e, o] = R.ravel()
            scene.trans[e, o] = t
    return scene


def test_eight_objects_per_env(oracle_lib):
    mesh = scenes.hand_mesh(0, sizes=SMALL["sizes"])
    scene = _eight_object_scene(mesh, 16, 11)
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_FULL)
    plan = make_plan(mesh, 16, 8, backward=True)
    u, cobj, na = gpu_step(plan, scene, model)
    ref = oracle_lib.forward(mesh, scene, model)
    log(f"[gpu] eight objects per env: objects winning somewhere {np.unique(cobj[cobj >= 0]).tolist()}, "
        f"max|dU| {max_err(u, ref['u']):.2e}")
    assert np.array_equal(cobj, ref["contact_obj"])
    assert np.array_equal(na, ref["n_active"])
    assert max_err(u, ref["u"]) <= 1e-5
    assert len(np.unique(cobj[cobj >= 0])) >= 6
    # adjoint: decay-only on every env, full model on the envs clear of the margin
    w = np.random.default_rng(3).standard_normal((3, 16, mesh.n_nodes))
    m2 = model.with_mode(MODE_DECAY_ONLY)
    _compare_all(gpu_step_backward(plan, scene, m2, w), oracle_lib.backward(mesh, scene, m2, w), MODE_DECAY_ONLY)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    log(f"[gpu]   full-model adjoint envs compared {n_clean}/16")
    assert n_clean >= 2
    _compare_all(gpu_step_backward(plan, sc, model, w, saved=True), oracle_lib.backward(mesh, sc, model, w),
                 MODE_FULL)


def _largest_patch_mesh():
    pos, nrm = scenes._grid_patch(256, 256, 0.125, (0.0, 0.0, 0.0))
    return scenes._assemble_mesh([(pos, nrm)], [0.125], [(0.0, 0.0, 0.0)], [(256, 256, 0.0)])


def test_largest_patch(oracle_lib):
    mesh = _largest_patch_mesh()
    assert mesh.n_nodes == 65536
    scene = scenes._empty_scene(2, 1)
    rng = np.random.default_rng(21)
    # env 0: a sphere pressed 1 mm; env 1: a rotated box pressed 2 mm
    scene.n_obj[:] = 1
    scene.type[0, 0] = SPHERE
    scene.shape[0, 0, 0] = 5.0
    scene.trans[0, 0] = (1.3, -2.1, 5.0 - 1.0)
    R = scenes.random_rotation(rng)
    half = np.array([4.0, 3.0, 2.0])
    scene.type[1, 0] = BOX
    scene.shape[1, 0, :3] = half
    scene.rot[1, 0] = R.ravel()
    n = np.array([0.0, 0.0, 1.0])
    scene.trans[1, 0] = (-3.0, 2.5, 0.0) + (scenes.support_extent(BOX, half, R, n) - 2.0) * n
    model = scenes.draw_model(np.random.default_rng([4, 1]), mesh.pitch, MODE_FULL)
    plan = make_plan(mesh, 2, 1, backward=True)
    u, cobj, na = gpu_step(plan, scene, model)
    ref = oracle_lib.forward(mesh, scene, model)
    log(f"[gpu] largest patch (65536 nodes): active {na.ravel().tolist()}, max|dU| {max_err(u, ref['u']):.2e}")
    assert np.array_equal(cobj, ref["contact_obj"])
    assert np.array_equal(na, ref["n_active"])
    assert na.max() > 1024 and na.min() > 500   # active sets spanning one and several LDS chunks
    assert max_err(u, ref["u"]) <= 1e-5
    w = np.random.default_rng(8).standard_normal((3, 2, mesh.n_nodes))
    m2 = model.with_mode(MODE_DECAY_ONLY)
    _compare_all(gpu_step_backward(plan, scene, m2, w), oracle_lib.backward(mesh, scene, m2, w), MODE_DECAY_ONLY)


def test_zero_envs(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model = scenes.config2(n_envs=4, **SMALL)
    plan = make_plan(mesh, 4, 3, backward=True)
    empty = scene.select(np.zeros(0, dtype=np.int64))
    ds, dm = DevScene(empty), DevModel(model)
    N, K = plan.N, plan.K
    u = torch.empty((3, 0, N), device=dev)
    cobj = torch.empty((0, N), dtype=torch.int8, device=dev)
    na = torch.empty((0, K), dtype=torch.int32, device=dev)
    _native.etac_step(plan, ds.struct(plan), dm.struct(plan), u, cobj, na)
    _native.etac_contact(plan, ds.struct(plan), cobj, torch.empty((3, 0, N), device=dev), na)
    _native.etac_propagate(plan, dm.struct(plan), 0, cobj, u, torch.empty((3, 0, N), device=dev))
    ga = torch.full((K,), 7.0, device=dev)
    gp = torch.full((17411,), 7.0, device=dev)
    _native.etac_step_backward(plan, ds.struct(plan), dm.struct(plan), u, torch.empty((0, 3, 9), device=dev),
                               torch.empty((0, 3, 3), device=dev), ga, gp)
    torch.cuda.synchronize()
    # sums over no env: the parameter gradients are zero
    assert float(ga.abs().max()) == 0.0 and float(gp.abs().max()) == 0.0
