"""GPU parity of the forward path (etac_contact, etac_propagate, etac_step)
against the FP64 oracle: contact_obj and n_active bit-exact, displacements
within 1e-5 mm (max abs)."""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY, SPHERE, BOX, CAPSULE
from tests.gpu_util import (TOL_U, gpu_contact, gpu_propagate, gpu_step, log, make_plan, max_err)

pytestmark = pytest.mark.gpu

MODES = [MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY]


def _check_step(oracle_lib, mesh, scene, model, plan=None, label=""):
    log(f"[gpu] step parity {label} E={scene.n_envs} N={mesh.n_nodes} mode={model.mode}")
    plan = plan or make_plan(mesh, scene.n_envs, scene.max_obj)
    u, cobj, na = gpu_step(plan, scene, model)
    ref = oracle_lib.forward(mesh, scene, model)
    assert np.array_equal(cobj, ref["contact_obj"]), "contact_obj differs"
    assert np.array_equal(na, ref["n_active"]), "n_active differs"
    err = max_err(u, ref["u"])
    log(f"[gpu]   max|dU| = {err:.3e} mm, active {int(na.sum())}")
    assert err <= TOL_U
    return u, cobj, na, ref


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_contact_config1(oracle_lib, seed):
    mesh, scene, _ = scenes.config1(seed)
    log(f"[gpu] contact config1 seed={seed}")
    plan = make_plan(mesh, 1, 1)
    cobj, uhat, na = gpu_contact(plan, scene)
    rc, ru, rn = oracle_lib.contact(mesh, scene)
    assert np.array_equal(cobj, rc)
    assert np.array_equal(na, rn)
    assert max_err(uhat, ru) <= 1e-6


def test_contact_config2_all_primitives(oracle_lib):
    mesh, scene, _ = scenes.config2(n_envs=256)
    log("[gpu] contact config2 E=256")
    plan = make_plan(mesh, 256, 3)
    cobj, uhat, na = gpu_contact(plan, scene)
    rc, ru, rn = oracle_lib.contact(mesh, scene)
    assert np.array_equal(cobj, rc)
    assert np.array_equal(na, rn)
    assert max_err(uhat, ru) <= 2e-6
    # every primitive type is exercised
    for ty in (SPHERE, BOX, CAPSULE):
        hit = [(e, o) for e in range(256) for o in range(scene.n_obj[e])
               if scene.type[e, o] == ty and np.any(rc[e] == o)]
        assert len(hit) > 5


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", [0, 5])
def test_step_config1(oracle_lib, mode, seed):
    mesh, scene, model = scenes.config1(seed, mode=mode)
    _check_step(oracle_lib, mesh, scene, model, label=f"config1 seed={seed}")


@pytest.mark.parametrize("mode", MODES)
def test_step_config2_small(oracle_lib, mode):
    mesh, scene, model = scenes.config2(n_envs=48, mode=mode)
    _check_step(oracle_lib, mesh, scene, model, label="config2 E=48")


def test_step_centred_mirror_symmetric_mask(oracle_lib):
    mesh, scene, model = scenes.config1(4, centred=True, mode=MODE_DECAY_ONLY)
    u, cobj, na, ref = _check_step(oracle_lib, mesh, scene, model, label="centred")
    m = (cobj[0] >= 0).reshape(32, 32)
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1]) and np.array_equal(m, m.T)


def test_no_contact_gives_exact_zeros(oracle_lib):
    mesh, scene, model = scenes.config1(0)
    scene.trans[0, 0, 2] = 5.5
    plan = make_plan(mesh, 1, 1)
    log("[gpu] no-contact zeros")
    for mode in MODES:
        u, cobj, na = gpu_step(plan, scene, model, mode)
        assert np.all(u == 0.0) and np.all(cobj == -1) and np.all(na == 0)


def test_fused_step_equals_contact_then_propagate(oracle_lib):
    mesh, scene, model = scenes.config2(n_envs=32)
    plan = make_plan(mesh, 32, 3)
    log("[gpu] fused vs unfused")
    u, cobj, na = gpu_step(plan, scene, model)
    c2, uh2, na2 = gpu_contact(plan, scene)
    assert np.array_equal(cobj, c2) and np.array_equal(na, na2)
    u2 = gpu_propagate(plan, model, c2, uh2)
    assert np.array_equal(u, u2)


@pytest.mark.parametrize("mode", MODES)
def test_propagate_given_contact(oracle_lib, mode):
    # Same FP32 inputs on both sides: oracle contact rounded to FP32.
    mesh, scene, model = scenes.config2(n_envs=16, mode=mode)
    rc, ru, _ = oracle_lib.contact(mesh, scene)
    ru32 = ru.astype(np.float32)
    plan = make_plan(mesh, 16, 3)
    log(f"[gpu] propagate given contact mode={mode}")
    u = gpu_propagate(plan, model, rc, ru32)
    ref = oracle_lib.propagate(mesh, model, rc, ru32.astype(np.float64))
    assert max_err(u, ref) <= TOL_U


def _ragged_mesh():
    # patch sizes that are not multiples of the 16-node MFMA tile or the
    # 256-thread workgroup, including a single-node patch
    sizes = [1, 17, 300, 1000, 255, 64]
    pos, nrm, offs, cen = [], [], [0], []
    for k, n in enumerate(sizes):
        nx = int(np.ceil(np.sqrt(n)))
        i = np.arange(n)
        x = (i % nx - (nx - 1) / 2.0) * 0.7 + 40.0 * k
        y = (i // nx - (nx - 1) / 2.0) * 0.7
        pos.append(np.stack([x, y, np.zeros(n)]))
        nrm.append(np.stack([np.zeros(n), np.zeros(n), np.ones(n)]))
        offs.append(offs[-1] + n)
        cen.append((40.0 * k, 0.0, 0.0))
    return scenes.Mesh(np.array(offs, np.int32), np.concatenate(pos, 1).astype(np.float32),
                       np.concatenate(nrm, 1).astype(np.float32), np.array(cen, np.float32),
                       np.full(len(sizes), 0.7), [])


@pytest.mark.parametrize("mode", MODES)
def test_step_ragged_patches(oracle_lib, mode):
    mesh = _ragged_mesh()
    E = 6
    scene = scenes._empty_scene(E, 2)
    rng = np.random.default_rng(42)
    for e in range(E):
        scene.n_obj[e] = 2
        for o in range(2):
            k = (e + o) % mesh.n_patches
            c = mesh.origin[k].astype(np.float64)
            r = rng.uniform(3.0, 9.0)
            scene.type[e, o] = SPHERE
            scene.shape[e, o, 0] = r
            scene.trans[e, o] = c + np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), r - rng.uniform(0.5, 3.0)])
    model = scenes.draw_model(np.random.default_rng(3), mesh.pitch, mode)
    _check_step(oracle_lib, mesh, scene, model, label="ragged")


def test_step_more_actives_than_one_lds_chunk(oracle_lib):
    # one 128 x 128 pad at 0.125 mm pitch, a large flat box pressed in: the
    # active set exceeds one staged chunk of the decay loop
    pos, nrm = scenes._grid_patch(128, 128, 0.125, (0.0, 0.0, 0.0))
    mesh = scenes._assemble_mesh([(pos, nrm)], [0.125], [(0.0, 0.0, 0.0)], [(128, 128, 0.0)])
    scene = scenes._empty_scene(2, 1)
    for e, depth in enumerate((0.3, 0.05)):
        scene.n_obj[e] = 1
        scene.type[e, 0] = BOX
        scene.shape[e, 0, :3] = (3.0, 2.5, 1.0)
        scene.trans[e, 0] = (0.2 * e, -0.1, 1.0 - depth)
    model = scenes.draw_model(np.random.default_rng(8), mesh.pitch, MODE_FULL)
    u, cobj, na, ref = _check_step(oracle_lib, mesh, scene, model, label="big active set")
    assert na[0, 0] > 1536


def test_fewer_envs_than_plan_and_repeatability(oracle_lib):
    mesh, scene, model = scenes.config2(n_envs=40)
    plan = make_plan(mesh, 64, 3)
    log("[gpu] E < plan E, repeat")
    u1, c1, n1 = gpu_step(plan, scene, model)
    u2, c2, n2 = gpu_step(plan, scene, model)
    assert np.array_equal(u1, u2) and np.array_equal(c1, c2) and np.array_equal(n1, n2)
    ref = oracle_lib.forward(mesh, scene, model)
    assert np.array_equal(c1, ref["contact_obj"])
    assert max_err(u1, ref["u"]) <= TOL_U


def test_config2_full_size_sampled(oracle_lib):
    # 4096 envs in the launch configuration the benchmark times: contact of
    # every env against the oracle, displacements of 24 sampled envs.
    mesh, scene, model = scenes.config2(n_envs=4096)
    plan = make_plan(mesh, 4096, 3)
    log("[gpu] config2 E=4096 full size")
    u, cobj, na = gpu_step(plan, scene, model)
    rc, _, rn = oracle_lib.contact(mesh, scene)
    assert np.array_equal(cobj, rc)
    assert np.array_equal(na, rn)
    envs = np.random.default_rng(0).choice(4096, size=24, replace=False)
    ref = oracle_lib.forward(mesh, scene.select(envs), model)
    err = max_err(u[:, envs], ref["u"])
    log(f"[gpu]   sampled max|dU| = {err:.3e}")
    assert err <= TOL_U


def test_hires_pads_full_size_sampled(oracle_lib):
    # 4096 envs x 4 pads of 128 x 128 nodes at 0.125 mm pitch (65536 nodes per
    # env, 2.7e8 per step), one sphere or box per pad: contact of 8 sampled envs
    # and their displacements against the oracle.  Active sets reach several
    # thousand nodes, so the decay loop streams several LDS chunks.
    mesh, scene, model = scenes.config4(n_envs=4096)
    plan = make_plan(mesh, 4096, 4)
    log("[gpu] hires pads E=4096 full size")
    u, cobj, na = gpu_step(plan, scene, model)
    envs = np.random.default_rng(1).choice(4096, size=8, replace=False)
    ref = oracle_lib.forward(mesh, scene.select(envs), model)
    assert np.array_equal(cobj[envs], ref["contact_obj"])
    assert np.array_equal(na[envs], ref["n_active"])
    assert na[envs].max() > 1536
    err = max_err(u[:, envs], ref["u"])
    log(f"[gpu]   sampled max|dU| = {err:.3e}")
    assert err <= TOL_U


def test_contact_pass_ragged_node_count(oracle_lib):
    # N not a multiple of 4: the contact kernel's scalar store path
    mesh = _ragged_mesh()
    assert mesh.n_nodes % 4 != 0
    E = 6
    scene = scenes._empty_scene(E, 2)
    rng = np.random.default_rng(5)
    for e in range(E):
        scene.n_obj[e] = 2
        for o in range(2):
            k = (e + 2 * o) % mesh.n_patches
            c = mesh.origin[k].astype(np.float64)
            r = rng.uniform(3.0, 9.0)
            scene.type[e, o] = SPHERE
            scene.shape[e, o, 0] = r
            scene.trans[e, o] = c + np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), r - rng.uniform(0.5, 3.0)])
    plan = make_plan(mesh, E, 2)
    log("[gpu] contact ragged N")
    cobj, uhat, na = gpu_contact(plan, scene)
    rc, ru, rn = oracle_lib.contact(mesh, scene)
    assert np.array_equal(cobj, rc) and np.array_equal(na, rn)
    assert max_err(uhat, ru) <= 1e-6
    assert int(na.sum()) > 0
