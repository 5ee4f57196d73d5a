"""Pins of the oracle's hand-written adjoint (differentiability, Table 1;
calibration by gradient descent, Sec. III-A "Learn Propagation Dynamics From
FEM").

Checked against FP64 central finite differences of the oracle's own forward
(a different computation from the adjoint), against autograd of an
independent torch float64 formulation (library differentiation), and against
exact zeros implied by symmetry."""
import numpy as np
import pytest
import torch

import scenes
from scenes import SPHERE, BOX, CAPSULE, MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY
from tests.torch_ref import primitive_disp, propagate_env, t64


def _fd_check(oracle_lib, mesh, scene, model, w, env_obj_list, phi_idx, rtol=1e-6):
    g = oracle_lib.backward(mesh, scene, model, w)
    checked = 0
    for (e, o) in env_obj_list:
        fd, ok = oracle_lib.fd_gradients(mesh, scene, model, w, env=e, obj=o, phi_idx=phi_idx)
        if not ok:
            continue  # a discrete decision flips inside +-h; resample
        checked += 1
        R = scene.rot[e, o].astype(np.float64)
        tw = oracle_lib.twist_from_grad_rot(g["grad_rot"][e, o], R)
        scale = max(np.abs(fd["trans"]).max(), np.abs(fd["twist"]).max(), 1e-3)
        np.testing.assert_allclose(g["grad_trans"][e, o], fd["trans"], rtol=rtol, atol=rtol * scale)
        np.testing.assert_allclose(tw, fd["twist"], rtol=rtol, atol=rtol * scale)
        np.testing.assert_allclose(g["grad_alpha"], fd["alpha"], rtol=rtol,
                                   atol=rtol * max(np.abs(fd["alpha"]).max(), 1e-3))
        if len(phi_idx):
            np.testing.assert_allclose(g["grad_phi"][list(phi_idx)], fd["phi"], rtol=rtol,
                                       atol=rtol * max(np.abs(fd["phi"]).max(), 1e-3))
    return checked


@pytest.mark.parametrize("mode", [MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY])
def test_config3_adjoint_vs_central_fd(oracle_lib, mode):
    # config 3: config-1 pads for seeds 0..7, loss weights ~ N(0,1); one env at
    # a time so each FD run is small.
    mesh, scene, model, w = scenes.config3()
    model = model.with_mode(mode)
    rng = np.random.default_rng(11)
    phi_idx = tuple(sorted(rng.choice(17411, size=12, replace=False))) if mode != MODE_DECAY_ONLY else ()
    checked = 0
    for e in range(4):
        sc = scene.select([e])
        checked += _fd_check(oracle_lib, mesh, sc, model, w[:, e:e + 1], [(0, 0)], phi_idx)
    assert checked >= 3


@pytest.mark.parametrize("ptype", [BOX, CAPSULE])
def test_pose_gradients_vs_fd_rotated_primitives(oracle_lib, ptype):
    # boxes and capsules in arbitrary orientation on the config-2 hand
    mesh = scenes.hand_mesh(0)
    full = scenes.hand_scene(mesh, 64, 1, placement="press")
    cands = [(e, o) for e in range(64) for o in range(full.n_obj[e]) if full.type[e, o] == ptype]
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_FULL)
    rng = np.random.default_rng(5)
    checked = 0
    for (e, o) in cands[:6]:
        sc = full.select([e])
        out = oracle_lib.forward(mesh, sc, model)
        if not np.any(out["contact_obj"][0] == o):
            continue
        w = rng.standard_normal((3, 1, mesh.n_nodes))
        checked += _fd_check(oracle_lib, mesh, sc, model, w, [(0, o)], ())
        if checked >= 2:
            break
    assert checked >= 2


def test_raw_rotation_entries_vs_fd(oracle_lib):
    # grad_rot is the derivative with respect to the nine entries of R taken as
    # free inputs of the implemented function (R need not stay orthonormal).
    mesh = scenes.hand_mesh(0)
    full = scenes.hand_scene(mesh, 64, 1, placement="press")
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_DECAY_ONLY)
    rng = np.random.default_rng(3)
    done = set()
    for e in range(64):
        for o in range(full.n_obj[e]):
            ty = int(full.type[e, o])
            if ty == SPHERE or ty in done:
                continue
            sc = full.select([e])
            out = oracle_lib.forward(mesh, sc, model)
            if not np.any(out["contact_obj"][0] == o):
                continue
            w = rng.standard_normal((3, 1, mesh.n_nodes))
            g = oracle_lib.backward(mesh, sc, model, w)
            fd = np.zeros(9)
            h = 1e-5
            for c in range(9):
                vals = []
                for sgn in (1, -1):
                    s2 = oracle_lib._F64Scene(sc)
                    s2.rot[0, o, c] += sgn * h
                    vals.append(np.sum(oracle_lib.forward(mesh, s2, model)["u"] * w))
                fd[c] = (vals[0] - vals[1]) / (2 * h)
            np.testing.assert_allclose(g["grad_rot"][0, o], fd, rtol=1e-5,
                                       atol=1e-5 * np.abs(fd).max())
            done.add(ty)
    assert done == {BOX, CAPSULE}


def test_contact_adjoint_vs_torch_autograd(oracle_lib):
    mesh = scenes.hand_mesh(0)
    sc = scenes.hand_scene(mesh, 32, 1)
    cobj, uhat, _ = oracle_lib.contact(mesh, sc)
    rng = np.random.default_rng(8)
    gu = rng.standard_normal(uhat.shape) * (cobj[None] >= 0)
    ref = oracle_lib.contact_backward(mesh, sc, gu)
    P = t64(mesh.pos.T)
    n_cmp = 0
    for e in range(sc.n_envs):
        for o in range(sc.n_obj[e]):
            sel = np.nonzero(cobj[e] == o)[0]
            if sel.size == 0:
                continue
            R = t64(sc.rot[e, o].reshape(3, 3), grad=True)
            t = t64(sc.trans[e, o], grad=True)
            u, _ = primitive_disp(int(sc.type[e, o]), sc.shape[e, o].astype(np.float64), R, t, P[sel])
            L = (u * t64(gu[:, e, sel].T)).sum()
            L.backward()
            np.testing.assert_allclose(ref["grad_trans"][e, o], t.grad.numpy(), rtol=1e-10, atol=1e-10)
            gR = np.zeros(9) if R.grad is None else R.grad.numpy().ravel()
            np.testing.assert_allclose(ref["grad_rot"][e, o], gR, rtol=1e-10, atol=1e-10)
            n_cmp += 1
    assert n_cmp >= 20


@pytest.mark.parametrize("mode", [MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY])
def test_propagation_adjoint_vs_torch_autograd(oracle_lib, mode):
    mesh, scene, model = scenes.config2(n_envs=2)
    model = model.with_mode(mode)
    cobj, uhat, _ = oracle_lib.contact(mesh, scene)
    rng = np.random.default_rng(2)
    gu = rng.standard_normal(uhat.shape)
    ref = oracle_lib.propagate_backward(mesh, model, cobj, uhat, gu)
    alpha = t64(model.alpha, grad=True)
    phi = t64(model.phi, grad=True)
    L = 0
    guh = []
    for e in range(2):
        uh = t64(uhat[:, e].T, grad=True)
        act = torch.tensor(cobj[e] >= 0)
        U = propagate_env(t64(mesh.pos.T), t64(mesh.nrm.T), t64(mesh.origin), mesh.patch_offset,
                          alpha, phi, act, uh, mode)
        L = L + (U * t64(gu[:, e].T)).sum()
        guh.append(uh)
    L.backward()
    ga = np.zeros(len(model.alpha)) if alpha.grad is None else alpha.grad.numpy()
    np.testing.assert_allclose(ref["grad_alpha"], ga, rtol=1e-9, atol=1e-9)
    if mode != MODE_DECAY_ONLY:
        np.testing.assert_allclose(ref["grad_phi"], phi.grad.numpy(), rtol=1e-9, atol=1e-9)
    for e in range(2):
        act = cobj[e] >= 0
        # passive u_hat entries are the constant zero padding, not inputs
        np.testing.assert_allclose(ref["grad_uhat"][:, e, act], guh[e].grad.numpy().T[:, act],
                                   rtol=1e-9, atol=1e-9)
        assert np.all(ref["grad_uhat"][:, e, ~act] == 0.0)


def test_sphere_rotation_gradient_is_zero_and_capsule_spin_is_free(oracle_lib):
    mesh = scenes.hand_mesh(0)
    sc = scenes.hand_scene(mesh, 48, 1)
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_FULL)
    w = np.random.default_rng(4).standard_normal((3, sc.n_envs, mesh.n_nodes))
    g = oracle_lib.backward(mesh, sc, model, w)
    out = oracle_lib.forward(mesh, sc, model)
    seen_cap = 0
    for e in range(sc.n_envs):
        for o in range(sc.n_obj[e]):
            if sc.type[e, o] == SPHERE:
                assert np.all(g["grad_rot"][e, o] == 0.0)
            if sc.type[e, o] == CAPSULE and np.any(out["contact_obj"][e] == o):
                R = sc.rot[e, o].astype(np.float64).reshape(3, 3)
                tw = oracle_lib.twist_from_grad_rot(g["grad_rot"][e, o], R)
                a = R[:, 2]
                scale = np.abs(tw).max() + np.abs(g["grad_trans"][e, o]).max()
                # exact for orthonormal R; R is rounded to FP32, hence ~1e-7 relative
                assert abs(tw @ a) < 1e-6 * max(scale, 1.0)
                seen_cap += 1
    assert seen_cap >= 2
