"""Pins of the oracle's propagation (Eq. 1 decay, residual network Phi,
Eq. 2 assembly; Sec. III-A "Modeling Contact Propagation Dynamics" and
"Residual Displacement Correction").

The oracle is checked against: an explicitly built propagation matrix Omega
multiplied with numpy (library routine), closed forms for one active node,
linearity, rigid-motion invariance of the decay term, permutation
equivariance and special cases of the network, an independent vectorised
torch float64 forward, and a hand-computed example stored under
tests/golden/."""
import json
import os

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

import scenes
from scenes import MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY, phi_offsets
from tests.torch_ref import propagate_env, t64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _contact(oracle_lib, seed=0, centred=False):
    mesh, scene, model = scenes.config1(seed, centred)
    cobj, uhat, na = oracle_lib.contact(mesh, scene)
    return mesh, scene, model, cobj, uhat


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_decay_equals_explicit_omega_matmul(oracle_lib, seed):
    # Eq. 1 written as the (n-m) x m matrix Omega times U_a (numpy @).
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, seed)
    U = oracle_lib.propagate(mesh, model, cobj, uhat, mode=MODE_DECAY_ONLY)
    act = cobj[0] >= 0
    P = mesh.pos.T.astype(np.float64)
    Om = np.exp(-float(model.alpha[0]) * cdist(P[~act], P[act]))
    Ua = uhat[:, 0, act].T
    np.testing.assert_allclose(U[:, 0, ~act].T, Om @ Ua, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(U[:, 0, act], uhat[:, 0, act])


def test_single_active_node_closed_form_and_monotone_decay(oracle_lib):
    mesh = scenes.pad32_mesh()
    cobj = -np.ones((1, mesh.n_nodes), np.int8)
    j = 16 * 32 + 16
    cobj[0, j] = 0
    uhat = np.zeros((3, 1, mesh.n_nodes))
    uhat[:, 0, j] = [0.1, -0.2, -0.7]
    model = scenes.Model(MODE_DECAY_ONLY, np.array([3.0], np.float32), np.zeros(17411, np.float32))
    U = oracle_lib.propagate(mesh, model, cobj, uhat)
    P = mesh.pos.astype(np.float64)
    d = np.linalg.norm(P - P[:, j:j + 1], axis=0)
    expect = np.exp(-3.0 * d)[None, :] * uhat[:, 0, j][:, None]
    expect[:, j] = uhat[:, 0, j]
    np.testing.assert_allclose(U[:, 0], expect, rtol=1e-13, atol=1e-300)
    # along a row of nodes moving away from j, |U| strictly decreases
    row = [16 * 32 + 16 + s for s in range(1, 16)]
    mags = np.linalg.norm(U[:, 0, row], axis=0)
    assert np.all(np.diff(mags) < 0)


def test_decay_is_linear_in_active_displacements(oracle_lib):
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 4)
    m = model.with_mode(MODE_DECAY_ONLY)
    U1 = oracle_lib.propagate(mesh, m, cobj, uhat)
    rng = np.random.default_rng(0)
    uhat2 = np.where(cobj[None] >= 0, rng.standard_normal(uhat.shape), 0.0)
    U2 = oracle_lib.propagate(mesh, m, cobj, uhat2)
    U12 = oracle_lib.propagate(mesh, m, cobj, 2.5 * uhat - 0.5 * uhat2)
    np.testing.assert_allclose(U12, 2.5 * U1 - 0.5 * U2, rtol=1e-11, atol=1e-13)


def test_decay_invariant_under_rigid_motion(oracle_lib):
    # The decay prior is translation invariant (Sec. III-A) and depends only on
    # distances: rotating and translating nodes and displacements together
    # rotates U.
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 5)
    m = model.with_mode(MODE_DECAY_ONLY)
    U = oracle_lib.propagate(mesh, m, cobj, uhat)
    R = scenes.random_rotation(np.random.default_rng(9))
    tr = np.array([3.0, -1.0, 2.0])
    mesh2 = scenes.Mesh(mesh.patch_offset, (R @ mesh.pos.astype(np.float64) + tr[:, None]),
                        R @ mesh.nrm.astype(np.float64), mesh.origin, mesh.pitch)
    uhat_r = np.einsum("ab,bek->aek", R, uhat)
    U2 = oracle_lib.propagate(mesh2, m, cobj, uhat_r)
    np.testing.assert_allclose(U2, np.einsum("ab,bek->aek", R, U), atol=1e-12)


def test_decay_mirror_symmetry_centred_indenter(oracle_lib):
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 2, centred=True)
    U = oracle_lib.propagate(mesh, model.with_mode(MODE_DECAY_ONLY), cobj, uhat)
    ux, uy, uz = (U[a, 0].reshape(32, 32) for a in range(3))
    np.testing.assert_allclose(ux, -ux[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(uy, uy[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(uz, uz[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(uz, uz[::-1, :], atol=1e-12)


def test_no_contact_gives_zero_deformation(oracle_lib):
    mesh, scene, model = scenes.config1(0)
    scene.trans[0, 0, 2] = 5.5          # sphere lifted clear of the pad
    for mode in (MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY):
        out = oracle_lib.forward(mesh, scene, model.with_mode(mode))
        assert out["n_active"].sum() == 0
        assert np.all(out["u"] == 0.0)


def test_zero_output_layer_reduces_full_to_decay_only(oracle_lib):
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 6)
    off = phi_offsets()
    phi = model.phi.copy()
    phi[off["W5"]:] = 0.0                      # W5 and b5
    m0 = scenes.Model(MODE_FULL, model.alpha, phi)
    U_full = oracle_lib.propagate(mesh, m0, cobj, uhat)
    U_dec = oracle_lib.propagate(mesh, m0.with_mode(MODE_DECAY_ONLY), cobj, uhat)
    np.testing.assert_array_equal(U_full, U_dec)


def test_full_is_sum_of_ablations_on_passive_nodes(oracle_lib):
    # Eq. 2: U_p = Omega U_a + Phi_p.  The two ablations (Table 2 rows) add up
    # to the full model; active nodes are u_hat in every mode.
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 7)
    Uf = oracle_lib.propagate(mesh, model, cobj, uhat, mode=MODE_FULL)
    Ud = oracle_lib.propagate(mesh, model, cobj, uhat, mode=MODE_DECAY_ONLY)
    Ur = oracle_lib.propagate(mesh, model, cobj, uhat, mode=MODE_RESIDUAL_ONLY)
    act = cobj[0] >= 0
    np.testing.assert_allclose(Uf[:, 0, ~act], Ud[:, 0, ~act] + Ur[:, 0, ~act], atol=1e-14)
    for U in (Uf, Ud, Ur):
        np.testing.assert_array_equal(U[:, 0, act], uhat[:, 0, act])
    # the residual is a genuine correction of a few hundredths of a mm
    r = np.abs(Ur[:, 0, ~act])
    assert 1e-3 < r.max() < 0.5


def test_residual_is_permutation_equivariant(oracle_lib):
    # Max-pooling makes the network symmetric in node order: permuting a
    # patch's nodes permutes the output rows.
    mesh, scene, model, cobj, uhat = _contact(oracle_lib, 8)
    perm = np.random.default_rng(1).permutation(mesh.n_nodes)
    mesh_p = scenes.Mesh(mesh.patch_offset, mesh.pos[:, perm], mesh.nrm[:, perm], mesh.origin, mesh.pitch)
    U = oracle_lib.propagate(mesh, model, cobj, uhat, mode=MODE_RESIDUAL_ONLY)
    Up = oracle_lib.propagate(mesh_p, model, cobj[:, perm], uhat[:, :, perm], mode=MODE_RESIDUAL_ONLY)
    np.testing.assert_allclose(Up, U[:, :, perm], atol=1e-14)


@pytest.mark.parametrize("mode", [MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY])
def test_forward_vs_independent_torch_float64(oracle_lib, mode):
    mesh, scene, model = scenes.config2(n_envs=3)
    out = oracle_lib.forward(mesh, scene, model.with_mode(mode))
    for e in range(3):
        act = torch.tensor(out["contact_obj"][e] >= 0)
        U = propagate_env(t64(mesh.pos.T), t64(mesh.nrm.T), t64(mesh.origin), mesh.patch_offset,
                          t64(model.alpha), t64(model.phi), act, t64(out["uhat"][:, e].T), mode)
        np.testing.assert_allclose(out["u"][:, e].T, U.numpy(), atol=1e-12, rtol=1e-12)


def test_golden_two_node_hand_example(oracle_lib):
    # Hand-computed example (values derived on paper, see the fixture).
    with open(os.path.join(GOLDEN, "two_node_example.json")) as f:
        g = json.load(f)
    mesh = scenes.Mesh(np.array([0, 2], np.int32), np.array(g["pos"], np.float32),
                       np.array(g["nrm"], np.float32), np.array([g["origin"]], np.float32),
                       np.array([1.0]), [])
    phi = np.zeros(17411, np.float32)
    off = phi_offsets()
    for name, (idx, val) in g["phi_entries"].items():
        for i, v in zip(idx, val):
            phi[off[name] + i] = v
    model = scenes.Model(g["mode"], np.array([g["alpha"]], np.float32), phi)
    cobj = np.array([g["contact_obj"]], np.int8)
    uhat = np.array(g["uhat"], np.float64).reshape(3, 1, 2)
    U = oracle_lib.propagate(mesh, model, cobj, uhat)
    np.testing.assert_allclose(U[:, 0, :], np.array(g["expected_u"]), atol=1e-12)
