"""Pins of the oracle's real-sensor regressor (attention-pooled PointNet,
appendix "Modeling Real Sensors"): a configuration that reduces it to a
closed form (softmax-weighted means of rectified inputs), invariance to node
order, to duplicating every node, to a constant added to every attention
score and to moving a patch with its origin, and the residual connection against an equivalent network without
it."""
import numpy as np
import pytest

import oracle
import scenes


def _pad(n=7, seed=0):
    """One flat patch of n nodes (random positions within 5 mm), origin 0."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-5.0, 5.0, size=(3, n))
    nrm = np.zeros((3, n)); nrm[2] = 1.0
    return scenes.Mesh(np.array([0, n], np.int32), pos, nrm, np.zeros((1, 3)), np.ones(1), [])


def _blocks(reg):
    return {k: reg[o:o + int(np.prod(sh))].reshape(sh) for k, (o, sh) in oracle.reg_offsets().items()}


def _closed_form_params():
    reg = np.zeros(oracle.REG_SIZE)
    B = _blocks(reg)
    B["E1"][:6, :6] = np.eye(6)          # h1[:6] = relu(x)
    B["E3"][:64, :64] = np.eye(64)       # f[:64] = h2 = h1 (E2 = 0: relu(0) + h1)
    B["A1"][0, 0] = 1.0                  # t0 = tanh(f0)
    B["a2"][0] = 1.0                     # s = tanh(relu(x0))
    B["D1"][:128, :128] = np.eye(128)    # relu(g[:128]) = g[:128] (g >= 0)
    B["D2"][:8, :8] = np.eye(8)          # y = g[:8]
    return reg


def test_closed_form_softmax_weighted_mean(oracle_lib):
    mesh = _pad(9)
    rng = np.random.default_rng(3)
    E = 3
    u = rng.uniform(-2.0, 2.0, size=(3, E, mesh.n_nodes))
    y = oracle.regress(mesh, _closed_form_params(), u)
    for e in range(E):
        x = np.concatenate([mesh.pos, u[:, e]], axis=0)      # [6][n]
        r = np.maximum(x, 0.0)
        s = np.tanh(r[0])
        a = np.exp(s - s.max()); a /= a.sum()
        exp = np.zeros(8)
        exp[:6] = r @ a
        assert np.allclose(y[e, 0], exp, rtol=1e-13, atol=1e-13)
    # the head's hidden layer rectifies: D1 = -I, d1 = 1 gives y = relu(1 - g)
    reg = _closed_form_params()
    B = _blocks(reg)
    B["D1"][:128, :128] = -np.eye(128)
    B["d1"][:] = 1.0
    y = oracle.regress(mesh, reg, u)
    for e in range(E):
        x = np.concatenate([mesh.pos, u[:, e]], axis=0)
        r = np.maximum(x, 0.0)
        s = np.tanh(r[0])
        a = np.exp(s - s.max()); a /= a.sum()
        g = np.zeros(8)
        g[:6] = r @ a
        assert np.allclose(y[e, 0], np.maximum(1.0 - g, 0.0), rtol=1e-13, atol=1e-13)
        assert (g > 1.0).any() and (g < 1.0).any()     # both sides of the hinge


def test_single_node_and_uniform_attention(oracle_lib):
    # one node: the attention weight is 1; zero score weights: plain mean
    reg = _closed_form_params()
    m1 = _pad(1, seed=5)
    u = np.random.default_rng(1).uniform(-1, 1, size=(3, 2, 1))
    y = oracle.regress(m1, reg, u)
    for e in range(2):
        x = np.concatenate([m1.pos[:, 0], u[:, e, 0]])
        assert np.allclose(y[e, 0, :6], np.maximum(x, 0.0), rtol=1e-14, atol=1e-14)
    B = _blocks(reg)
    B["a2"][:] = 0.0
    m = _pad(11, seed=6)
    u = np.random.default_rng(2).uniform(-1, 1, size=(3, 1, 11))
    y = oracle.regress(m, reg, u)
    x = np.concatenate([m.pos, u[:, 0]], axis=0)
    assert np.allclose(y[0, 0, :6], np.maximum(x, 0.0).mean(axis=1), rtol=1e-13, atol=1e-13)


def test_node_order_duplication_and_score_shift_change_nothing(oracle_lib):
    reg = scenes.draw_regressor(np.random.default_rng(4)).astype(np.float64)
    mesh = _pad(13, seed=7)
    u = np.random.default_rng(8).uniform(-2, 2, size=(3, 2, 13))
    y = oracle.regress(mesh, reg, u)
    perm = np.random.default_rng(9).permutation(13)
    mp = scenes.Mesh(mesh.patch_offset, mesh.pos[:, perm], mesh.nrm[:, perm], mesh.origin, mesh.pitch, [])
    assert np.allclose(oracle.regress(mp, reg, u[:, :, perm]), y, rtol=1e-12, atol=1e-12)
    dup = np.concatenate([np.arange(13), np.arange(13)])
    md = scenes.Mesh(np.array([0, 26], np.int32), mesh.pos[:, dup], mesh.nrm[:, dup], mesh.origin, mesh.pitch, [])
    assert np.allclose(oracle.regress(md, reg, u[:, :, dup]), y, rtol=1e-12, atol=1e-12)
    r2 = reg.copy()
    r2[oracle.reg_offsets()["a0"][0]] += 3.7
    assert np.allclose(oracle.regress(mesh, r2, u), y, rtol=1e-12, atol=1e-12)
    assert not np.allclose(y[0], y[1])     # the displacements do reach the output
    # moving the patch and its origin together: the inputs are p - o
    shift = np.array([[40.0], [-25.0], [7.5]])
    mt = scenes.Mesh(mesh.patch_offset, mesh.pos + shift, mesh.nrm, mesh.origin + shift.T, mesh.pitch, [])
    assert np.allclose(oracle.regress(mt, reg, u), y, rtol=1e-12, atol=1e-12)
    mo = scenes.Mesh(mesh.patch_offset, mesh.pos, mesh.nrm, mesh.origin + shift.T, mesh.pitch, [])
    assert not np.allclose(oracle.regress(mo, reg, u), y)


def test_residual_connection(oracle_lib):
    # with E2 = 0 and e2 = 0 the second layer passes h1 through (relu(0) + h1);
    # with E2 = I it doubles it (relu(h1) + h1, h1 >= 0): halving E3 then gives
    # the same network
    reg = scenes.draw_regressor(np.random.default_rng(10)).astype(np.float64)
    B = _blocks(reg)
    B["E2"][:] = 0.0
    B["e2"][:] = 0.0
    mesh = _pad(10, seed=11)
    u = np.random.default_rng(12).uniform(-2, 2, size=(3, 2, 10))
    ya = oracle.regress(mesh, reg, u)
    rb = reg.copy()
    Bb = _blocks(rb)
    Bb["E2"][:] = np.eye(64)
    Bb["E3"][:] *= 0.5
    yb = oracle.regress(mesh, rb, u)
    assert np.allclose(ya, yb, rtol=1e-12, atol=1e-12)
