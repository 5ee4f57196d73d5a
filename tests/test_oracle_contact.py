"""Pins of the oracle's contact pass (Sec. III-A: SDF contact of surface nodes
with rigid objects; active nodes take the local contact displacement).

Each test checks the oracle against something other than its own formulas:
exact rational arithmetic, brute-force sampling of the primitive surfaces, or
symmetry of the setup."""
from fractions import Fraction

import numpy as np
import pytest

import scenes
from scenes import SPHERE, BOX, CAPSULE


def one_env_scene(objs):
    """objs: list of (type, shape[4], R[3,3], t[3])."""
    s = scenes._empty_scene(1, len(objs))
    s.n_obj[0] = len(objs)
    for o, (ty, sh, R, t) in enumerate(objs):
        s.type[0, o] = ty
        s.shape[0, o] = np.asarray(sh, dtype=np.float32)
        s.rot[0, o] = np.asarray(R, dtype=np.float32).ravel()
        s.trans[0, o] = np.asarray(t, dtype=np.float32)
    return s


def points_mesh(p, n=None):
    """A single 'patch' holding arbitrary points (FP32)."""
    p = np.asarray(p, dtype=np.float32).reshape(3, -1)
    if n is None:
        n = np.zeros_like(p)
        n[2] = 1.0
    return scenes.Mesh(np.array([0, p.shape[1]], np.int32), p, np.asarray(n, np.float32),
                       np.zeros((1, 3), np.float32), np.array([1.0]), [])


def test_sphere_worked_example_node_below_centre(oracle_lib):
    # config-1 pad; sphere centre exactly above node (i, j): u_hat = (0, 0, -depth)
    mesh = scenes.pad32_mesh()
    node = 17 * 32 + 9
    x0, y0 = mesh.pos[0, node], mesh.pos[1, node]
    r, depth = 5.0, 1.25
    scene = one_env_scene([(SPHERE, [r, 0, 0, 0], np.eye(3), [x0, y0, r - depth])])
    cobj, uhat, na = oracle_lib.contact(mesh, scene)
    assert cobj[0, node] == 0
    np.testing.assert_allclose(uhat[:, 0, node], [0.0, 0.0, -depth], atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_sphere_active_set_exact_rational(oracle_lib, seed):
    # A node is active iff rho^2 + z0^2 < r^2, decided in exact rational
    # arithmetic on the same FP32 inputs.
    mesh, scene, _ = scenes.config1(seed)
    cobj, uhat, na = oracle_lib.contact(mesh, scene)
    t = [Fraction(float(v)) for v in scene.trans[0, 0]]
    r = Fraction(float(scene.shape[0, 0, 0]))
    n_checked = 0
    for i in range(mesh.n_nodes):
        p = [Fraction(float(mesh.pos[a, i])) for a in range(3)]
        s = sum((p[a] - t[a]) ** 2 for a in range(3))
        if abs(float(s - r * r)) < 1e-9:
            continue  # too close to the surface for the FP64 predicate to be exact
        n_checked += 1
        assert (cobj[0, i] == 0) == (s < r * r), i
    assert n_checked > 1000
    assert na[0, 0] == int((cobj[0] >= 0).sum())
    # passive nodes carry no displacement
    assert np.all(uhat[:, 0, cobj[0] < 0] == 0.0)


def _sample_surface(ptype, shape, R, t, res):
    """Dense samples of a primitive surface in world coordinates."""
    if ptype == SPHERE:
        n = res * res * 4
        k = np.arange(n) + 0.5
        th = np.arccos(1 - 2 * k / n)
        ph = np.pi * (1 + 5 ** 0.5) * k
        q = shape[0] * np.stack([np.cos(ph) * np.sin(th), np.sin(ph) * np.sin(th), np.cos(th)], 1)
    elif ptype == BOX:
        h = shape[:3]
        pts = []
        u = np.linspace(-1, 1, res)
        A, B = np.meshgrid(u, u)
        A, B = A.ravel(), B.ravel()
        for c in range(3):
            a, b = [x for x in range(3) if x != c]
            for sg in (-1, 1):
                q = np.zeros((A.size, 3))
                q[:, c] = sg * h[c]
                q[:, a] = A * h[a]
                q[:, b] = B * h[b]
                pts.append(q)
        q = np.concatenate(pts)
    else:
        r, L = shape[0], shape[1]
        th = np.linspace(0, 2 * np.pi, res, endpoint=False)
        z = np.linspace(-L, L, res)
        TH, Z = np.meshgrid(th, z)
        cyl = np.stack([r * np.cos(TH.ravel()), r * np.sin(TH.ravel()), Z.ravel()], 1)
        n = res * res
        k = np.arange(n) + 0.5
        tt = np.arccos(1 - k / n)          # upper hemisphere
        ph = np.pi * (1 + 5 ** 0.5) * k
        hemi = r * np.stack([np.cos(ph) * np.sin(tt), np.sin(ph) * np.sin(tt), np.cos(tt)], 1)
        top = hemi + [0, 0, L]
        bot = hemi * [1, 1, -1] - [0, 0, L]
        q = np.concatenate([cyl, top, bot])
    return q @ R.T + t


@pytest.mark.parametrize("ptype", [SPHERE, BOX, CAPSULE])
def test_penetration_vs_brute_force_surface_sampling(oracle_lib, ptype):
    rng = np.random.default_rng(100 + ptype)
    R = np.eye(3) if ptype == SPHERE else scenes.random_rotation(rng)
    shape = {SPHERE: [4.0, 0, 0, 0], BOX: [3.0, 2.0, 1.5, 0], CAPSULE: [1.5, 3.0, 0, 0]}[ptype]
    t = np.array([1.0, -2.0, 0.5])
    R32 = R.astype(np.float32).astype(np.float64)
    # random points in the object frame, mostly inside
    ext = np.array({SPHERE: [4, 4, 4], BOX: [3, 2, 1.5], CAPSULE: [1.5, 1.5, 4.5]}[ptype])
    q = rng.uniform(-1.15, 1.15, size=(400, 3)) * ext
    p = (q @ R32.T + t).astype(np.float32)
    mesh = points_mesh(p.T)
    scene = one_env_scene([(ptype, shape, R, t)])
    cobj, uhat, _ = oracle_lib.contact(mesh, scene)
    surf = _sample_surface(ptype, np.asarray(shape, float), R32, t.astype(np.float32).astype(float), 180)
    spacing = {SPHERE: 0.05, BOX: 0.04, CAPSULE: 0.06}[ptype]
    pp = p.astype(np.float64)
    from scipy.spatial import cKDTree
    tree = cKDTree(surf)
    dist, _ = tree.query(pp)
    act = cobj[0] >= 0
    assert 50 < act.sum() < 400
    u = uhat[:, 0, :].T
    # |u_hat| is the distance to the surface
    np.testing.assert_allclose(np.linalg.norm(u[act], axis=1), dist[act], atol=spacing)
    # p + u_hat lies on the surface
    d_on, _ = tree.query(pp[act] + u[act])
    assert d_on.max() < spacing


@pytest.mark.parametrize("ptype", [SPHERE, BOX, CAPSULE])
def test_points_beyond_the_surface_are_passive(oracle_lib, ptype):
    # points scaled 1% beyond the brute-force surface samples are outside
    rng = np.random.default_rng(7 + ptype)
    R = np.eye(3) if ptype == SPHERE else scenes.random_rotation(rng)
    R32 = R.astype(np.float32).astype(np.float64)
    shape = {SPHERE: [4.0, 0, 0, 0], BOX: [3.0, 2.0, 1.5, 0], CAPSULE: [1.5, 3.0, 0, 0]}[ptype]
    t = np.zeros(3)
    surf = _sample_surface(ptype, np.asarray(shape, float), R32, t, 40)
    p_out = (surf * 1.01).astype(np.float32)
    p_in = (surf * 0.99).astype(np.float32)
    for pts, expect in ((p_out, False), (p_in, True)):
        mesh = points_mesh(pts.T)
        cobj, _, _ = oracle_lib.contact(mesh, one_env_scene([(ptype, shape, R, t)]))
        assert np.all((cobj[0] >= 0) == expect)


def test_mirror_symmetric_mask_centred_indenter(oracle_lib):
    # 32x32 pad centred at 0 (pitch 0.5, coordinates exact in FP32) and a
    # centred sphere: the active mask is invariant under both mirrors and the
    # transpose, bit for bit.
    mesh, scene, _ = scenes.config1(3, centred=True)
    cobj, uhat, _ = oracle_lib.contact(mesh, scene)
    m = (cobj[0] >= 0).reshape(32, 32)
    assert m.sum() > 0
    assert np.array_equal(m, m[::-1, :])
    assert np.array_equal(m, m[:, ::-1])
    assert np.array_equal(m, m.T)
    ux = uhat[0, 0].reshape(32, 32)
    uz = uhat[2, 0].reshape(32, 32)
    np.testing.assert_allclose(ux, -ux[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(uz, uz[:, ::-1], atol=1e-12)


def test_deepest_object_wins_and_ties_to_lowest_index(oracle_lib):
    p = np.array([[0.0], [0.0], [0.0]], np.float32)
    mesh = points_mesh(p)
    # sphere A: depth 1; sphere B: depth 2 -> B wins
    s = one_env_scene([(SPHERE, [3, 0, 0, 0], np.eye(3), [0, 0, 2.0]),
                       (SPHERE, [3, 0, 0, 0], np.eye(3), [0, 0, 1.0])])
    cobj, uhat, _ = oracle_lib.contact(mesh, s)
    assert cobj[0, 0] == 1
    np.testing.assert_allclose(uhat[:, 0, 0], [0, 0, -2.0], atol=1e-12)
    # identical objects -> lowest index
    s = one_env_scene([(SPHERE, [3, 0, 0, 0], np.eye(3), [0, 0, 1.0])] * 3)
    cobj, _, _ = oracle_lib.contact(mesh, s)
    assert cobj[0, 0] == 0
    # box (depth 0.5 along z) vs sphere (depth 1) -> sphere (index 1)
    s = one_env_scene([(BOX, [5, 5, 1.0, 0], np.eye(3), [0, 0, 0.5]),
                       (SPHERE, [3, 0, 0, 0], np.eye(3), [0, 0, 2.0])])
    cobj, uhat, _ = oracle_lib.contact(mesh, s)
    assert cobj[0, 0] == 1


def test_degenerate_centre_and_axis_use_minus_normal(oracle_lib):
    p = np.array([[1.0], [2.0], [3.0]], np.float32)
    n = np.array([[0.0], [0.6], [0.8]], np.float32)
    mesh = points_mesh(p, n)
    for ty, sh in ((SPHERE, [2.0, 0, 0, 0]), (CAPSULE, [2.0, 5.0, 0, 0])):
        s = one_env_scene([(ty, sh, np.eye(3), [1.0, 2.0, 3.0])])
        cobj, uhat, _ = oracle_lib.contact(mesh, s)
        assert cobj[0, 0] == 0
        np.testing.assert_allclose(uhat[:, 0, 0], -2.0 * n[:, 0].astype(np.float64), atol=1e-12)


def test_box_face_tie_goes_to_lowest_axis_and_zero_is_positive(oracle_lib):
    # point at the box centre of a cube: all slacks equal -> face x, sign +
    p = np.zeros((3, 1), np.float32)
    mesh = points_mesh(p)
    s = one_env_scene([(BOX, [1.0, 1.0, 1.0, 0], np.eye(3), [0, 0, 0])])
    cobj, uhat, _ = oracle_lib.contact(mesh, s)
    np.testing.assert_allclose(uhat[:, 0, 0], [1.0, 0, 0], atol=0)


def test_surface_nodes_are_passive(oracle_lib):
    # strict inequality: a node exactly on the sphere is passive
    p = np.array([[0.0], [0.0], [2.0]], np.float32)
    mesh = points_mesh(p)
    s = one_env_scene([(SPHERE, [2.0, 0, 0, 0], np.eye(3), [0, 0, 0])])
    cobj, _, _ = oracle_lib.contact(mesh, s)
    assert cobj[0, 0] == -1


def test_config2_contact_fraction_band(oracle_lib):
    mesh, scene, _ = scenes.config2(n_envs=64)
    cobj, _, na = oracle_lib.contact(mesh, scene)
    frac = (cobj >= 0).mean(axis=1)
    assert 0.03 < frac.mean() < 0.15
    assert np.array_equal(na.sum(axis=1), (cobj >= 0).sum(axis=1))
