"""Pins of the oracle's triangle-mesh contact (Sec. III-A contact detection
against object SDFs; the objects of Sec. IV are meshes).

Each test checks the oracle against something independent of its own
formulas: a different point-triangle distance (plane projection by a linear
solve, else the nearest of the three clamped segments) and dense sampling;
qhull's convex hull planes (scipy); the generalised winding number (solid
angles, Van Oosterom and Strackee) for the inside test of a non-convex rock;
and the box primitive for a triangulated cube."""
import numpy as np
import pytest

import scenes
from scenes import BOX, SPHERE
from scenes import trimeshes as tm
from tests.test_oracle_contact import one_env_scene, points_mesh


# ---------------------------------------------------------------------------
# independent geometry
# ---------------------------------------------------------------------------

def seg_closest(q, a, b):
    d = b - a
    t = np.clip(np.dot(q - a, d) / np.dot(d, d), 0.0, 1.0)
    return a + t * d


def tri_closest_independent(q, a, b, c):
    """Nearest point of the triangle: the plane projection when its
    barycentric coordinates (a 2x2 solve) are all >= 0, else the nearest of
    the three edge segments."""
    e1, e2 = b - a, c - a
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    v, w = np.linalg.solve(G, np.array([e1 @ (q - a), e2 @ (q - a)]))
    if v >= 0 and w >= 0 and v + w <= 1:
        return a + v * e1 + w * e2
    cands = [seg_closest(q, a, b), seg_closest(q, b, c), seg_closest(q, c, a)]
    return min(cands, key=lambda p: np.sum((q - p) ** 2))


def mesh_distance_independent(q, V):
    """Distance of q to a mesh given as corners V [T][3][3]."""
    return min(np.sqrt(np.sum((q - tri_closest_independent(q, *t)) ** 2)) for t in V)


def winding_number(q, V):
    """Generalised winding number of a closed outward-oriented mesh at q."""
    A, B, Cc = V[:, 0] - q, V[:, 1] - q, V[:, 2] - q
    la, lb, lc = (np.linalg.norm(X, axis=1) for X in (A, B, Cc))
    num = np.einsum("ij,ij->i", A, np.cross(B, Cc))
    den = la * lb * lc + np.einsum("ij,ij->i", A, B) * lc + np.einsum("ij,ij->i", B, Cc) * la \
        + np.einsum("ij,ij->i", Cc, A) * lb
    return float(np.sum(2.0 * np.arctan2(num, den)) / (4.0 * np.pi))


def corners(ms, m):
    return ms.verts.astype(np.float64)[ms.mesh_tris(m)]


def mesh_scene(objs):
    """objs: list of (mesh index or primitive (type, shape), R, t)."""
    lst = []
    for what, R, t in objs:
        if isinstance(what, int):
            lst.append((tm.MESH, (float(what), 0, 0, 0), R, t))
        else:
            lst.append((what[0], what[1], R, t))
    return one_env_scene(lst)


def single_mesh_set(verts, tris):
    return tm.merge([(np.asarray(verts, np.float64), np.asarray(tris))], ("m",))


# ---------------------------------------------------------------------------
# point-triangle distance
# ---------------------------------------------------------------------------

def test_closest_point_vs_independent_and_sampling(oracle_lib):
    rng = np.random.default_rng(0)
    feats = set()
    for it in range(3000):
        a, b, c = rng.standard_normal((3, 3)) * rng.uniform(0.2, 3.0)
        if it % 5 == 0:          # skinny and obtuse triangles
            c = a + (b - a) * rng.uniform(0.2, 0.8) + rng.standard_normal(3) * 0.05
        q = rng.standard_normal(3) * 3.0
        s, cp, f = oracle_lib.closest_point(q, a, b, c)
        feats.add(f)
        ref = tri_closest_independent(q, a, b, c)
        assert abs(np.sqrt(s) - np.linalg.norm(q - ref)) <= 1e-9 * (1 + np.linalg.norm(q - ref))
        assert np.allclose(cp, ref, atol=1e-7)
        assert abs(s - np.sum((q - cp) ** 2)) <= 1e-12 * (1 + s)
        # the feature names where cp lies
        if f == 4:
            assert np.array_equal(cp, a)
        elif f == 5:
            assert np.array_equal(cp, b)
        elif f == 6:
            assert np.array_equal(cp, c)
        elif f in (1, 2, 3):
            p0, p1 = {1: (a, b), 2: (b, c), 3: (c, a)}[f]
            assert np.linalg.norm(np.cross(cp - p0, p1 - p0)) <= 1e-9 * (1 + np.linalg.norm(p1 - p0) ** 2)
        if it < 200:   # dense barycentric sampling never beats the closest point
            u = rng.uniform(size=(4000, 2))
            u[u.sum(1) > 1] = 1 - u[u.sum(1) > 1]
            P = a + u[:, :1] * (b - a) + u[:, 1:] * (c - a)
            assert np.min(np.sum((P - q) ** 2, axis=1)) >= s - 1e-12
    assert feats == set(range(7))


# ---------------------------------------------------------------------------
# signed distance of whole meshes
# ---------------------------------------------------------------------------

def convex_hull_set(rng, n_pts=60, scale=(10.0, 10.0, 10.0)):
    from scipy.spatial import ConvexHull
    P = rng.standard_normal((n_pts, 3)) * np.asarray(scale)
    P = P.astype(np.float32).astype(np.float64)
    h = ConvexHull(P)
    tris = h.simplices.copy()
    for i, (t, eq) in enumerate(zip(tris, h.equations)):
        n = np.cross(P[t[1]] - P[t[0]], P[t[2]] - P[t[0]])
        if n @ eq[:3] < 0:
            tris[i] = t[[0, 2, 1]]
    used = np.unique(tris)
    remap = -np.ones(len(P), np.int64)
    remap[used] = np.arange(len(used))
    return single_mesh_set(P[used], remap[tris]), h.equations


def test_convex_hull_inside_and_depth_vs_qhull_planes(oracle_lib):
    rng = np.random.default_rng(1)
    checked_in = 0
    # two round hulls, then two flat ones whose rims are sharp edges (face
    # normals almost opposite): there the sign needs the edge and vertex
    # pseudo-normals, the closest face's normal alone gets it wrong
    for trial, scale in enumerate([(10, 10, 10)] * 2 + [(10, 10, 0.4)] * 2):
        ms, eqs = convex_hull_set(rng, scale=scale)
        R = scenes.random_rotation(rng)
        t = rng.standard_normal(3) * 5
        q = rng.uniform(-20, 20, size=(3000, 3)) * np.minimum(1.0, np.asarray(scale) / 5.0)   # object frame
        p = (q @ R.T + t).astype(np.float32)               # world, FP32 as the library receives
        qd = (p.astype(np.float64) - t.astype(np.float32).astype(np.float64)) @ R.astype(np.float32).astype(np.float64)
        mesh = points_mesh(p.T)
        scene = mesh_scene([(0, R, t)])
        cobj, uhat, na = oracle_lib.contact_mesh(mesh, scene, ms)
        plane = qd @ eqs[:, :3].T + eqs[:, 3]              # signed plane distances (unit normals)
        mx = plane.max(1)
        clear = np.abs(mx) > 1e-7
        inside = cobj[0] == 0
        assert np.array_equal(inside[clear], (mx < 0)[clear])
        Rf = R.astype(np.float32).astype(np.float64)
        for i in np.flatnonzero(inside & clear):
            j = np.argmax(plane[i])
            srt = np.sort(plane[i])
            if srt[-1] - srt[-2] < 1e-7:
                continue                                    # two nearest faces: several closest points
            depth = -plane[i, j]
            u_ref = Rf @ (eqs[j, :3] * depth)
            assert np.allclose(uhat[:, 0, i], u_ref, atol=1e-9), (trial, i)
            checked_in += 1
        assert np.array_equal(na[0], [inside.sum()])
    assert checked_in > 500


def test_nonconvex_rock_inside_by_winding_number_and_depth(oracle_lib):
    rng = np.random.default_rng(2)
    ms = tm.merge([tm.rock_mesh(rng, radius=10.0, amp=0.45, subdiv=2)], ("rock",))
    V = corners(ms, 0)
    R = scenes.random_rotation(rng).astype(np.float32).astype(np.float64)
    t = np.array([1.0, -2.0, 0.5])
    q = rng.standard_normal((600, 3)) * 6.0
    p = (q @ R.T + t).astype(np.float32)
    qd = (p.astype(np.float64) - t) @ R
    cobj, uhat, _ = oracle_lib.contact_mesh(points_mesh(p.T), mesh_scene([(0, R, t)]), ms)
    n_in = 0
    for i in range(len(q)):
        w = winding_number(qd[i], V)
        assert abs(w - round(w)) < 1e-6 and round(w) in (0, 1)
        d = mesh_distance_independent(qd[i], V)
        if d < 1e-6:
            continue
        assert (cobj[0, i] == 0) == (round(w) == 1), i
        if cobj[0, i] == 0:
            n_in += 1
            w_obj = np.linalg.solve(R, uhat[:, 0, i])      # u_hat = R (c - q); R is FP32, not exactly orthogonal
            assert abs(np.linalg.norm(w_obj) - d) <= 1e-9 * (1 + d)
            # the node moved by u_hat lands on the surface
            assert mesh_distance_independent(qd[i] + w_obj, V) <= 1e-9
    assert n_in > 80


def test_triangulated_cube_matches_box_primitive(oracle_lib):
    rng = np.random.default_rng(3)
    ms = tm.merge([tm.cube_mesh(half=8.0, n=4)], ("cube",))
    R = scenes.random_rotation(rng)
    t = np.array([0.3, 0.2, -0.1])
    p = (rng.uniform(-10, 10, size=(4000, 3)) @ R.T + t).astype(np.float32)
    mesh = points_mesh(p.T)
    cm, um, nm = oracle_lib.contact_mesh(mesh, mesh_scene([(0, R, t)]), ms)
    cb, ub, nb = oracle_lib.contact(mesh, one_env_scene([(BOX, (8.0, 8.0, 8.0, 0), R, t)]))
    assert np.array_equal(cm, cb)
    assert np.array_equal(nm, nb)
    assert (cm >= 0).sum() > 1000
    assert np.allclose(um, ub, atol=1e-9)


def test_deepest_object_wins_across_primitives_and_meshes(oracle_lib):
    rng = np.random.default_rng(4)
    ms = tm.object_set(scale=0.25)
    objs = [(2, np.eye(3), (0.0, 0.0, 0.0)), ((SPHERE, (5.0, 0, 0, 0)), np.eye(3), (2.0, 0.0, 0.0)),
            (0, scenes.random_rotation(rng), (-1.0, 1.0, 0.0)), (3, scenes.random_rotation(rng), (0.0, 0.0, 1.0))]
    p = rng.uniform(-8, 8, size=(3, 3000)).astype(np.float32)
    mesh = points_mesh(p)
    cobj, uhat, _ = oracle_lib.contact_mesh(mesh, mesh_scene(objs), ms)
    depth = np.full((len(objs), p.shape[1]), -np.inf)
    single = []
    for o, ob in enumerate(objs):
        c, u, _ = oracle_lib.contact_mesh(mesh, mesh_scene([ob]), ms)
        single.append(u)
        hit = c[0] == 0
        depth[o, hit] = np.linalg.norm(u[:, 0, hit], axis=0)
    win = np.where(np.isfinite(depth).any(0), np.argmax(depth, axis=0), -1)
    assert np.array_equal(cobj[0], win)
    assert len(np.unique(win)) == 5
    for o in range(len(objs)):
        sel = win == o
        assert np.array_equal(uhat[:, 0, sel], single[o][:, 0, sel])


def test_mesh_objects_ignored_by_primitive_contact_and_bad_index(oracle_lib):
    ms = tm.object_set(scale=0.25)
    p = np.zeros((3, 4), np.float32)
    p[0] = [0.0, 1.0, 2.0, 3.0]
    mesh = points_mesh(p)
    s = mesh_scene([(0, np.eye(3), (0, 0, 0))])
    c, _, _ = oracle_lib.contact(mesh, s)
    assert (c == -1).all()
    c, _, _ = oracle_lib.contact_mesh(mesh, s, ms)
    assert (c == 0).all()
    for bad in (4.0, -1.0, 0.5):
        s.shape[0, 0, 0] = bad
        c, u, na = oracle_lib.contact_mesh(mesh, s, ms)
        assert (c == -1).all() and (u == 0).all() and (na == 0).all()


def test_surface_points_are_passive(oracle_lib):
    # nodes exactly at vertices, edge midpoints and face centroids of a cube
    ms = tm.merge([tm.cube_mesh(half=4.0, n=2)], ("cube",))
    V = corners(ms, 0)
    pts = np.concatenate([V[:, 0], (V[:, 0] + V[:, 1]) / 2, V.mean(1)]).astype(np.float32)
    c, _, _ = oracle_lib.contact_mesh(points_mesh(pts.T), mesh_scene([(0, np.eye(3), (0, 0, 0))]), ms)
    assert (c == -1).all()


def test_open_or_misoriented_mesh_is_rejected(oracle_lib):
    v, f = tm.cube_mesh(half=4.0, n=1)
    p = np.zeros((3, 1), np.float32)
    s = mesh_scene([(0, np.eye(3), (0, 0, 0))])
    with pytest.raises(RuntimeError):
        oracle_lib.contact_mesh(points_mesh(p), s, single_mesh_set(v, f[1:]))
    g = f.copy()
    g[0] = g[0, [0, 2, 1]]
    with pytest.raises(RuntimeError):
        oracle_lib.contact_mesh(points_mesh(p), s, single_mesh_set(v, g))


def test_object_set_is_closed_and_oriented(oracle_lib):
    ms = tm.object_set()
    for m in range(ms.n_meshes):
        V = corners(ms, m)
        assert abs(winding_number(np.zeros(3), V) - 1.0) < 1e-9
        pn = oracle_lib.mesh_pseudonormals(ms, m)
        assert np.allclose(np.linalg.norm(pn[:, 0], axis=1), 1.0)


# ---------------------------------------------------------------------------
# adjoint with respect to the poses
# ---------------------------------------------------------------------------

def _fd_mesh(oracle_lib, mesh, scene, ms, g, e, o, h=1e-6):
    """Central differences of L = sum(g * u_hat) in FP64 for the translation
    and the twist (R' = exp([w]_x) R) of object o of env e.  Returns the six
    values and whether the contact masks agreed on both sides of every step."""
    S = oracle_lib._F64Scene(scene)
    out, ok = [], True
    for kind in ("t", "w"):
        for c in range(3):
            vals, masks = [], []
            for sgn in (1, -1):
                Sp = oracle_lib._F64Scene(S)
                if kind == "t":
                    Sp.trans[e, o, c] += sgn * h
                else:
                    w = np.zeros(3)
                    w[c] = sgn * h
                    Sp.rot[e, o] = (oracle_lib.expm_so3(w) @ S.rot[e, o].reshape(3, 3)).ravel()
                cobj, uhat, _ = oracle_lib.contact_mesh(mesh, Sp, ms)
                vals.append(float(np.sum(g * uhat)))
                masks.append(cobj)
            ok &= bool(np.array_equal(*masks))
            out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out), ok


@pytest.mark.parametrize("mesh_idx", [0, 1, 2, 3, "L"])
def test_mesh_pose_adjoint_vs_central_differences(oracle_lib, mesh_idx):
    # each stand-in mesh, and an L-shaped prism whose reflex edge is the
    # closest feature of some nodes (edge Jacobian), pressed into the pad at
    # a random pose: the analytic translation and twist gradients against
    # FP64 central differences
    rng = np.random.default_rng(2 if mesh_idx == "L" else 40 + mesh_idx)
    if mesh_idx == "L":
        ms, mesh_idx = tm.merge([tm.l_prism_mesh()], ("L",)), 0
        edge_case = True
    else:
        ms, edge_case = tm.object_set(scale=0.25), False
    mesh = scenes.pad32_mesh()
    R = scenes.random_rotation(rng)
    h = ms.support_extent(mesh_idx, R, np.array([0.0, 0.0, -1.0]))
    t = np.array([0.3, -0.2, h - 2.5]) if edge_case else np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), h - 1.5])
    scene = mesh_scene([(mesh_idx, R, t)])
    if edge_case:
        feat = oracle_lib.contact_mesh_features(mesh, scene, ms)
        assert ((feat >= 1) & (feat <= 3)).sum() >= 2
    g = rng.standard_normal((3, 1, mesh.n_nodes))
    cobj, _, _ = oracle_lib.contact_mesh(mesh, scene, ms)
    assert (cobj >= 0).sum() > 30
    ref = oracle_lib.contact_mesh_backward(mesh, scene, ms, g)
    fd, ok = _fd_mesh(oracle_lib, mesh, scene, ms, g, 0, 0)
    assert ok
    an = np.concatenate([ref["grad_trans"][0, 0],
                         oracle_lib.twist_from_grad_rot(ref["grad_rot"][0, 0], scene.rot[0, 0].astype(np.float64))])
    scale = np.max(np.abs(an))
    assert np.allclose(an, fd, rtol=1e-5, atol=1e-6 * scale), (an, fd)


def test_mesh_adjoint_with_a_primitive_and_raw_rotation_entries(oracle_lib):
    # a triangulated cube at a random pose beside a sphere: the sphere's part
    # equals the primitive adjoint, and the cube's rotation gradient matches
    # differences along all nine entries of R taken as free inputs
    rng = np.random.default_rng(7)
    ms = tm.merge([tm.cube_mesh(half=3.0, n=2)], ("cube",))
    mesh = scenes.pad32_mesh()
    corner_down = scenes.random_rotation(rng)
    objs = [(0, corner_down, (1.0, -1.5, ms.support_extent(0, corner_down, np.array([0, 0, -1.0])) - 1.0)),
            ((SPHERE, (3.0, 0, 0, 0)), np.eye(3), (-4.0, 3.0, 2.2))]
    scene = mesh_scene(objs)
    g = rng.standard_normal((3, 1, mesh.n_nodes))
    cobj, _, _ = oracle_lib.contact_mesh(mesh, scene, ms)
    assert {0, 1} <= set(np.unique(cobj).tolist())
    ref = oracle_lib.contact_mesh_backward(mesh, scene, ms, g)
    # the sphere's part equals the primitive adjoint of a scene holding only the sphere's winners
    only_sphere = g * (cobj == 1)[None]
    prim = oracle_lib.contact_backward(mesh, scene, only_sphere)
    assert np.allclose(ref["grad_trans"][0, 1], prim["grad_trans"][0, 1], rtol=1e-12, atol=1e-12)
    # raw rotation entries of the cube by differences
    S = oracle_lib._F64Scene(scene)
    hstep = 1e-6
    for k in range(9):
        vals = []
        for sgn in (1, -1):
            Sp = oracle_lib._F64Scene(S)
            Sp.rot[0, 0, k] += sgn * hstep
            vals.append(float(np.sum(g * oracle_lib.contact_mesh(mesh, Sp, ms)[1])))
        fd = (vals[0] - vals[1]) / (2 * hstep)
        assert abs(fd - ref["grad_rot"][0, 0, k]) <= 1e-5 * (1 + abs(fd)), (k, fd, ref["grad_rot"][0, 0, k])
