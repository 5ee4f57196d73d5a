"""Seeded synthetic closed triangle meshes for rigid objects, and hand scenes
that hold them.

The paper's objects (an egg, a can, a rock, a cube; Sec. IV) are meshes whose
signed distance fields drive contact.  Their files are not available, so
stand-ins of the same kinds and sizes are drawn here: an egg-shaped
ellipsoid, a capped cylinder, a star-shaped rock with random bumps (not
convex) and a cube with subdivided faces.  This module only draws geometry:
vertex positions (FP64, rounded once to FP32), triangle index lists with
outward orientation, and object placements.  It holds none of the contact
arithmetic.

A mesh set concatenates several meshes:

* verts       float32 [V][3]   object-frame vertex positions, mm
* tris        int32   [T][3]   vertex indices, counter-clockwise seen from
                               outside (right-hand normal points outward)
* tri_offset  int32   [M+1]    mesh m owns triangles tri_offset[m] ..
                               tri_offset[m+1]-1

An object of type MESH (3) in a scene names its mesh by shape[0] (the mesh
index as a float); shape[1..3] are unused.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import HAND_OFFSET, _empty_scene, draw_primitive, random_rotation, support_extent

MESH = 3


@dataclass
class TriMeshSet:
    verts: np.ndarray       # float32 [V][3]
    tris: np.ndarray        # int32 [T][3]
    tri_offset: np.ndarray  # int32 [M+1]
    names: tuple

    @property
    def n_meshes(self):
        return int(self.tri_offset.shape[0] - 1)

    @property
    def n_verts(self):
        return int(self.verts.shape[0])

    @property
    def n_tris(self):
        return int(self.tris.shape[0])

    def mesh_tris(self, m):
        return self.tris[self.tri_offset[m]:self.tri_offset[m + 1]]

    def mesh_verts(self, m):
        """Vertices used by mesh m (FP64)."""
        return self.verts[np.unique(self.mesh_tris(m))].astype(np.float64)

    def radius(self, m):
        return float(np.sqrt((self.mesh_verts(m) ** 2).sum(1)).max())

    def support_extent(self, m, R, u):
        """Largest extent of mesh m, rotated by R, along unit direction u."""
        return float((self.mesh_verts(m) @ (R.T @ u)).max())


def _weld(tri_pts):
    """Triangles given by corner coordinates [T][3][3] -> (verts, tris) with
    coincident corners merged."""
    key = {}
    verts, tris = [], []
    for tri in tri_pts:
        idx = []
        for p in tri:
            k = tuple(np.round(p, 9))
            if k not in key:
                key[k] = len(verts)
                verts.append(p)
            idx.append(key[k])
        tris.append(idx)
    return np.asarray(verts, np.float64), np.asarray(tris, np.int64)


def _orient_outward(verts, tris, centre=(0.0, 0.0, 0.0)):
    """Flip triangles whose normal points towards `centre` (star-shaped
    meshes about it)."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", (a + b + c) / 3.0 - np.asarray(centre), n) < 0.0
    tris = tris.copy()
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def icosphere(subdiv):
    """Unit icosphere: the icosahedron with every triangle split into four,
    `subdiv` times, vertices pushed to the unit sphere (20 * 4^subdiv
    triangles)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
                  [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
                  [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    verts = list(v)
    for _ in range(subdiv):
        mid = {}

        def midpoint(i, j):
            k = (min(i, j), max(i, j))
            if k not in mid:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mid[k] = len(verts) - 1
            return mid[k]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.asarray(nf)
    verts = np.asarray(verts)
    return verts, _orient_outward(verts, np.asarray(f))


def egg_mesh(radius=20.0, length=28.0, taper=0.15, subdiv=3):
    """Egg: an ellipsoid of equatorial radius `radius` and half-length
    `length` along z, the +z half narrowed by `taper` (convex)."""
    v, f = icosphere(subdiv)
    z = v[:, 2]
    s = 1.0 - taper * np.clip(z, 0.0, None)
    out = np.stack([v[:, 0] * radius * s, v[:, 1] * radius * s, z * length], axis=1)
    return out, f


def can_mesh(radius=15.0, half_len=30.0, n_seg=48, n_rings=8):
    """Can: a capped cylinder about z, fan-triangulated caps (convex)."""
    th = 2.0 * np.pi * np.arange(n_seg) / n_seg
    zs = np.linspace(-half_len, half_len, n_rings + 1)
    ring = lambda z: np.stack([radius * np.cos(th), radius * np.sin(th), np.full(n_seg, z)], axis=1)
    tris = []
    for j in range(n_rings):
        lo, hi = ring(zs[j]), ring(zs[j + 1])
        for i in range(n_seg):
            i1 = (i + 1) % n_seg
            tris += [[lo[i], lo[i1], hi[i1]], [lo[i], hi[i1], hi[i]]]
    for z in (-half_len, half_len):
        r, c = ring(z), np.array([0.0, 0.0, z])
        for i in range(n_seg):
            tris.append([c, r[i], r[(i + 1) % n_seg]])
    v, f = _weld(np.asarray(tris))
    return v, _orient_outward(v, f)


def rock_mesh(rng, radius=20.0, amp=0.3, n_bumps=12, subdiv=3):
    """Rock: a unit icosphere whose radius along direction d is
    radius (1 + sum_k a_k exp(-|d - c_k|^2 / w_k^2)), with bump heights a_k
    in U(-amp, amp) (dents and knobs, so not convex) about random centres;
    star-shaped about the origin, so closed and outward oriented."""
    v, f = icosphere(subdiv)
    c = rng.standard_normal((n_bumps, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    a = rng.uniform(-amp, amp, n_bumps)
    w = rng.uniform(0.35, 0.7, n_bumps)
    d2 = ((v[:, None, :] - c[None]) ** 2).sum(-1)
    r = radius * (1.0 + (a * np.exp(-d2 / w ** 2)).sum(1))
    return v * r[:, None], f


def cube_mesh(half=20.0, n=8):
    """Cube of half side `half`, every face an n x n grid of split squares
    (convex)."""
    g = np.linspace(-half, half, n + 1)
    tris = []
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            u_ax, v_ax = [a for a in range(3) if a != ax]
            for i in range(n):
                for j in range(n):
                    q = []
                    for (ii, jj) in ((i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)):
                        p = np.zeros(3)
                        p[ax] = sgn * half
                        p[u_ax], p[v_ax] = g[ii], g[jj]
                        q.append(p)
                    tris += [[q[0], q[1], q[2]], [q[0], q[2], q[3]]]
    v, f = _weld(np.asarray(tris))
    return v, _orient_outward(v, f)


def l_prism_mesh(arm=4.0, width=2.0, half_height=3.0):
    """An L-shaped prism along z (not convex): the L of two arms of length
    `arm` and width `width` in the xy plane, centred on its bounding box,
    extruded over z in [-half_height, half_height].  Its inner corner is a
    reflex edge."""
    L = np.array([[0, 0], [arm, 0], [arm, width], [width, width], [width, arm], [0, arm]], np.float64)
    L -= L.max(0) / 2.0
    n = len(L)
    v = np.concatenate([np.c_[L, np.full(n, -half_height)], np.c_[L, np.full(n, half_height)]])
    f = []
    for k in range(1, n - 1):              # caps: fans from the outer corner (the L is star-shaped from it)
        f.append([n + 0, n + k, n + k + 1])
        f.append([0, k + 1, k])
    for k in range(n):                     # sides, the polygon counter-clockwise seen from +z
        k1 = (k + 1) % n
        f += [[k, k1, n + k1], [k, n + k1, n + k]]
    return v, np.asarray(f)


def merge(meshes, names):
    """Concatenate (verts, tris) pairs into a TriMeshSet (vertices rounded to
    FP32 once)."""
    verts, tris, off = [], [], [0]
    base = 0
    for v, f in meshes:
        verts.append(v)
        tris.append(np.asarray(f) + base)
        base += len(v)
        off.append(off[-1] + len(f))
    return TriMeshSet(np.concatenate(verts).astype(np.float32), np.concatenate(tris).astype(np.int32),
                      np.asarray(off, np.int32), tuple(names))


def object_set(seed=0, scale=1.0, subdiv=3, cube_n=8, can_seg=48):
    """The four stand-in objects (egg, can, rock, cube), lengths times
    `scale`: 1280, 864, 1280 and 768 triangles at the defaults."""
    rng = np.random.default_rng([seed, 31])
    ms = [egg_mesh(subdiv=subdiv), can_mesh(n_seg=can_seg), rock_mesh(rng, subdiv=subdiv), cube_mesh(n=cube_n)]
    return merge([(v * scale, f) for v, f in ms], ("egg", "can", "rock", "cube"))


def hand_mesh_scene(mesh, meshset, n_envs, seed=2, max_obj=3, p_mesh=1.0, offset=HAND_OFFSET, scale=1.0):
    """Per env: object count U{1..max_obj}; each object is a mesh of the set
    (uniform index, uniform rotation) with probability p_mesh, else a
    primitive drawn as by draw_primitive.  Placement as for the primitives:
    a node p* uniform over the hand, the object's extreme point along -z at
    depth U(offset) below it.  Env e draws from stream (seed, e)."""
    scene = _empty_scene(n_envs, max_obj)
    for e in range(n_envs):
        rng = np.random.default_rng([seed, e, 3])
        cnt = int(rng.integers(1, max_obj + 1))
        scene.n_obj[e] = cnt
        for o in range(cnt):
            node = int(rng.integers(0, mesh.n_nodes))
            p = mesh.pos[:, node].astype(np.float64)
            n = np.array([0.0, 0.0, 1.0])
            s = rng.uniform(offset[0] * scale, offset[1] * scale)
            if rng.uniform() < p_mesh:
                m = int(rng.integers(0, meshset.n_meshes))
                R = random_rotation(rng)
                h = meshset.support_extent(m, R, -n)
                scene.type[e, o] = MESH
                scene.shape[e, o] = (float(m), 0.0, 0.0, 0.0)
            else:
                ptype, shape, R = draw_primitive(rng, scale)
                h = support_extent(ptype, shape, R, n)
                scene.type[e, o] = ptype
                scene.shape[e, o] = shape
            scene.rot[e, o] = R.ravel()
            scene.trans[e, o] = p + (h - s) * n
    return scene
