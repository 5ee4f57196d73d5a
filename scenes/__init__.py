"""Seeded synthetic workloads for the ETac tactile step.

This module only draws inputs: elastomer patch geometry, rigid primitives and
their poses, and propagation-model parameters.  It holds none of the method's
arithmetic (no penetration test, no propagation, no network), so that the FP64
oracle and the GPU path can both consume exactly the same arrays.

Every array handed to either side is FP32 (positions in mm, alpha in 1/mm);
geometry is built in FP64 and rounded once.  Layouts:

* mesh.pos, mesh.nrm   float32 [3][N]   SoA, x then y then z
* mesh.patch_offset    int32   [K+1]    patch k owns nodes offset[k]..offset[k+1]-1
* mesh.origin          float32 [K][3]   per-patch origin o_k fed to the network
* scene.type           int32   [E][O]   0 sphere, 1 box, 2 capsule
* scene.shape          float32 [E][O][4] sphere (r) | box (hx,hy,hz) | capsule (r, half_len)
* scene.rot            float32 [E][O][9] row-major R, world x = R q + t
* scene.trans          float32 [E][O][3]
* model.alpha          float32 [K]
* model.phi            float32 [17411]  packed residual-network weights

Workload recipes follow the paper's setting (Sec. III-A: node-discretised
elastomer surfaces touched by rigid objects; Sec. IV-A: indentation depths of
a few mm on flat and curved elastomers) at the sizes of the benchmark configs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SPHERE, BOX, CAPSULE = 0, 1, 2
MODE_FULL, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY = 0, 1, 2

# Packed residual-network layout (row-major [out][in] weights, then bias),
# widths 9 -> 64 -> 64 | max-pool 64 | 64 -> 64 | [f; g'] 128 -> 64 -> 3.
PHI_LAYERS = (("W1", 64, 9), ("W2", 64, 64), ("W3", 64, 64), ("W4", 64, 128), ("W5", 3, 64))
PHI_SIZE = sum(o * i + o for _, o, i in PHI_LAYERS)
assert PHI_SIZE == 17411


def phi_offsets():
    """Offsets of each weight / bias block inside the packed parameter vector."""
    off, cur = {}, 0
    for name, o, i in PHI_LAYERS:
        off[name] = cur
        cur += o * i
        off["b" + name[1:]] = cur
        cur += o
    return off


@dataclass
class Mesh:
    patch_offset: np.ndarray  # int32 [K+1]
    pos: np.ndarray           # float32 [3][N]
    nrm: np.ndarray           # float32 [3][N]
    origin: np.ndarray        # float32 [K][3]
    pitch: np.ndarray         # float64 [K] (metadata)
    grid: list = field(default_factory=list)   # per patch (nx, ny, curved_radius or 0)

    @property
    def n_patches(self):
        return int(self.patch_offset.shape[0] - 1)

    @property
    def n_nodes(self):
        return int(self.pos.shape[1])

    def patch_sizes(self):
        return np.diff(self.patch_offset).astype(np.int64)


@dataclass
class Scene:
    n_obj: np.ndarray   # int32 [E]
    type: np.ndarray    # int32 [E][O]
    shape: np.ndarray   # float32 [E][O][4]
    rot: np.ndarray     # float32 [E][O][9]
    trans: np.ndarray   # float32 [E][O][3]

    @property
    def n_envs(self):
        return int(self.n_obj.shape[0])

    @property
    def max_obj(self):
        return int(self.type.shape[1])

    def select(self, envs):
        envs = np.asarray(envs)
        return Scene(self.n_obj[envs].copy(), self.type[envs].copy(), self.shape[envs].copy(),
                     self.rot[envs].copy(), self.trans[envs].copy())

    def copy(self):
        return self.select(np.arange(self.n_envs))


@dataclass
class Model:
    mode: int
    alpha: np.ndarray   # float32 [K]
    phi: np.ndarray     # float32 [PHI_SIZE]

    def with_mode(self, mode):
        return Model(int(mode), self.alpha.copy(), self.phi.copy())


# ----------------------------------------------------------------------------
# geometry helpers (FP64, rounded to FP32 once at the end)
# ----------------------------------------------------------------------------

def _grid_patch(nx, ny, pitch, centre, curved_radius=0.0):
    """Nodes of one rectangular patch; index j*nx + i; outward normal +z at the
    centre.  A curved patch is wrapped on a cylinder about its long (x) axis."""
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    u = (i - (nx - 1) / 2.0) * pitch
    v = (j - (ny - 1) / 2.0) * pitch
    U, V = np.meshgrid(u, v)            # [ny][nx] -> flattened j*nx + i
    U, V = U.ravel(), V.ravel()
    if curved_radius > 0.0:
        th = V / curved_radius
        x, y, z = U, curved_radius * np.sin(th), curved_radius * (np.cos(th) - 1.0)
        nxv, nyv, nzv = np.zeros_like(th), np.sin(th), np.cos(th)
    else:
        x, y, z = U, V, np.zeros_like(U)
        nxv, nyv, nzv = np.zeros_like(U), np.zeros_like(U), np.ones_like(U)
    pos = np.stack([x + centre[0], y + centre[1], z + centre[2]])
    nrm = np.stack([nxv, nyv, nzv])
    return pos, nrm


def _assemble_mesh(patches, pitches, centres, grids):
    offs = [0]
    for p, _ in patches:
        offs.append(offs[-1] + p.shape[1])
    pos = np.concatenate([p for p, _ in patches], axis=1)
    nrm = np.concatenate([n for _, n in patches], axis=1)
    return Mesh(np.asarray(offs, dtype=np.int32), pos.astype(np.float32),
                nrm.astype(np.float32), np.asarray(centres, dtype=np.float32),
                np.asarray(pitches, dtype=np.float64), grids)


def random_rotation(rng):
    """Uniform rotation on SO(3) from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def support_extent(ptype, shape, R, u):
    """Largest extent of a primitive from its centre along unit direction u
    (placement geometry only)."""
    if ptype == SPHERE:
        return shape[0]
    if ptype == BOX:
        return sum(shape[c] * abs(float(R[:, c] @ u)) for c in range(3))
    return shape[0] + shape[1] * abs(float(R[:, 2] @ u))


def draw_phi(rng):
    """Residual-network parameters: every weight and bias ~ U(+-1/sqrt(fan_in));
    the output layer (W5, b5) is scaled by 0.02 so residuals stay a few
    hundredths of a mm, the size of correction the paper's ablation implies."""
    parts = []
    for name, o, i in PHI_LAYERS:
        lim = 1.0 / np.sqrt(i)
        W = rng.uniform(-lim, lim, size=(o, i))
        b = rng.uniform(-lim, lim, size=o)
        if name == "W5":
            W, b = W * 0.02, b * 0.02
        parts += [W.ravel(), b]
    phi = np.concatenate(parts).astype(np.float32)
    assert phi.size == PHI_SIZE
    return phi


REG_LAYERS = (("E1", 64, 6), ("e1", 64, 1), ("E2", 64, 64), ("e2", 64, 1), ("E3", 256, 64), ("e3", 256, 1),
              ("A1", 128, 256), ("a1", 128, 1), ("a2", 128, 1), ("a0", 4, 1), ("D1", 128, 256), ("d1", 128, 1),
              ("D2", 8, 128), ("d2", 8, 1))
REG_SIZE = sum(o * i for _, o, i in REG_LAYERS)


def draw_regressor(rng):
    """Real-sensor regressor parameters (packed as REG_LAYERS): every weight
    and bias U(+-1/sqrt(fan_in)) of its layer; a0 (the attention score's
    offset, softmax-invariant) is 0."""
    fan = {"e1": 6, "e2": 64, "e3": 64, "a1": 256, "a2": 128, "d1": 256, "d2": 128}
    parts = []
    for name, o, i in REG_LAYERS:
        n = fan.get(name, i)
        lim = 1.0 / np.sqrt(n)
        if name == "a0":
            parts.append(np.zeros(o * i))
        else:
            parts.append(rng.uniform(-lim, lim, size=o * i))
    reg = np.concatenate(parts).astype(np.float32)
    assert reg.size == REG_SIZE
    return reg


def draw_model(rng, pitches, mode=MODE_FULL):
    """alpha_k = kappa_k / pitch_k with kappa ~ U(1.5, 3)."""
    kappa = rng.uniform(1.5, 3.0, size=len(pitches))
    alpha = (kappa / np.asarray(pitches, dtype=np.float64)).astype(np.float32)
    return Model(mode, alpha, draw_phi(rng))


def _empty_scene(E, O):
    rot = np.zeros((E, O, 9), dtype=np.float32)
    rot[:, :, 0] = rot[:, :, 4] = rot[:, :, 8] = 1.0
    return Scene(np.zeros(E, np.int32), np.zeros((E, O), np.int32),
                 np.zeros((E, O, 4), np.float32), rot, np.zeros((E, O, 3), np.float32))


# ----------------------------------------------------------------------------
# config 1 / 3: one flat 32x32 pad, pitch 0.5 mm, one sphere indenter
# ----------------------------------------------------------------------------

def pad32_mesh():
    pos, nrm = _grid_patch(32, 32, 0.5, (0.0, 0.0, 0.0))
    return _assemble_mesh([(pos, nrm)], [0.5], [(0.0, 0.0, 0.0)], [(32, 32, 0.0)])


def pad_sphere_env(rng, centred=False, radius=5.0, depth=None):
    """Sphere r = 5 mm, centre uniform over the pad interior, pressed
    U(0.2, 1.5) mm deep.  Draw order: x0, y0, depth."""
    x0, y0 = rng.uniform(-7.75, 7.75, size=2)
    d = rng.uniform(0.2, 1.5) if depth is None else depth
    if centred:
        x0 = y0 = 0.0
    return (x0, y0, radius - d), radius


def config1(seed=0, centred=False, mode=MODE_FULL):
    """Single env, single flat 32x32 pad (0.5 mm pitch), one sphere."""
    mesh = pad32_mesh()
    rng = np.random.default_rng(seed)
    scene = _empty_scene(1, 1)
    (x0, y0, z0), r = pad_sphere_env(rng, centred)
    scene.n_obj[0] = 1
    scene.type[0, 0] = SPHERE
    scene.shape[0, 0, 0] = r
    scene.trans[0, 0] = (x0, y0, z0)
    model = draw_model(np.random.default_rng([seed, 1]), mesh.pitch, mode)
    return mesh, scene, model


def config3(seeds=range(8), mode=MODE_FULL, loss_seed=1234, model_seed=None):
    """Config 1 pads for the given seeds (default 0..7) as envs sharing the pad
    and the model (drawn as config 1's for model_seed, default the first
    seed), plus loss weights w ~ N(0,1) of shape [3][E][N]."""
    mesh = pad32_mesh()
    seeds = list(seeds)
    scene = _empty_scene(len(seeds), 1)
    for e, s in enumerate(seeds):
        (x0, y0, z0), r = pad_sphere_env(np.random.default_rng(s))
        scene.n_obj[e] = 1
        scene.type[e, 0] = SPHERE
        scene.shape[e, 0, 0] = r
        scene.trans[e, 0] = (x0, y0, z0)
    model = draw_model(np.random.default_rng([seeds[0] if model_seed is None else model_seed, 1]), mesh.pitch, mode)
    w = np.random.default_rng(loss_seed).standard_normal((3, len(seeds), mesh.n_nodes))
    return mesh, scene, model, w


# ----------------------------------------------------------------------------
# config 2 / 5: a hand of 16 patches of uneven size, 1-3 primitives per env
# ----------------------------------------------------------------------------

HAND_SIZES = (64, 128, 256, 512, 1024)
HAND_GRIDS = {64: (8, 8), 128: (16, 8), 256: (16, 16), 512: (32, 16), 1024: (32, 32)}


def hand_mesh(seed=0, n_patches=16, spacing=45.0, sizes=HAND_SIZES):
    """16 patches, sizes i.i.d. from {64..1024} nodes, 1 mm pitch, half flat and
    half wrapped on a cylinder of radius U(8, 15) mm about the long axis, laid
    out on a 4x4 grid 45 mm apart so that patches never overlap."""
    rng = np.random.default_rng([seed, 7])
    sizes = rng.choice(sizes, size=n_patches)
    curved = np.zeros(n_patches, bool)
    curved[rng.permutation(n_patches)[: n_patches // 2]] = True
    radii = rng.uniform(8.0, 15.0, size=n_patches)
    side = int(np.ceil(np.sqrt(n_patches)))
    patches, centres, grids = [], [], []
    for k in range(n_patches):
        nx, ny = HAND_GRIDS[int(sizes[k])]
        c = ((k % side - (side - 1) / 2.0) * spacing, (k // side - (side - 1) / 2.0) * spacing, 0.0)
        rc = radii[k] if curved[k] else 0.0
        patches.append(_grid_patch(nx, ny, 1.0, c, rc))
        centres.append(c)
        grids.append((nx, ny, float(rc)))
    return _assemble_mesh(patches, [1.0] * n_patches, centres, grids)


def draw_primitive(rng, scale=1.0):
    """Type uniform over sphere (r U(10,40)), box (sides U(20,60)), capsule
    (r U(8,20), length U(30,80)); orientation uniform on SO(3), R = I for a
    sphere.  All lengths are multiplied by `scale`.  Returns (type, shape[4], R)."""
    ptype = int(rng.integers(0, 3))
    shape = np.zeros(4)
    if ptype == SPHERE:
        shape[0] = rng.uniform(10.0, 40.0)
        R = np.eye(3)
    elif ptype == BOX:
        shape[:3] = rng.uniform(20.0, 60.0, size=3) / 2.0
        R = random_rotation(rng)
    else:
        shape[0] = rng.uniform(8.0, 20.0)
        shape[1] = rng.uniform(30.0, 80.0) / 2.0
        R = random_rotation(rng)
    return ptype, shape * scale, R


# Depth of a primitive's extreme point below the touched node, mm (objects
# posed within 10 mm of the patch surface).  With this range the fraction of
# a hand's nodes in contact averages about 7 % (median 6 %, 90th percentile
# 13 %), inside the few-to-30 % band of the benchmark recipe.
HAND_OFFSET = (2.0, 10.0)


def place_primitive(rng, mesh, ptype, shape, R, offset=HAND_OFFSET):
    """Pick a node p* uniformly (so patches are weighted by node count) and put
    the primitive's extreme point in the approach direction -z (all patches
    face +z) at signed depth s below p*."""
    node = int(rng.integers(0, mesh.n_nodes))
    p = mesh.pos[:, node].astype(np.float64)
    n = np.array([0.0, 0.0, 1.0])
    s = rng.uniform(*offset)
    h = support_extent(ptype, shape, R, n)
    return p + (h - s) * n


# Footprint placement: the env's objects together cover a drawn fraction of
# its nodes.  FOOT_GOAL is the range of that fraction; an object covers at
# most FOOT_CAP of its patch, and its node is drawn inside the patch inset by
# FOOT_INSET of the patch's half-extent on each side.
FOOT_GOAL = (0.08, 0.24)
FOOT_CAP = 0.85
FOOT_INSET = 0.35
# a curved patch bends away from a flat footprint: its area target is
# enlarged by this factor
FOOT_CURVED = 1.6


def _frame(n, rng):
    """Orthonormal tangent vectors (t1, t2) of unit normal n, rotated by a
    uniform in-plane angle."""
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = np.cross(n, a)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    return np.cos(phi) * t1 + np.sin(phi) * t2, -np.sin(phi) * t1 + np.cos(phi) * t2


def _tilt(R, n, rng, max_deg=2.0):
    """R rotated about a random tangent axis by up to max_deg degrees."""
    t1, _ = _frame(n, rng)
    return _rodrigues_batch(t1 * np.deg2rad(rng.uniform(-max_deg, max_deg)))[...] @ R


def footprint_primitive(rng, n, area, scale=1.0, span=np.inf):
    """A primitive, its rotation and its press depth along -n such that the
    part below the tangent plane has the given cross-section area (mm^2), by
    the closed forms of its shape (the patch's curvature is ignored):
    sphere (r U(10, 40)) pressed d deep: pi (2 r d - d^2); capsule (r U(8, 20),
    length U(30, 80)) with its axis in the tangent plane: a stadium of half
    width w = sqrt(2 r d - d^2), 4 w L + pi w^2 with L at most `span` / 2 (the
    part of the stadium over the patch); box with a face on the tangent
    plane: the face, whose sides are set to the area (the third side
    U(20, 60)), pressed U(1, 3) mm.  Boxes and capsules get a uniform in-plane
    rotation and a tilt of up to 2 degrees about their centre.  Returns (type,
    shape[4], R, depth, ext): ext is the untilted extent of the object from
    its centre towards the surface, so the centre goes ext - depth above the
    pressed node along its normal."""
    ptype = int(rng.integers(0, 3))
    shape = np.zeros(4)
    if ptype == SPHERE:
        r = rng.uniform(10.0, 40.0) * scale
        r = max(r, np.sqrt(area / (0.8 * np.pi)))          # the disc must be able to reach the area
        d = r - np.sqrt(max(r * r - area / np.pi, 0.0))
        shape[0] = r
        return ptype, shape, np.eye(3), d, r
    t1, t2 = _frame(n, rng)
    if ptype == CAPSULE:
        r = rng.uniform(8.0, 20.0) * scale
        L = rng.uniform(30.0, 80.0) / 2.0 * scale
        Le = min(L, 0.5 * span)
        # 4 w Le + pi w^2 = area  ->  w
        w = (-4.0 * Le + np.sqrt(16.0 * Le * Le + 4.0 * np.pi * area)) / (2.0 * np.pi)
        w = min(w, 0.95 * r)
        d = r - np.sqrt(r * r - w * w)
        shape[0], shape[1] = r, L
        R = np.stack([t2, n, t1], axis=1)      # object z (the axis) along t1
        return ptype, shape, _tilt(R, n, rng), d, r
    a = np.sqrt(area) * np.exp(rng.uniform(-0.3, 0.3))   # face sides a x area / a
    b = area / a
    shape[0], shape[1], shape[2] = a / 2.0, b / 2.0, rng.uniform(20.0, 60.0) / 2.0 * scale
    R = np.stack([t1, t2, n], axis=1)          # object z along the normal: face on the tangent plane
    return ptype, shape, _tilt(R, n, rng), rng.uniform(1.0, 3.0) * scale, shape[2]


def _footprint_env(rng, mesh, cnt, scale):
    """Objects of one env placed by footprint (see FOOT_GOAL)."""
    sizes = mesh.patch_sizes().astype(np.float64)
    pitch = mesh.pitch
    goal = rng.uniform(*FOOT_GOAL) * mesh.n_nodes
    share = goal / cnt
    fits = np.nonzero(FOOT_CAP * sizes >= share)[0]
    if fits.size < cnt:                    # not enough patches that hold the share: the largest ones
        fits = np.argsort(-sizes)[:max(cnt, fits.size)]
    w = sizes[fits] / sizes[fits].sum()
    patches = rng.choice(fits, size=cnt, replace=False, p=w)
    out = []
    for k in patches:
        k = int(k)
        nodes = min(share, FOOT_CAP * sizes[k])
        nx, ny, rc = mesh.grid[k]
        area = nodes * pitch[k] ** 2 * (FOOT_CURVED if rc > 0 else 1.0)
        i = int(np.clip(np.round(rng.uniform(FOOT_INSET, 1.0 - FOOT_INSET) * (nx - 1)), 0, nx - 1))
        j = int(np.clip(np.round(rng.uniform(FOOT_INSET, 1.0 - FOOT_INSET) * (ny - 1)), 0, ny - 1))
        node = int(mesh.patch_offset[k]) + j * nx + i
        p = mesh.pos[:, node].astype(np.float64)
        n = mesh.nrm[:, node].astype(np.float64)
        n /= np.linalg.norm(n)
        ptype, shape, R, d, ext = footprint_primitive(rng, n, area, scale, span=min(nx, ny) * pitch[k])
        out.append((ptype, shape, R, p + (ext - d) * n))
    return out


def hand_scene(mesh, n_envs, seed=1, max_obj=3, offset=HAND_OFFSET, scale=1.0, placement="footprint"):
    """Per env: object count U{1,2,3}, then per object type/shape/rotation and
    placement.  Env e draws from its own stream (seed, e) so that any subset
    of envs can be regenerated alone.  placement "footprint" (the benchmark
    hand): the objects cover FOOT_GOAL of the env's nodes together, each
    pressed along the normal of a node of its own patch (footprint_primitive);
    "press": each object's extreme point `offset` mm below a uniformly drawn
    node in the approach direction -z, orientation uniform on SO(3).  `scale`
    shrinks objects and press depths together (small-patch hands)."""
    scene = _empty_scene(n_envs, max_obj)
    for e in range(n_envs):
        rng = np.random.default_rng([seed, e])
        cnt = int(rng.integers(1, max_obj + 1))
        scene.n_obj[e] = cnt
        if placement == "footprint":
            objs = _footprint_env(rng, mesh, cnt, scale)
        else:
            objs = []
            for o in range(cnt):
                ptype, shape, R = draw_primitive(rng, scale)
                t = place_primitive(rng, mesh, ptype, shape, R, (offset[0] * scale, offset[1] * scale))
                objs.append((ptype, shape, R, t))
        for o, (ptype, shape, R, t) in enumerate(objs):
            scene.type[e, o] = ptype
            scene.shape[e, o] = shape
            scene.rot[e, o] = R.ravel()
            scene.trans[e, o] = t
    return scene


def config2(n_envs=4096, hand_seed=0, env_seed=1, mode=MODE_FULL, sizes=HAND_SIZES, scale=1.0,
            placement="footprint"):
    """Batched forward: n_envs envs of a 16-patch hand with 1-3 primitives,
    placed by footprint (the benchmark's contact band) or by press depth.
    `sizes` narrows the patch-size draw (small-patch hands for the gradient
    checks)."""
    mesh = hand_mesh(hand_seed, sizes=sizes)
    scene = hand_scene(mesh, n_envs, env_seed, scale=scale, placement=placement)
    model = draw_model(np.random.default_rng([hand_seed, 1]), mesh.pitch, mode)
    return mesh, scene, model


# ----------------------------------------------------------------------------
# config 4: 4 flat 128x128 pads at 0.125 mm pitch, one object per pad
# ----------------------------------------------------------------------------

def hires_mesh(n=128, pitch=0.125, spacing=24.0):
    patches, centres, grids = [], [], []
    for k in range(4):
        c = ((k % 2 - 0.5) * spacing, (k // 2 - 0.5) * spacing, 0.0)
        patches.append(_grid_patch(n, n, pitch, c))
        centres.append(c)
        grids.append((n, n, 0.0))
    return _assemble_mesh(patches, [pitch] * 4, centres, grids)


def hires_scene(mesh, n_envs, seed=3):
    """One sphere (r U(3,8)) or box (sides U(4,12), SO(3)-uniform) per pad,
    pressed U(0.1, 2) mm deep at a point uniform over the pad inset 2 mm."""
    K = mesh.n_patches
    scene = _empty_scene(n_envs, K)
    for e in range(n_envs):
        rng = np.random.default_rng([seed, e])
        scene.n_obj[e] = K
        for k in range(K):
            o0, o1 = mesh.patch_offset[k], mesh.patch_offset[k + 1]
            lo = mesh.pos[:2, o0:o1].min(axis=1).astype(np.float64) + 2.0
            hi = mesh.pos[:2, o0:o1].max(axis=1).astype(np.float64) - 2.0
            xy = rng.uniform(lo, hi)
            depth = rng.uniform(0.1, 2.0)
            if rng.uniform() < 0.5:
                ptype, shape, R = SPHERE, np.array([rng.uniform(3.0, 8.0), 0, 0, 0]), np.eye(3)
            else:
                shape = np.zeros(4)
                shape[:3] = rng.uniform(4.0, 12.0, size=3) / 2.0
                ptype, R = BOX, random_rotation(rng)
            n = np.array([0.0, 0.0, 1.0])
            h = support_extent(ptype, shape, R, n)
            t = np.array([xy[0], xy[1], 0.0]) + (h - depth) * n
            scene.type[e, k] = ptype
            scene.shape[e, k] = shape
            scene.rot[e, k] = R.ravel()
            scene.trans[e, k] = t
    return scene


def config4(n_envs=4096, seed=3, mode=MODE_FULL):
    mesh = hires_mesh()
    scene = hires_scene(mesh, n_envs, seed)
    model = draw_model(np.random.default_rng([seed, 1]), mesh.pitch, mode)
    return mesh, scene, model


# ----------------------------------------------------------------------------
# config 5: smooth random trajectories of the config-2 objects
# ----------------------------------------------------------------------------

def _rodrigues_batch(w):
    """exp([w]_x) for w [..., 3] (Rodrigues' formula, FP64)."""
    th = np.linalg.norm(w, axis=-1)[..., None, None]
    safe = np.where(th > 1e-15, th, 1.0)
    k = w / safe[..., 0]
    z = np.zeros_like(k[..., 0])
    K = np.stack([z, -k[..., 2], k[..., 1], k[..., 2], z, -k[..., 0], -k[..., 1], k[..., 0], z],
                 axis=-1).reshape(*w.shape[:-1], 3, 3)
    eye = np.broadcast_to(np.eye(3), K.shape)
    R = eye + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)
    return np.where(th > 1e-15, R, eye)


def trajectory(scene, n_steps, seed=5, v_std=5.0, w_std=0.05, rho=0.9, box=10.0):
    """Smooth random object motion for a graph-captured rollout.

    Per object: AR(1) translational velocity (stationary std v_std mm/step)
    and angular velocity (std w_std rad/step); the displacement from the
    initial pose is reflected to stay within +-box mm per axis.  Spheres keep
    R = I.  Returns rot [T][E][O][9] and trans [T][E][O][3] in FP32."""
    E, O = scene.type.shape
    rng = np.random.default_rng(seed)
    sig = np.sqrt(1.0 - rho * rho)
    t0 = scene.trans.astype(np.float64)
    R = scene.rot.astype(np.float64).reshape(E, O, 3, 3).copy()
    spin = (scene.type != SPHERE)[..., None]
    off = np.zeros((E, O, 3))
    v = rng.normal(0.0, v_std, size=(E, O, 3))
    w = rng.normal(0.0, w_std, size=(E, O, 3))
    rots = np.empty((n_steps, E, O, 9), np.float32)
    trans = np.empty((n_steps, E, O, 3), np.float32)
    for s in range(n_steps):
        rots[s] = R.reshape(E, O, 9)
        trans[s] = t0 + off
        v = rho * v + sig * rng.normal(0.0, v_std, size=v.shape)
        w = rho * w + sig * rng.normal(0.0, w_std, size=w.shape)
        off = off + v
        over = off > box
        off[over] = 2 * box - off[over]
        v[over] = -v[over]
        under = off < -box
        off[under] = -2 * box - off[under]
        v[under] = -v[under]
        R = np.where(spin[..., None], _rodrigues_batch(w) @ R, R)
    return rots, trans
