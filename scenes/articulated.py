"""Synthetic articulated hand: links, their collision primitives, sensor
patches in link frames, link poses from joint angles, and grasp scenes.

Input generation only (seeded, synthetic): nothing here evaluates contact,
propagation or rewards.  The layout follows a five-finger hand of the kind the
paper's RL experiments use (palm plus three phalanges per finger, tactile
skin on the palmar side of every link, Sec. IV-B); sizes are stand-ins.

Frames.  Every link frame has y along the bone (towards the fingertip) and z
along the palmar normal (the side that grasps); x = y cross z.  The palm frame
sits at the palm centre.  A phalanx frame sits on its proximal joint; its
capsule runs from y = 0 to y = 2 l (half length l, radius r).  Flexion turns
a child about its joint's x axis, moving its y axis towards +z.  Poses map a
link-frame point q to world x = R q + t.

Patches.  Node positions, normals and origins of patch k are given in the
frame of the link that carries it (`patch_link[k]`), on that link's own
collision surface: a flat grid on the palm's palmar face, and grids wrapped on
the palmar half of each phalanx capsule.
"""
from dataclasses import dataclass

import numpy as np

from . import BOX, CAPSULE, SPHERE, Mesh, Scene, _empty_scene, draw_model, draw_primitive, support_extent

NONE = -1   # a link without a collision primitive

PALM_HALF = (42.0, 45.0, 12.0)            # palm box half extents (x, y, z)
# per finger (thumb, index, middle, ring, little): phalanx lengths 2 l and radius
FINGER_LEN = ((40.0, 30.0, 24.0), (44.0, 26.0, 20.0), (46.0, 28.0, 22.0), (42.0, 26.0, 20.0), (34.0, 20.0, 18.0))
FINGER_RADIUS = (10.0, 9.0, 9.5, 9.0, 8.0)
FINGER_BASE_X = (None, -27.0, -9.0, 9.0, 27.0)
# patch grids: (nodes along the bone, nodes around it, pitch)
PALM_GRID = (32, 32, 2.5)
PHALANX_GRID = ((32, 16, 1.25), (16, 16, 1.25), (16, 8, 1.0))


@dataclass
class Hand:
    n_links: int
    parent: np.ndarray       # int32 [L], -1 for the palm
    patch_link: np.ndarray   # int32 [K]
    collide: np.ndarray      # uint32 [L] bit j: link j's primitive is tested against patches on link l
    prim_type: np.ndarray    # int32 [L]
    prim_shape: np.ndarray   # float32 [L][4]
    prim_rot: np.ndarray     # float32 [L][9] primitive pose in its link frame
    prim_trans: np.ndarray   # float32 [L][3]
    # kinematics (scene generation only)
    joint_offset: np.ndarray  # float64 [L][3] joint position in the parent frame
    base_rot: np.ndarray      # float64 [L][3][3] fixed rotation of the joint frame in the parent frame


def _rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _ry(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# capsule axis (object z) along the link's y axis: columns are the capsule's
# x, y, z axes in the link frame
_CAPSULE_IN_LINK = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0]])


def _flat_patch(nx, ny, pitch, z):
    i = (np.arange(nx) - (nx - 1) / 2.0) * pitch
    j = (np.arange(ny) - (ny - 1) / 2.0) * pitch
    U, V = np.meshgrid(i, j)
    pos = np.stack([U.ravel(), V.ravel(), np.full(U.size, z)])
    nrm = np.stack([np.zeros(U.size), np.zeros(U.size), np.ones(U.size)])
    return pos, nrm


def _wrapped_patch(n_along, n_around, pitch, radius, y_mid):
    """Grid on the cylinder of `radius` about the link's y axis, centred on
    the palmar direction +z at y = y_mid."""
    u = (np.arange(n_along) - (n_along - 1) / 2.0) * pitch + y_mid
    th = (np.arange(n_around) - (n_around - 1) / 2.0) * pitch / radius
    Y, T = np.meshgrid(u, th)          # node index: around-major, along-minor
    Y, T = Y.ravel(), T.ravel()
    pos = np.stack([radius * np.sin(T), Y, radius * np.cos(T)])
    nrm = np.stack([np.sin(T), np.zeros_like(T), np.cos(T)])
    return pos, nrm


def hand(adjacent_only=True):
    """The 16-link hand (palm, then thumb, index, middle, ring, little with
    three phalanges each) and its 16 patches (one per link).

    collide[l] holds every link except l itself, its parent and its children
    (joint neighbours overlap by construction); with adjacent_only=False it
    also drops the other phalanges of the same finger."""
    L = 16
    parent = np.full(L, -1, np.int32)
    prim_type = np.full(L, NONE, np.int32)
    prim_shape = np.zeros((L, 4))
    prim_rot = np.tile(np.eye(3), (L, 1, 1))
    prim_trans = np.zeros((L, 3))
    joint_offset = np.zeros((L, 3))
    base_rot = np.tile(np.eye(3), (L, 1, 1))
    prim_type[0] = BOX
    prim_shape[0, :3] = PALM_HALF
    patches = [_flat_patch(PALM_GRID[0], PALM_GRID[1], PALM_GRID[2], PALM_HALF[2])]
    pitches = [PALM_GRID[2]]
    origins = [np.array([0.0, 0.0, PALM_HALF[2]])]
    grids = [(PALM_GRID[0], PALM_GRID[1], 0.0)]
    for f in range(5):
        r = FINGER_RADIUS[f]
        for s in range(3):
            l = 1 + 3 * f + s
            parent[l] = 0 if s == 0 else l - 1
            half = FINGER_LEN[f][s] / 2.0
            prim_type[l] = CAPSULE
            prim_shape[l, :2] = (r, half)
            prim_rot[l] = _CAPSULE_IN_LINK
            prim_trans[l] = (0.0, half, 0.0)
            if s == 0:
                if f == 0:   # thumb: on the palm's radial side, turned towards the palm centre
                    joint_offset[l] = (-PALM_HALF[0] + 6.0, -8.0, 2.0)
                    base_rot[l] = _rz(np.deg2rad(55.0)) @ _ry(np.deg2rad(-35.0))
                else:
                    joint_offset[l] = (FINGER_BASE_X[f], PALM_HALF[1], 0.0)
            else:
                joint_offset[l] = (0.0, FINGER_LEN[f][s - 1], 0.0)
            na, nb, pitch = PHALANX_GRID[s]
            patches.append(_wrapped_patch(na, nb, pitch, r, half))
            pitches.append(pitch)
            origins.append(np.array([0.0, half, r]))
            grids.append((na, nb, r))
    collide = np.zeros(L, np.uint32)
    for l in range(L):
        bits = 0
        for j in range(L):
            if j == l or parent[j] == l or parent[l] == j or prim_type[j] == NONE:
                continue
            if not adjacent_only and l > 0 and j > 0 and (l - 1) // 3 == (j - 1) // 3:
                continue
            bits |= 1 << j
        collide[l] = bits
    offs = [0]
    for p, _ in patches:
        offs.append(offs[-1] + p.shape[1])
    mesh = Mesh(np.asarray(offs, np.int32), np.concatenate([p for p, _ in patches], axis=1).astype(np.float32),
                np.concatenate([n for _, n in patches], axis=1).astype(np.float32),
                np.asarray(origins, np.float32), np.asarray(pitches, np.float64), grids)
    h = Hand(L, parent, np.arange(L, dtype=np.int32), collide, prim_type, prim_shape.astype(np.float32),
             prim_rot.reshape(L, 9).astype(np.float32), prim_trans.astype(np.float32), joint_offset, base_rot)
    return h, mesh


@dataclass
class Links:
    rot: np.ndarray     # float32 [E][L][9]
    trans: np.ndarray   # float32 [E][L][3]

    def select(self, envs):
        envs = np.asarray(envs)
        return Links(self.rot[envs].copy(), self.trans[envs].copy())


def forward_kinematics(h, angles, root_R, root_t):
    """Link poses of one env from joint angles [L][2] (flexion, abduction;
    the palm's entry is unused) and the palm's world pose.  FP64."""
    L = h.n_links
    R = np.zeros((L, 3, 3))
    t = np.zeros((L, 3))
    R[0], t[0] = root_R, root_t
    for l in range(1, L):
        p = h.parent[l]
        local = h.base_rot[l] @ _rz(angles[l, 1]) @ _rx(angles[l, 0])
        R[l] = R[p] @ local
        t[l] = R[p] @ h.joint_offset[l] + t[p]
    return R, t


def draw_angles(rng, h, curl=(0.0, 1.0)):
    """Flexion U(0, c * limit) per joint with one curl factor c ~ U(curl) per
    finger (MCP 85, PIP 100, DIP 75 degrees; thumb 60, 70, 70), abduction
    U(-12, 12) degrees on the first joint of each finger."""
    a = np.zeros((h.n_links, 2))
    lim = np.deg2rad([[85.0, 100.0, 75.0]] * 4)
    lim_t = np.deg2rad([60.0, 70.0, 70.0])
    for f in range(5):
        c = rng.uniform(*curl)
        for s in range(3):
            l = 1 + 3 * f + s
            top = lim_t[s] if f == 0 else lim[f - 1][s]
            a[l, 0] = c * top * rng.uniform(0.7, 1.0)
        a[1 + 3 * f, 1] = np.deg2rad(rng.uniform(-12.0, 12.0))
    return a


def _extent_along(ptype, shape, R, u):
    """support_extent for an array of unit directions u [n][3]."""
    if ptype == SPHERE:
        return np.full(u.shape[0], float(shape[0]))
    if ptype == BOX:
        return sum(float(shape[c]) * np.abs(u @ R[:, c]) for c in range(3))
    return float(shape[0]) + float(shape[1]) * np.abs(u @ R[:, 2])


def _finger_chain(h, f, flex, abd, R0, t0):
    """World poses of finger f's three links for a batch of flexion triples
    flex [n][3] (placement only; same composition as forward_kinematics)."""
    n = flex.shape[0]
    Rs, ts = [], []
    Rp = np.broadcast_to(R0, (n, 3, 3))
    tp = np.broadcast_to(t0, (n, 3))
    for s in range(3):
        l = 1 + 3 * f + s
        c, sn = np.cos(flex[:, s]), np.sin(flex[:, s])
        Rx = np.zeros((n, 3, 3))
        Rx[:, 0, 0] = 1.0
        Rx[:, 1, 1], Rx[:, 1, 2], Rx[:, 2, 1], Rx[:, 2, 2] = c, -sn, sn, c
        local = (h.base_rot[l] @ _rz(abd if s == 0 else 0.0)) @ Rx
        t = np.einsum("nab,b->na", Rp, h.joint_offset[l]) + tp
        R = Rp @ local
        Rs.append(R)
        ts.append(t)
        Rp, tp = R, t
    return Rs, ts


def _finger_gaps(h, f, Rs, ts, centre, ptype, shape, Ro):
    """Smallest clearance between finger f's capsules and the object for each
    pose of the batch, the object's extent taken along the direction to the
    closest point of each capsule axis."""
    gap = np.full(Rs[0].shape[0], np.inf)
    for s in range(3):
        l = 1 + 3 * f + s
        r, half = float(h.prim_shape[l, 0]), float(h.prim_shape[l, 1])
        a = ts[s]
        b = a + 2.0 * half * Rs[s][:, :, 1]
        ab = b - a
        tt = np.clip(np.einsum("na,na->n", centre - a, ab) / np.einsum("na,na->n", ab, ab), 0.0, 1.0)
        d = a + tt[:, None] * ab - centre
        dist = np.linalg.norm(d, axis=1)
        u = d / np.maximum(dist, 1e-12)[:, None]
        gap = np.minimum(gap, dist - r - _extent_along(ptype, shape, Ro, u))
    return gap


def grasp_scene(h, mesh, n_envs, seed=11, max_obj=2, scale=0.8, press=(1.0, 4.0), steps=40):
    """Per env: palm pose uniform on SO(3) about a point within 50 mm of the
    origin; 1..max_obj primitives (sizes scale x draw_primitive's) pressed
    press mm into the palm's face at a point with |x| <= 18, 0 <= y <= 30 of
    the palm frame; then every finger closes (one curl factor scaling its
    three flexion limits, with a fixed jitter per joint, raised in `steps`
    steps) until one of its capsules is press mm into the first object, by
    capsule-axis distance and the object's extent along that direction, or
    its joints reach their limits.  Abduction U(-12, 12) degrees.  Placement
    geometry only; contact itself is never evaluated here.  Returns (Scene,
    Links)."""
    from . import random_rotation
    rng = np.random.default_rng([seed, 23])
    L = h.n_links
    scene = _empty_scene(n_envs, max_obj)
    rot = np.zeros((n_envs, L, 9), np.float32)
    trans = np.zeros((n_envs, L, 3), np.float32)
    lim = np.deg2rad([[60.0, 70.0, 70.0]] + [[85.0, 100.0, 75.0]] * 4)
    for e in range(n_envs):
        R0 = random_rotation(rng)
        t0 = rng.uniform(-50.0, 50.0, size=3)
        zp = R0[:, 2]
        cnt = int(rng.integers(1, max_obj + 1))
        scene.n_obj[e] = cnt
        objs = []
        for o in range(cnt):
            ptype, shape, Ro = draw_primitive(rng, scale)
            ext = support_extent(ptype, shape, Ro, zp)
            anchor = np.array([rng.uniform(-18.0, 18.0), rng.uniform(0.0, 30.0), PALM_HALF[2]])
            c = R0 @ anchor + t0 + (ext - rng.uniform(*press)) * zp
            scene.type[e, o] = ptype
            scene.shape[e, o] = shape
            scene.rot[e, o] = Ro.reshape(9)
            scene.trans[e, o] = c
            objs.append((ptype, shape, Ro, c))
        angles = np.zeros((L, 2))
        jitter = rng.uniform(0.7, 1.0, size=(5, 3))
        abd = np.deg2rad(rng.uniform(-12.0, 12.0, size=5))
        goal = rng.uniform(*press, size=5)
        ptype, shape, Ro, c = objs[0]
        frac = np.arange(steps + 1) / steps
        for f in range(5):
            flex = frac[:, None] * (lim[f] * jitter[f])[None, :]
            Rs, ts = _finger_chain(h, f, flex, abd[f], R0, t0)
            hit = np.nonzero(_finger_gaps(h, f, Rs, ts, c, ptype, shape, Ro) <= -goal[f])[0]
            i = int(hit[0]) if hit.size else steps
            angles[1 + 3 * f: 4 + 3 * f, 0] = flex[i]
            angles[1 + 3 * f, 1] = abd[f]
        R, t = forward_kinematics(h, angles, R0, t0)
        rot[e] = R.reshape(L, 9)
        trans[e] = t
    return scene, Links(rot, trans)


def config_hand(n_envs=4096, seed=11, mode=0, adjacent_only=True):
    """Articulated-hand workload: the 16-link hand, grasp scenes, a model with
    alpha_k = kappa_k / pitch_k.  Returns (hand, mesh, scene, links, model)."""
    h, mesh = hand(adjacent_only)
    scene, links = grasp_scene(h, mesh, n_envs, seed)
    model = draw_model(np.random.default_rng([seed, 29]), mesh.pitch, mode)
    return h, mesh, scene, links, model


def identity_links(h, n_envs):
    """Every link at the world origin with R = I (the hand step then sees the
    objects as the plain step does)."""
    rot = np.zeros((n_envs, h.n_links, 9), np.float32)
    rot[:, :, 0] = rot[:, :, 4] = rot[:, :, 8] = 1.0
    return Links(rot, np.zeros((n_envs, h.n_links, 3), np.float32))


__all__ = ["Hand", "Links", "hand", "forward_kinematics", "draw_angles", "grasp_scene", "config_hand",
           "identity_links", "NONE", "SPHERE", "BOX", "CAPSULE"]
