"""FP64 CPU oracle of the ETac tactile step (ctypes wrapper around etac_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports it.

Every function takes the same FP32 input arrays the GPU library receives (see
the ``scenes`` module for layouts), promotes them exactly to FP64 and returns
FP64 results.  Parity status of each function is recorded in the test files
that pin it (tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "etac_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PHI_SIZE = 17411


def build(force=True):
    """Compile the oracle with gcc: FP64, SSE2 doubles, no FMA contraction, no
    fast-math, OpenMP over environments."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-msse2", "-mfpmath=sse", "-Wall", "-Wno-unknown-pragmas",
           SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads():
    return int(_load().oracle_num_threads())


def set_num_threads(n):
    """Threads of the oracle's parallel loops from here on."""
    _load().oracle_set_num_threads(C.c_int(int(n)))


def _mesh_args(mesh):
    return (C.c_int(mesh.n_patches), C.c_int(mesh.n_nodes), _i32(mesh.patch_offset),
            _f64(mesh.pos), _f64(mesh.nrm), _f64(mesh.origin))


def _scene_args(scene):
    return (C.c_int(scene.n_envs), C.c_int(scene.max_obj), _i32(scene.n_obj), _i32(scene.type),
            _f64(scene.shape), _f64(scene.rot), _f64(scene.trans))


def _call(fn, *args):
    conv = [(_p(a) if isinstance(a, np.ndarray) else a) for a in args]
    rc = fn(*conv)
    if rc != 0:
        raise RuntimeError(f"oracle call failed with {rc}")


def contact(mesh, scene):
    """Contact pass.  Returns contact_obj int8 [E][N], uhat f64 [3][E][N],
    n_active int32 [E][K]."""
    lib = _load()
    K, N, off, pos, nrm, _ = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    cobj = np.empty((E.value, N.value), np.int8)
    uhat = np.empty((3, E.value, N.value), np.float64)
    na = np.empty((E.value, K.value), np.int32)
    _call(lib.oracle_contact, K, N, off, pos, nrm, E, O, n_obj, typ, shape, rot, trans, cobj, uhat, na)
    return cobj, uhat, na


def propagate(mesh, model, contact_obj, uhat, mode=None):
    """Eqs. 1-2 on given contact results.  uhat may be FP32 or FP64."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    cobj = np.ascontiguousarray(contact_obj, dtype=np.int8)
    E = cobj.shape[0]
    U = np.empty((3, E, N.value), np.float64)
    m = model.mode if mode is None else mode
    _call(lib.oracle_propagate, K, N, off, pos, nrm, origin, C.c_int(E), C.c_int(m),
          _f64(model.alpha), _f64(model.phi), cobj, _f64(uhat), U)
    return U


def forward(mesh, scene, model, with_sig=False):
    """Whole step.  Returns dict(u, contact_obj, uhat, n_active[, sig, margin])."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    e, n = E.value, N.value
    U = np.empty((3, e, n), np.float64)
    cobj = np.empty((e, n), np.int8)
    uhat = np.empty((3, e, n), np.float64)
    na = np.empty((e, K.value), np.int32)
    sig = np.empty(e, np.uint64) if with_sig else None
    margin = np.empty(e, np.float64) if with_sig else None
    _call(lib.oracle_forward, K, N, off, pos, nrm, origin, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(model.mode), _f64(model.alpha), _f64(model.phi), U, cobj, uhat, na,
          sig if sig is not None else None, margin if margin is not None else None)
    out = dict(u=U, contact_obj=cobj, uhat=uhat, n_active=na)
    if with_sig:
        out.update(sig=sig, margin=margin)
    return out


def item_margins(mesh, scene, model):
    """Decision margin of every (env, patch) item [E][K]: the smallest distance
    of a ReLU input or max-pool runner-up gap from its decision boundary
    (inf for items that evaluate no network), and the forward's outputs."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    e, n = E.value, N.value
    U = np.empty((3, e, n), np.float64)
    cobj = np.empty((e, n), np.int8)
    uhat = np.empty((3, e, n), np.float64)
    na = np.empty((e, K.value), np.int32)
    margin = np.empty((e, K.value), np.float64)
    _call(lib.oracle_item_margins, K, N, off, pos, nrm, origin, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(model.mode), _f64(model.alpha), _f64(model.phi), U, cobj, uhat, na, margin)
    return dict(u=U, contact_obj=cobj, uhat=uhat, n_active=na, margin=margin)


def propagate_backward(mesh, model, contact_obj, uhat, grad_u):
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    cobj = np.ascontiguousarray(contact_obj, dtype=np.int8)
    E = cobj.shape[0]
    guhat = np.empty((3, E, N.value), np.float64)
    ga = np.empty(K.value, np.float64)
    gp = np.empty(PHI_SIZE, np.float64)
    _call(lib.oracle_propagate_backward, K, N, off, pos, nrm, origin, C.c_int(E), C.c_int(model.mode),
          _f64(model.alpha), _f64(model.phi), cobj, _f64(uhat), _f64(grad_u), guhat, ga, gp)
    return dict(grad_uhat=guhat, grad_alpha=ga, grad_phi=gp)


def contact_backward(mesh, scene, grad_uhat):
    lib = _load()
    K, N, off, pos, nrm, _ = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    grot = np.empty((E.value, O.value, 9), np.float64)
    gt = np.empty((E.value, O.value, 3), np.float64)
    _call(lib.oracle_contact_backward, K, N, off, pos, nrm, E, O, n_obj, typ, shape, rot, trans,
          _f64(grad_uhat), grot, gt)
    return dict(grad_rot=grot, grad_trans=gt)


def backward(mesh, scene, model, grad_u):
    """Adjoint of L = sum(grad_u * U) w.r.t. rot, trans, alpha, phi (and the
    intermediate dL/du_hat)."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    grot = np.empty((E.value, O.value, 9), np.float64)
    gt = np.empty((E.value, O.value, 3), np.float64)
    ga = np.empty(K.value, np.float64)
    gp = np.empty(PHI_SIZE, np.float64)
    guhat = np.empty((3, E.value, N.value), np.float64)
    _call(lib.oracle_backward, K, N, off, pos, nrm, origin, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(model.mode), _f64(model.alpha), _f64(model.phi), _f64(grad_u), grot, gt, ga, gp, guhat)
    return dict(grad_rot=grot, grad_trans=gt, grad_alpha=ga, grad_phi=gp, grad_uhat=guhat)


# ----------------------------------------------------------------------------
# central finite differences on the FP64 oracle
# ----------------------------------------------------------------------------

class _F64Scene:
    """FP64 copy of a scene so that FD perturbations are not rounded to FP32."""

    def __init__(self, s):
        self.n_obj = s.n_obj.copy()
        self.type = s.type.copy()
        self.shape = s.shape.astype(np.float64)
        self.rot = s.rot.astype(np.float64)
        self.trans = s.trans.astype(np.float64)

    n_envs = property(lambda self: int(self.n_obj.shape[0]))
    max_obj = property(lambda self: int(self.type.shape[1]))


class _F64Model:
    def __init__(self, m):
        self.mode = m.mode
        self.alpha = m.alpha.astype(np.float64)
        self.phi = m.phi.astype(np.float64)


def skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]], dtype=np.float64)


def expm_so3(w):
    """Rodrigues' formula for exp([w]_x)."""
    th = np.linalg.norm(w)
    if th == 0.0:
        return np.eye(3)
    K = skew(w / th)
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def loss_and_sig(mesh, scene, model, w):
    out = forward(mesh, scene, model, with_sig=True)
    return float(np.sum(out["u"] * w)), out["sig"]


def fd_gradients(mesh, scene, model, w, env=0, obj=0, h=1e-4, phi_idx=(), shrink=(1e-5, 1e-6)):
    """Central differences (L(theta+h) - L(theta-h)) / 2h of L = sum(w * U) in
    FP64 for: the 3 translations and 3 twist components (R' = exp([+-h e_k]_x) R)
    of object `obj` in env `env`, alpha of every patch, and the listed phi
    entries.

    The model is only piecewise smooth: a difference whose two sides take a
    different discrete decision (active set, winner, face, clamp, ReLU
    pattern, arg-max) is not a derivative.  Such a difference is retaken with
    the smaller steps in `shrink`; if every step straddles a decision the
    result is flagged.  Returns (dict of FD values, ok) where ok is False if
    any entry stayed flagged; the dict's "ok_each" holds the flag of every
    entry (same keys and shapes)."""
    S = _F64Scene(scene)
    M = _F64Model(model)
    ok = True
    res = {}
    flags = []

    def central(perturb):
        nonlocal ok
        for step in (h,) + tuple(shrink):
            Sp, Mp = _F64Scene(S), _F64Model(M)
            Sm, Mm = _F64Scene(S), _F64Model(M)
            perturb(Sp, Mp, step)
            perturb(Sm, Mm, -step)
            lp, sp = loss_and_sig(mesh, Sp, Mp, w)
            lm, sm = loss_and_sig(mesh, Sm, Mm, w)
            if np.array_equal(sp, sm):
                flags.append(True)
                return (lp - lm) / (2 * step)
        ok = False
        flags.append(False)
        return (lp - lm) / (2 * step)

    def shift_t(c):
        def f(S_, M_, s):
            S_.trans[env, obj, c] += s
        return f

    def twist(c):
        def f(S_, M_, s):
            e = np.zeros(3)
            e[c] = s
            R = S_.rot[env, obj].reshape(3, 3)
            S_.rot[env, obj] = (expm_so3(e) @ R).ravel()
        return f

    def shift_alpha(k):
        def f(S_, M_, s):
            M_.alpha[k] += s
        return f

    def shift_phi(i):
        def f(S_, M_, s):
            M_.phi[i] += s
        return f

    each = {}
    for key, fns in (("trans", [shift_t(c) for c in range(3)]), ("twist", [twist(c) for c in range(3)]),
                     ("alpha", [shift_alpha(k) for k in range(mesh.n_patches)]),
                     ("phi", [shift_phi(i) for i in phi_idx])):
        flags.clear()
        res[key] = np.array([central(f) for f in fns])
        each[key] = np.array(flags, dtype=bool)
    res["ok_each"] = each
    return res, ok


def twist_from_grad_rot(grad_rot, R):
    """dL/dw_k = sum_ab G_ab ([e_k]_x R)_ab for R' = exp([w]_x) R, w -> 0."""
    G = np.asarray(grad_rot, dtype=np.float64).reshape(3, 3)
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    out = np.empty(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        out[k] = np.sum(G * (skew(e) @ R))
    return out


# ----------------------------------------------------------------------------
# triangle-mesh objects
# ----------------------------------------------------------------------------

def closest_point(q, a, b, c):
    """Closest point of triangle (a, b, c) to q.  Returns (squared distance,
    closest point [3], feature: 0 face, 1 edge ab, 2 bc, 3 ca, 4 vertex a, 5 b,
    6 c)."""
    lib = _load()
    lib.oracle_closest_point.restype = C.c_double
    cp = np.empty(3, np.float64)
    feat = np.empty(1, np.int32)
    s = lib.oracle_closest_point(*[_p(_f64(x)) for x in (q, a, b, c)], _p(cp), _p(feat))
    return float(s), cp, int(feat[0])


def mesh_pseudonormals(meshset, m):
    """Pseudo-normals [T][7][3] of mesh m of a TriMeshSet (face, edges ab bc
    ca, vertices a b c)."""
    lib = _load()
    t0, t1 = int(meshset.tri_offset[m]), int(meshset.tri_offset[m + 1])
    pn = np.empty((t1 - t0, 7, 3), np.float64)
    _call(lib.oracle_mesh_pseudonormals, C.c_int(meshset.n_verts), _f64(meshset.verts), _i32(meshset.tris),
          C.c_int(t0), C.c_int(t1), pn)
    return pn


def contact_mesh(mesh, scene, meshset):
    """Contact with primitives and triangle-mesh objects (type 3, shape[0] =
    mesh index into `meshset`).  Returns contact_obj, uhat, n_active as
    contact()."""
    lib = _load()
    K, N, off, pos, nrm, _ = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    cobj = np.empty((E.value, N.value), np.int8)
    uhat = np.empty((3, E.value, N.value), np.float64)
    na = np.empty((E.value, K.value), np.int32)
    _call(lib.oracle_contact_mesh, K, N, off, pos, nrm, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(meshset.n_meshes), _i32(meshset.tri_offset), C.c_int(meshset.n_verts), _f64(meshset.verts),
          _i32(meshset.tris), cobj, uhat, na)
    return cobj, uhat, na


def contact_mesh_backward(mesh, scene, meshset, grad_uhat):
    """Pose gradients of L = sum(grad_uhat * u_hat) with primitives and mesh
    objects (contact recomputed; winner, triangle and feature held fixed).
    Returns dict(grad_rot [E][O][9], grad_trans [E][O][3])."""
    lib = _load()
    K, N, off, pos, nrm, _ = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    grot = np.empty((E.value, O.value, 9), np.float64)
    gt = np.empty((E.value, O.value, 3), np.float64)
    _call(lib.oracle_contact_mesh_backward, K, N, off, pos, nrm, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(meshset.n_meshes), _i32(meshset.tri_offset), C.c_int(meshset.n_verts), _f64(meshset.verts),
          _i32(meshset.tris), _f64(grad_uhat), grot, gt)
    return dict(grad_rot=grot, grad_trans=gt)


def contact_mesh_features(mesh, scene, meshset):
    """Test hook: the closest-point feature (0 face, 1-3 edges ab bc ca, 4-6
    vertices a b c) of each node won by a mesh object, else -1.  int32 [E][N]."""
    lib = _load()
    K, N, off, pos, nrm, _ = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    feat = np.empty((E.value, N.value), np.int32)
    _call(lib.oracle_contact_mesh_features, K, N, off, pos, nrm, E, O, n_obj, typ, shape, rot, trans,
          C.c_int(meshset.n_meshes), _i32(meshset.tri_offset), C.c_int(meshset.n_verts), _f64(meshset.verts),
          _i32(meshset.tris), feat)
    return feat


# ----------------------------------------------------------------------------
# articulated hand (link frames, self-contact, contact reward)
# ----------------------------------------------------------------------------

def _hand_args(hand, links, rel32):
    return (C.c_int(int(hand.n_links)), _i32(hand.patch_link), np.ascontiguousarray(hand.collide, np.uint32),
            _i32(hand.prim_type), _f64(hand.prim_shape), _f64(hand.prim_rot), _f64(hand.prim_trans),
            _f64(links.rot), _f64(links.trans), C.c_int(1 if rel32 else 0))


def hand_forward(mesh, hand, scene, links, model, omega_a=1.0, rel32=True, with_sig=False, with_margin=False):
    """Articulated-hand step: contact of every patch in its link frame against
    the env's objects and the other links' collision primitives, then Eqs.
    1-2 in the link frames, and the contact-reward terms.  Returns dict(u,
    uhat, contact_obj (object o, O + j for link j), n_active, n_touch, n_a,
    link_mask, r_contact[, sig][, margin [E][K]: each item's decision margin
    as in item_margins])."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    e, n, k = E.value, N.value, K.value
    out = dict(u=np.empty((3, e, n)), uhat=np.empty((3, e, n)), contact_obj=np.empty((e, n), np.int8),
               n_active=np.empty((e, k), np.int32), n_touch=np.empty((e, k), np.int32),
               n_a=np.empty(e, np.int32), link_mask=np.empty(e, np.uint32), r_contact=np.empty(e))
    sig = np.empty(e, np.uint64) if with_sig else None
    margin = np.empty((e, k)) if with_margin else None
    _call(lib.oracle_hand_forward, K, N, off, pos, nrm, origin, E, O, n_obj, typ, shape, rot, trans,
          *_hand_args(hand, links, rel32), C.c_int(model.mode), _f64(model.alpha), _f64(model.phi),
          C.c_double(float(omega_a)), out["u"], out["contact_obj"], out["uhat"], out["n_active"], out["n_touch"],
          out["n_a"], out["link_mask"], out["r_contact"], sig, margin)
    if with_sig:
        out["sig"] = sig
    if with_margin:
        out["margin"] = margin
    return out


def hand_backward(mesh, hand, scene, links, model, grad_u, rel32=True):
    """Adjoint of L = sum(grad_u * U) of the hand step with respect to object
    poses, link poses, alpha and phi."""
    lib = _load()
    K, N, off, pos, nrm, origin = _mesh_args(mesh)
    E, O, n_obj, typ, shape, rot, trans = _scene_args(scene)
    e, o, L = E.value, O.value, int(hand.n_links)
    res = dict(grad_rot=np.empty((e, o, 9)), grad_trans=np.empty((e, o, 3)), grad_link_rot=np.empty((e, L, 9)),
               grad_link_trans=np.empty((e, L, 3)), grad_alpha=np.empty(K.value), grad_phi=np.empty(PHI_SIZE),
               grad_uhat=np.empty((3, e, N.value)))
    _call(lib.oracle_hand_backward, K, N, off, pos, nrm, origin, E, O, n_obj, typ, shape, rot, trans,
          *_hand_args(hand, links, rel32), C.c_int(model.mode), _f64(model.alpha), _f64(model.phi), _f64(grad_u),
          res["grad_rot"], res["grad_trans"], res["grad_link_rot"], res["grad_link_trans"], res["grad_alpha"],
          res["grad_phi"], res["grad_uhat"])
    return res


class _F64Links:
    def __init__(self, lk):
        self.rot = lk.rot.astype(np.float64)
        self.trans = lk.trans.astype(np.float64)


def hand_fd_gradients(mesh, hand, scene, links, model, w, env=0, link=None, obj=None, h=1e-4,
                      shrink=(1e-5, 1e-6)):
    """Central differences of L = sum(w * U) of the hand step in FP64 (relative
    poses kept in FP64) for the 3 translations and 3 twists (R' = exp([+-h
    e_k]_x) R) of link `link` or object `obj` of env `env`.  A difference whose
    two sides take different discrete decisions is retaken with the smaller
    steps; returns (dict(trans, twist, ok_each), ok)."""
    S0, M0, L0 = _F64Scene(scene), _F64Model(model), _F64Links(links)
    flags = []

    def loss(S_, L_):
        out = hand_forward(mesh, hand, S_, L_, M0, rel32=False, with_sig=True)
        return float(np.sum(out["u"] * w)), out["sig"]

    def central(perturb):
        for step in (h,) + tuple(shrink):
            Sp, Lp, Sm, Lm = _F64Scene(S0), _F64Links(L0), _F64Scene(S0), _F64Links(L0)
            for A, B in ((Sp, Lp), (Sm, Lm)):
                A.n_obj, A.type, A.shape = S0.n_obj, S0.type, S0.shape
            perturb(Sp, Lp, step)
            perturb(Sm, Lm, -step)
            lp, sp = loss(Sp, Lp)
            lm, sm = loss(Sm, Lm)
            if np.array_equal(sp, sm):
                flags.append(True)
                return (lp - lm) / (2 * step)
        flags.append(False)
        return (lp - lm) / (2 * step)

    def target(S_, L_):
        if link is not None:
            return L_.rot[env, link], L_.trans[env, link]
        return S_.rot[env, obj], S_.trans[env, obj]

    def shift_t(c):
        def f(S_, L_, s):
            target(S_, L_)[1][c] += s
        return f

    def twist(c):
        def f(S_, L_, s):
            e = np.zeros(3)
            e[c] = s
            R = target(S_, L_)[0]
            R[:] = (expm_so3(e) @ R.reshape(3, 3)).ravel()
        return f

    res, each = {}, {}
    for key, fns in (("trans", [shift_t(c) for c in range(3)]), ("twist", [twist(c) for c in range(3)])):
        flags.clear()
        res[key] = np.array([central(f) for f in fns])
        each[key] = np.array(flags, dtype=bool)
    res["ok_each"] = each
    return res, all(bool(v.all()) for v in each.values())


# ----------------------------------------------------------------------------
# real-sensor regressor (inference)
# ----------------------------------------------------------------------------

REG_SIZE = 88204
REG_LAYERS = (("E1", 64, 6), ("e1", 64, 1), ("E2", 64, 64), ("e2", 64, 1), ("E3", 256, 64), ("e3", 256, 1),
              ("A1", 128, 256), ("a1", 128, 1), ("a2", 128, 1), ("a0", 4, 1), ("D1", 128, 256), ("d1", 128, 1),
              ("D2", 8, 128), ("d2", 8, 1))


def reg_offsets():
    """Offset and shape of every block of the packed regressor parameters."""
    out, off = {}, 0
    for name, o, i in REG_LAYERS:
        out[name] = (off, (o, i) if i > 1 else (o,))
        off += o * i
    assert off == REG_SIZE
    return out


def regress(mesh, reg, u):
    """Taxel outputs y [E][K][8] of the attention-pooled PointNet regressor
    for displacements u [3][E][N] (FP64)."""
    lib = _load()
    K, N, off, pos, _, origin = _mesh_args(mesh)
    uu = _f64(u)
    E = uu.shape[1]
    y = np.empty((E, K.value, 8))
    _call(lib.oracle_regress, K, N, off, pos, origin, C.c_int(E), _f64(reg), uu, y)
    return y
