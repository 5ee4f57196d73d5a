"""ctypes binding of libetac.so: the C ABI of include/etac.h, one Python
function per exported symbol with the same name.  Argument marshalling only;
every step of the computation runs in the library's HIP kernels.

Tensors passed in must already live on the plan's GPU with the documented
dtype, shape and contiguity; they are checked here and passed as raw device
pointers.  Every call is enqueued on torch's current stream of that device.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetac.so")

ETAC_OK = 0
ETAC_SPHERE, ETAC_BOX, ETAC_CAPSULE, ETAC_MESH = 0, 1, 2, 3
ETAC_FULL, ETAC_DECAY_ONLY, ETAC_RESIDUAL_ONLY = 0, 1, 2
ETAC_PHI_SIZE = 17411
ETAC_SAVED_WORDS = 128     # 32-bit words of the pooling record per (env, patch) item
ETAC_MAX_OBJ = 8
ETAC_PLAN_BACKWARD = 1
ETAC_TIMER_CONTACT, ETAC_TIMER_STEP, ETAC_TIMER_BACKWARD, ETAC_TIMER_REDUCE, ETAC_TIMER_BWD_DECAY = 0, 1, 2, 3, 4
ETAC_TIMER_REGRESS = 5
ETAC_REG_SIZE = 88204      # packed regressor parameters
ETAC_TAXELS = 8
ETAC_TIMER_SLOTS = 256

EXPORTED = (
    "etac_plan_create", "etac_plan_destroy", "etac_contact", "etac_propagate", "etac_step", "etac_step_static",
    "etac_plan_set_hand", "etac_hand_contact", "etac_hand_step", "etac_hand_step_backward",
    "etac_contact_backward", "etac_propagate_backward", "etac_step_backward",
    "etac_status_string", "etac_last_hip_error", "etac_plan_info", "etac_plan_set_occupancy",
    "etac_plan_set_timing", "etac_plan_kernel_time", "etac_plan_set_batch",
    "etac_plan_set_launch", "etac_plan_get_launch", "etac_plan_autotune",
    "etac_meshset_create", "etac_meshset_destroy", "etac_contact_mesh", "etac_contact_mesh_backward",
    "etac_regress",
)


class etac_mesh(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("n_nodes", C.c_int32), ("patch_offset", C.c_void_p),
                ("pos", C.c_void_p), ("nrm", C.c_void_p), ("origin", C.c_void_p)]


class etac_scene(C.Structure):
    _fields_ = [("n_envs", C.c_int32), ("max_obj", C.c_int32), ("n_obj", C.c_void_p), ("type", C.c_void_p),
                ("shape", C.c_void_p), ("rot", C.c_void_p), ("trans", C.c_void_p)]


class etac_model(C.Structure):
    _fields_ = [("mode", C.c_int32), ("alpha", C.c_void_p), ("phi", C.c_void_p)]


class etac_hand(C.Structure):
    _fields_ = [("n_links", C.c_int32), ("patch_link", C.c_void_p), ("collide", C.c_void_p),
                ("prim_type", C.c_void_p), ("prim_shape", C.c_void_p), ("prim_rot", C.c_void_p),
                ("prim_trans", C.c_void_p)]


class etac_links(C.Structure):
    _fields_ = [("rot", C.c_void_p), ("trans", C.c_void_p)]


class etac_reward(C.Structure):
    _fields_ = [("omega_a", C.c_float), ("n_touch", C.c_void_p), ("n_a", C.c_void_p), ("link_mask", C.c_void_p),
                ("r_contact", C.c_void_p)]


class EtacError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().etac_status_string(status).decode()
        extra = ""
        if status == -5:
            extra = f" (HIP error {lib().etac_last_hip_error()})"
        super().__init__(f"{fn} failed: {status} {msg}{extra}")
        self.status = status


_lib = None


def lib():
    """Load libetac.so.  Fails loudly if the HIP library has not been built:
    there is no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_20295_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        P = C.POINTER
        sig = {
            "etac_plan_create": ([P(etac_mesh), i32, i32, C.c_uint32, P(vp)], i32),
            "etac_plan_destroy": ([vp], i32),
            "etac_contact": ([vp, P(etac_scene), vp, vp, vp, vp], i32),
            "etac_meshset_create": ([i32, vp, i32, vp, vp, P(vp)], i32),
            "etac_meshset_destroy": ([vp], i32),
            "etac_contact_mesh": ([vp, vp, P(etac_scene), vp, vp, vp, vp, vp], i32),
            "etac_contact_mesh_backward": ([vp, vp, P(etac_scene), vp, vp, vp, vp, vp, vp], i32),
            "etac_propagate": ([vp, P(etac_model), i32, vp, vp, vp, vp, vp], i32),
            "etac_step": ([vp, P(etac_scene), P(etac_model), vp, vp, vp, vp, vp], i32),
            "etac_step_static": ([vp, P(etac_scene), P(etac_model), vp, vp, vp, vp, vp], i32),
            "etac_contact_backward": ([vp, P(etac_scene), vp, vp, vp, vp], i32),
            "etac_propagate_backward": ([vp, P(etac_model), i32, vp, vp, vp, vp, vp, vp, vp, vp], i32),
            "etac_step_backward": ([vp, P(etac_scene), P(etac_model), vp, vp, vp, vp, vp, vp, vp], i32),
            "etac_status_string": ([i32], C.c_char_p),
            "etac_last_hip_error": ([], i32),
            "etac_plan_info": ([vp, P(i32), P(i32), P(i64)], i32),
            "etac_plan_set_occupancy": ([vp, i32], i32),
            "etac_plan_set_timing": ([vp, i32], i32),
            "etac_plan_set_batch": ([vp, i32], i32),
            "etac_plan_set_launch": ([vp, i32, i32, i32, i32, i32], i32),
            "etac_plan_get_launch": ([vp, P(i32)], i32),
            "etac_plan_autotune": ([vp, P(etac_scene), P(etac_model), vp, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                                    P(i32), vp], i32),
            "etac_plan_kernel_time": ([vp, i32, P(i32), P(C.c_double)], i32),
            "etac_plan_set_hand": ([vp, P(etac_hand)], i32),
            "etac_hand_contact": ([vp, P(etac_scene), P(etac_links), vp, vp, vp, P(etac_reward), vp], i32),
            "etac_hand_step": ([vp, P(etac_scene), P(etac_links), P(etac_model), vp, vp, vp, P(etac_reward), vp,
                                vp], i32),
            "etac_hand_step_backward": ([vp, P(etac_scene), P(etac_links), P(etac_model), vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp], i32),
            "etac_regress": ([vp, vp, i32, vp, vp, vp, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(fn, status):
    if status != ETAC_OK:
        raise EtacError(fn, status)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _req(t, dtype, shape, name, device):
    import torch
    if t is None:
        return
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or t.device != device:
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {device}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


class Plan:
    """An etac_plan for one mesh (host arrays, scenes.Mesh layout) on the
    current GPU, sized for up to n_envs envs with up to max_obj objects."""

    def __init__(self, patch_offset, pos, nrm, origin, n_envs, max_obj, backward=False):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._off = np.ascontiguousarray(patch_offset, dtype=np.int32)
        self._pos = np.ascontiguousarray(pos, dtype=np.float32)
        self._nrm = np.ascontiguousarray(nrm, dtype=np.float32)
        self._origin = np.ascontiguousarray(origin, dtype=np.float32)
        self.K = int(self._off.shape[0] - 1)
        self.N = int(self._pos.shape[1])
        self.n_envs, self.max_obj = int(n_envs), int(max_obj)
        m = etac_mesh(self.K, self.N, self._off.ctypes.data, self._pos.ctypes.data, self._nrm.ctypes.data,
                      self._origin.ctypes.data)
        h = C.c_void_p()
        _check("etac_plan_create", lib().etac_plan_create(C.byref(m), self.n_envs, self.max_obj,
                                                          ETAC_PLAN_BACKWARD if backward else 0, C.byref(h)))
        self.handle = h

    @classmethod
    def from_mesh(cls, mesh, n_envs, max_obj, backward=False):
        return cls(mesh.patch_offset, mesh.pos, mesh.nrm, mesh.origin, n_envs, max_obj, backward)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().etac_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n_items, grid, nbytes = C.c_int32(), C.c_int32(), C.c_int64()
        _check("etac_plan_info", lib().etac_plan_info(self.handle, C.byref(n_items), C.byref(grid), C.byref(nbytes)))
        return dict(n_items=n_items.value, grid=grid.value, scratch_bytes=nbytes.value)

    def set_occupancy(self, wg_per_cu):
        _check("etac_plan_set_occupancy", lib().etac_plan_set_occupancy(self.handle, int(wg_per_cu)))

    def set_batch(self, items):
        _check("etac_plan_set_batch", lib().etac_plan_set_batch(self.handle, int(items)))

    def set_launch(self, fwd_wg_per_cu=0, fwd_batch=0, bwd_batch=0, decay_wg_per_cu=0, net_batch=0):
        _check("etac_plan_set_launch", lib().etac_plan_set_launch(self.handle, int(fwd_wg_per_cu), int(fwd_batch),
                                                                  int(bwd_batch), int(decay_wg_per_cu),
                                                                  int(net_batch)))

    def launch(self):
        """(fwd workgroups per CU, fwd batch, decay-adjoint batch, decay
        workgroups per CU, network-adjoint claim)"""
        out = (C.c_int32 * 5)()
        _check("etac_plan_get_launch", lib().etac_plan_get_launch(self.handle, out))
        return tuple(out)

    def set_timing(self, enable):
        _check("etac_plan_set_timing", lib().etac_plan_set_timing(self.handle, 1 if enable else 0))

    def kernel_time(self, timer):
        """(launches, total device ms) of the latest launches of one timed
        kernel since timing was turned on or last read; resets that timer."""
        n, ms = C.c_int32(), C.c_double()
        _check("etac_plan_kernel_time", lib().etac_plan_kernel_time(self.handle, int(timer), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    # -- struct marshalling ---------------------------------------------------
    def scene_struct(self, n_obj, type_, shape, rot, trans):
        import torch
        E, O = int(type_.shape[0]), int(type_.shape[1])
        _req(n_obj, torch.int32, (E,), "n_obj", self.device)
        _req(type_, torch.int32, (E, O), "type", self.device)
        _req(shape, torch.float32, (E, O, 4), "shape", self.device)
        _req(rot, torch.float32, (E, O, 9), "rot", self.device)
        _req(trans, torch.float32, (E, O, 3), "trans", self.device)
        st = etac_scene(E, O, _ptr(n_obj), _ptr(type_), _ptr(shape), _ptr(rot), _ptr(trans))
        st._keep = (n_obj, type_, shape, rot, trans)   # the struct holds raw pointers: keep the tensors alive
        return st

    def set_hand(self, hand):
        """Attach an articulated hand (scenes.articulated.Hand layout: n_links,
        patch_link, collide, prim_type, prim_shape, prim_rot, prim_trans)."""
        self._hand_host = (np.ascontiguousarray(hand.patch_link, np.int32),
                           np.ascontiguousarray(hand.collide, np.uint32),
                           np.ascontiguousarray(hand.prim_type, np.int32),
                           np.ascontiguousarray(hand.prim_shape, np.float32),
                           np.ascontiguousarray(hand.prim_rot, np.float32),
                           np.ascontiguousarray(hand.prim_trans, np.float32))
        pl, co, pt, ps, pr, pp = self._hand_host
        if pl.shape != (self.K,):
            raise ValueError(f"patch_link: expected ({self.K},), got {pl.shape}")
        self.L = int(hand.n_links)
        h = etac_hand(self.L, pl.ctypes.data, co.ctypes.data, pt.ctypes.data, ps.ctypes.data, pr.ctypes.data,
                      pp.ctypes.data)
        _check("etac_plan_set_hand", lib().etac_plan_set_hand(self.handle, C.byref(h)))

    def links_struct(self, rot, trans):
        import torch
        E = int(rot.shape[0])
        _req(rot, torch.float32, (E, self.L, 9), "link rot", self.device)
        _req(trans, torch.float32, (E, self.L, 3), "link trans", self.device)
        st = etac_links(_ptr(rot), _ptr(trans))
        st._keep = (rot, trans)
        return st

    def reward_struct(self, n_envs, omega_a=1.0, n_touch=None, n_a=None, link_mask=None, r_contact=None):
        import torch
        E = int(n_envs)
        _req(n_touch, torch.int32, (E, self.K), "n_touch", self.device)
        _req(n_a, torch.int32, (E,), "n_a", self.device)
        _req(link_mask, torch.int32, (E,), "link_mask (bits as int32)", self.device)
        _req(r_contact, torch.float32, (E,), "r_contact", self.device)
        st = etac_reward(float(omega_a), _ptr(n_touch), _ptr(n_a), _ptr(link_mask), _ptr(r_contact))
        st._keep = (n_touch, n_a, link_mask, r_contact)
        return st

    def model_struct(self, mode, alpha, phi):
        import torch
        _req(alpha, torch.float32, (self.K,), "alpha", self.device)
        _req(phi, torch.float32, (ETAC_PHI_SIZE,), "phi", self.device)
        st = etac_model(int(mode), _ptr(alpha), _ptr(phi))
        st._keep = (alpha, phi)
        return st


def etac_contact(plan, scene, contact_obj, uhat, n_active):
    import torch
    E = scene.n_envs
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(uhat, torch.float32, (3, E, plan.N), "uhat", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _check("etac_contact", lib().etac_contact(plan.handle, C.byref(scene), _ptr(contact_obj), _ptr(uhat),
                                              _ptr(n_active), _stream(plan.device)))


class MeshSet:
    """An etac_meshset on the current GPU: closed triangle meshes of rigid
    objects (verts float32 [V][3], tris int32 [T][3], tri_offset int32
    [M+1]; layout of scenes.trimeshes.TriMeshSet)."""

    def __init__(self, verts, tris, tri_offset):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        v = np.ascontiguousarray(verts, dtype=np.float32)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        off = np.ascontiguousarray(tri_offset, dtype=np.int32)
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3 or off.ndim != 1 or off.size < 2:
            raise ValueError("verts [V][3], tris [T][3], tri_offset [M+1] expected")
        if int(off[-1]) != t.shape[0]:
            raise ValueError("tri_offset[-1] must equal the triangle count")
        self.n_meshes = int(off.size - 1)
        h = C.c_void_p()
        _check("etac_meshset_create", lib().etac_meshset_create(self.n_meshes, off.ctypes.data, int(v.shape[0]),
                                                                v.ctypes.data, t.ctypes.data, C.byref(h)))
        self.handle = h

    @classmethod
    def from_set(cls, ms):
        return cls(ms.verts, ms.tris, ms.tri_offset)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().etac_meshset_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def etac_contact_mesh(plan, meshset, scene, contact_obj, uhat, n_active, hit=None):
    import torch
    E = scene.n_envs
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(uhat, torch.float32, (3, E, plan.N), "uhat", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(hit, torch.int32, (E, plan.N), "hit", plan.device)
    _check("etac_contact_mesh", lib().etac_contact_mesh(plan.handle, meshset.handle, C.byref(scene),
                                                        _ptr(contact_obj), _ptr(uhat), _ptr(n_active), _ptr(hit),
                                                        _stream(plan.device)))


def etac_contact_mesh_backward(plan, meshset, scene, grad_uhat, grad_rot, grad_trans, contact_obj=None, hit=None):
    import torch
    E, O = scene.n_envs, scene.max_obj
    _req(grad_uhat, torch.float32, (3, E, plan.N), "grad_uhat", plan.device)
    _req(grad_rot, torch.float32, (E, O, 9), "grad_rot", plan.device)
    _req(grad_trans, torch.float32, (E, O, 3), "grad_trans", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(hit, torch.int32, (E, plan.N), "hit", plan.device)
    _check("etac_contact_mesh_backward",
           lib().etac_contact_mesh_backward(plan.handle, meshset.handle, C.byref(scene), _ptr(grad_uhat),
                                            _ptr(contact_obj), _ptr(hit), _ptr(grad_rot), _ptr(grad_trans),
                                            _stream(plan.device)))


def saved_buffer(plan, n_envs):
    """A pooling-record buffer for n_envs envs (int32 [E K][ETAC_SAVED_WORDS],
    contents written by a forward call given it)."""
    import torch
    return torch.empty((int(n_envs) * plan.K, ETAC_SAVED_WORDS), dtype=torch.int32, device=plan.device)


def etac_propagate(plan, model, n_envs, contact_obj, uhat, u, saved=None):
    import torch
    E = int(n_envs)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(uhat, torch.float32, (3, E, plan.N), "uhat", plan.device)
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _check("etac_propagate", lib().etac_propagate(plan.handle, C.byref(model), E, _ptr(contact_obj), _ptr(uhat),
                                                  _ptr(u), _ptr(saved), _stream(plan.device)))


def etac_step(plan, scene, model, u, contact_obj, n_active, saved=None):
    import torch
    E = scene.n_envs
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _check("etac_step", lib().etac_step(plan.handle, C.byref(scene), C.byref(model), _ptr(u), _ptr(contact_obj),
                                        _ptr(n_active), _ptr(saved), _stream(plan.device)))


def etac_step_static(plan, scene, model, u, contact_obj, n_active, saved=None):
    """etac_step without allocation: the kernel's scratch is the library's
    static device array (see include/etac.h)."""
    import torch
    E = scene.n_envs
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _check("etac_step_static", lib().etac_step_static(plan.handle, C.byref(scene), C.byref(model), _ptr(u),
                                                      _ptr(contact_obj), _ptr(n_active), _ptr(saved),
                                                      _stream(plan.device)))


def etac_contact_backward(plan, scene, grad_uhat, grad_rot, grad_trans):
    import torch
    E, O = scene.n_envs, scene.max_obj
    _req(grad_uhat, torch.float32, (3, E, plan.N), "grad_uhat", plan.device)
    _req(grad_rot, torch.float32, (E, O, 9), "grad_rot", plan.device)
    _req(grad_trans, torch.float32, (E, O, 3), "grad_trans", plan.device)
    _check("etac_contact_backward", lib().etac_contact_backward(plan.handle, C.byref(scene), _ptr(grad_uhat),
                                                                _ptr(grad_rot), _ptr(grad_trans),
                                                                _stream(plan.device)))


def etac_propagate_backward(plan, model, n_envs, contact_obj, uhat, grad_u, grad_uhat, grad_alpha, grad_phi,
                            saved=None):
    import torch
    E = int(n_envs)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(uhat, torch.float32, (3, E, plan.N), "uhat", plan.device)
    _req(grad_u, torch.float32, (3, E, plan.N), "grad_u", plan.device)
    _req(grad_uhat, torch.float32, (3, E, plan.N), "grad_uhat", plan.device)
    _req(grad_alpha, torch.float32, (plan.K,), "grad_alpha", plan.device)
    _req(grad_phi, torch.float32, (ETAC_PHI_SIZE,), "grad_phi", plan.device)
    _check("etac_propagate_backward",
           lib().etac_propagate_backward(plan.handle, C.byref(model), E, _ptr(contact_obj), _ptr(uhat),
                                         _ptr(grad_u), _ptr(saved), _ptr(grad_uhat), _ptr(grad_alpha),
                                         _ptr(grad_phi), _stream(plan.device)))


def etac_step_backward(plan, scene, model, grad_u, grad_rot, grad_trans, grad_alpha, grad_phi, saved=None):
    import torch
    E, O = scene.n_envs, scene.max_obj
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _req(grad_u, torch.float32, (3, E, plan.N), "grad_u", plan.device)
    _req(grad_rot, torch.float32, (E, O, 9), "grad_rot", plan.device)
    _req(grad_trans, torch.float32, (E, O, 3), "grad_trans", plan.device)
    _req(grad_alpha, torch.float32, (plan.K,), "grad_alpha", plan.device)
    _req(grad_phi, torch.float32, (ETAC_PHI_SIZE,), "grad_phi", plan.device)
    _check("etac_step_backward",
           lib().etac_step_backward(plan.handle, C.byref(scene), C.byref(model), _ptr(grad_u), _ptr(saved),
                                    _ptr(grad_rot), _ptr(grad_trans), _ptr(grad_alpha), _ptr(grad_phi),
                                    _stream(plan.device)))


def etac_plan_autotune(plan, scene, model, u, contact_obj, n_active, grad_u=None, grad_rot=None, grad_trans=None,
                       grad_alpha=None, grad_phi=None, reps=3, saved=None):
    """Time the candidate launch shapes on these inputs, keep the fastest and
    return it as in Plan.launch().  With grad_u None only the forward is
    tuned."""
    import torch
    E, O = scene.n_envs, scene.max_obj
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    if grad_u is not None:
        _req(grad_u, torch.float32, (3, E, plan.N), "grad_u", plan.device)
        _req(grad_rot, torch.float32, (E, O, 9), "grad_rot", plan.device)
        _req(grad_trans, torch.float32, (E, O, 3), "grad_trans", plan.device)
        _req(grad_alpha, torch.float32, (plan.K,), "grad_alpha", plan.device)
        _req(grad_phi, torch.float32, (ETAC_PHI_SIZE,), "grad_phi", plan.device)
    best = (C.c_int32 * 5)()
    _check("etac_plan_autotune",
           lib().etac_plan_autotune(plan.handle, C.byref(scene), C.byref(model), _ptr(grad_u), _ptr(u),
                                    _ptr(contact_obj), _ptr(n_active), _ptr(saved), _ptr(grad_rot), _ptr(grad_trans),
                                    _ptr(grad_alpha), _ptr(grad_phi), int(reps), best, _stream(plan.device)))
    return tuple(best)


def etac_hand_contact(plan, scene, links, contact_obj, uhat, n_active, reward=None):
    import torch
    E = scene.n_envs
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(uhat, torch.float32, (3, E, plan.N), "uhat", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _check("etac_hand_contact", lib().etac_hand_contact(plan.handle, C.byref(scene), C.byref(links), _ptr(contact_obj),
                                                        _ptr(uhat), _ptr(n_active),
                                                        C.byref(reward) if reward is not None else None,
                                                        _stream(plan.device)))


def etac_hand_step(plan, scene, links, model, u, contact_obj, n_active, reward=None, saved=None):
    import torch
    E = scene.n_envs
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(contact_obj, torch.int8, (E, plan.N), "contact_obj", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _check("etac_hand_step", lib().etac_hand_step(plan.handle, C.byref(scene), C.byref(links), C.byref(model),
                                                  _ptr(u), _ptr(contact_obj), _ptr(n_active),
                                                  C.byref(reward) if reward is not None else None, _ptr(saved),
                                                  _stream(plan.device)))


def etac_hand_step_backward(plan, scene, links, model, grad_u, grad_rot, grad_trans, grad_link_rot, grad_link_trans,
                            grad_alpha, grad_phi, saved=None):
    import torch
    E, O = scene.n_envs, scene.max_obj
    _req(saved, torch.int32, (E * plan.K, ETAC_SAVED_WORDS), "saved", plan.device)
    _req(grad_u, torch.float32, (3, E, plan.N), "grad_u", plan.device)
    _req(grad_rot, torch.float32, (E, O, 9), "grad_rot", plan.device)
    _req(grad_trans, torch.float32, (E, O, 3), "grad_trans", plan.device)
    _req(grad_link_rot, torch.float32, (E, plan.L, 9), "grad_link_rot", plan.device)
    _req(grad_link_trans, torch.float32, (E, plan.L, 3), "grad_link_trans", plan.device)
    _req(grad_alpha, torch.float32, (plan.K,), "grad_alpha", plan.device)
    _req(grad_phi, torch.float32, (ETAC_PHI_SIZE,), "grad_phi", plan.device)
    _check("etac_hand_step_backward",
           lib().etac_hand_step_backward(plan.handle, C.byref(scene), C.byref(links), C.byref(model), _ptr(grad_u),
                                         _ptr(saved), _ptr(grad_rot), _ptr(grad_trans), _ptr(grad_link_rot),
                                         _ptr(grad_link_trans), _ptr(grad_alpha), _ptr(grad_phi),
                                         _stream(plan.device)))


def etac_regress(plan, reg, u, n_active, taxels):
    """Real-sensor taxel outputs taxels [E][K][8] of the displacement field u
    [3][E][N] (n_active [E][K] from the same step)."""
    import torch
    E = u.shape[1] if u is not None and u.dim() == 3 else 0
    _req(reg, torch.float32, (ETAC_REG_SIZE,), "reg", plan.device)
    _req(u, torch.float32, (3, E, plan.N), "u", plan.device)
    _req(n_active, torch.int32, (E, plan.K), "n_active", plan.device)
    _req(taxels, torch.float32, (E, plan.K, ETAC_TAXELS), "taxels", plan.device)
    _check("etac_regress", lib().etac_regress(plan.handle, _ptr(reg), int(E), _ptr(u), _ptr(n_active), _ptr(taxels),
                                              _stream(plan.device)))
