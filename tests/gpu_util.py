"""Helpers of the GPU parity tests: upload seeded scenes to the device and run
the C-ABI calls through the ctypes binding."""
import sys

import numpy as np

TOL_U = 1e-5   # mm, FP32 GPU vs FP64 oracle (max abs)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def to_dev(a, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev).contiguous()


class DevScene:
    def __init__(self, scene):
        torch, _ = torch_dev()
        self.n_obj = to_dev(scene.n_obj.astype(np.int32))
        self.type = to_dev(scene.type.astype(np.int32))
        self.shape = to_dev(scene.shape.astype(np.float32))
        self.rot = to_dev(scene.rot.astype(np.float32))
        self.trans = to_dev(scene.trans.astype(np.float32))
        self.E, self.O = scene.type.shape

    def struct(self, plan):
        return plan.scene_struct(self.n_obj, self.type, self.shape, self.rot, self.trans)


class DevModel:
    def __init__(self, model):
        self.mode = model.mode
        self.alpha = to_dev(model.alpha.astype(np.float32))
        self.phi = to_dev(model.phi.astype(np.float32))

    def struct(self, plan, mode=None):
        return plan.model_struct(self.mode if mode is None else mode, self.alpha, self.phi)


def make_plan(mesh, n_envs, max_obj, backward=False):
    from paper_2604_20295_amd import _native
    return _native.Plan.from_mesh(mesh, n_envs, max_obj, backward)


def gpu_contact(plan, scene):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    ds = DevScene(scene)
    E, N, K = ds.E, plan.N, plan.K
    cobj = torch.full((E, N), 99, dtype=torch.int8, device=dev)
    uhat = torch.full((3, E, N), float("nan"), dtype=torch.float32, device=dev)
    na = torch.full((E, K), -7, dtype=torch.int32, device=dev)
    _native.etac_contact(plan, ds.struct(plan), cobj, uhat, na)
    torch.cuda.synchronize()
    return cobj.cpu().numpy(), uhat.cpu().numpy(), na.cpu().numpy()


def gpu_step(plan, scene, model, mode=None):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    ds, dm = DevScene(scene), DevModel(model)
    E, N, K = ds.E, plan.N, plan.K
    u = torch.full((3, E, N), float("nan"), dtype=torch.float32, device=dev)
    cobj = torch.full((E, N), 99, dtype=torch.int8, device=dev)
    na = torch.full((E, K), -7, dtype=torch.int32, device=dev)
    _native.etac_step(plan, ds.struct(plan), dm.struct(plan, mode), u, cobj, na)
    torch.cuda.synchronize()
    return u.cpu().numpy(), cobj.cpu().numpy(), na.cpu().numpy()


def gpu_propagate(plan, model, cobj, uhat, mode=None):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    dm = DevModel(model)
    E = cobj.shape[0]
    c = to_dev(cobj.astype(np.int8))
    uh = to_dev(uhat.astype(np.float32))
    u = torch.full((3, E, plan.N), float("nan"), dtype=torch.float32, device=dev)
    _native.etac_propagate(plan, dm.struct(plan, mode), E, c, uh, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def max_err(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)))) if np.size(a) else 0.0
