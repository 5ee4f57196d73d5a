"""The fused step that allocates nothing (etac_step_static): its kernel's
scratch is the library's file-scope device array instead of the plan's.
Called through the C ABI, it gives exactly etac_step's results, on two
calls in a row (the second with fewer envs), and on a plan with
high-resolution pads, where the array holds fewer persistent workgroups than
the plan's grid."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import DevModel, DevScene, log, make_plan, torch_dev

pytestmark = pytest.mark.gpu


def _run(fn, plan, scene, model, saved=False):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    ds, dm = DevScene(scene), DevModel(model)
    E = ds.E
    u = torch.full((3, E, plan.N), float("nan"), dtype=torch.float32, device=dev)
    cobj = torch.full((E, plan.N), 99, dtype=torch.int8, device=dev)
    na = torch.full((E, plan.K), -7, dtype=torch.int32, device=dev)
    rec = torch.full((E * plan.K, _native.ETAC_SAVED_WORDS), -1, dtype=torch.int32, device=dev) if saved else None
    fn(plan, ds.struct(plan), dm.struct(plan), u, cobj, na, saved=rec)
    torch.cuda.synchronize()
    out = [u.cpu().numpy(), cobj.cpu().numpy(), na.cpu().numpy()]
    if saved:
        out.append(rec.cpu().numpy())
    return out


def _same(a, b, what):
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=False), what


def test_static_step_equals_step(oracle_lib):
    from paper_2604_20295_amd import _native
    mesh, scene, model = scenes.config2(n_envs=256)
    plan = make_plan(mesh, 256, scene.max_obj)
    log("[gpu] etac_step_static vs etac_step: 256-env hand, then 64 envs")
    ref = _run(_native.etac_step, plan, scene, model, saved=True)
    got = _run(_native.etac_step_static, plan, scene, model, saved=True)
    _same(ref, got, "256 envs")
    small = scene.select(np.arange(64))
    ref2 = _run(_native.etac_step, plan, small, model)
    got2 = _run(_native.etac_step_static, plan, small, model)
    _same(ref2, got2, "64 envs")
    out = oracle_lib.forward(mesh, small, model)
    assert np.array_equal(got2[1], out["contact_obj"])
    assert float(np.max(np.abs(got2[0] - out["u"]))) <= 1e-5


def test_static_step_with_fewer_workgroups(oracle_lib):
    # patches of 16384 nodes: one workgroup's slice is 512 KiB, so the 64 MiB
    # array holds fewer workgroups than the plan's persistent grid
    from paper_2604_20295_amd import _native
    mesh, scene, model = scenes.config4(n_envs=96)
    plan = make_plan(mesh, 96, scene.max_obj)
    log("[gpu] etac_step_static vs etac_step: 96 envs of high-resolution pads, then 8")
    _same(_run(_native.etac_step, plan, scene, model), _run(_native.etac_step_static, plan, scene, model), "96 envs")
    small = scene.select(np.arange(8))
    _same(_run(_native.etac_step, plan, small, model), _run(_native.etac_step_static, plan, small, model), "8 envs")
