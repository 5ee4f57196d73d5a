"""Host-side validation of the C ABI against a real plan: every check runs
before anything is enqueued, so the calls below return their status codes
without launching a kernel (a GPU is needed only to create the plan)."""
import ctypes as C

import numpy as np
import pytest

import scenes
from tests.gpu_util import DevModel, DevScene, log, make_plan, to_dev, torch_dev

pytestmark = pytest.mark.gpu

OK, ERR_NULL, ERR_SHAPE, ERR_VALUE, ERR_WORKSPACE, ERR_CAPTURE = 0, -1, -2, -3, -4, -6


def _setup(E=4, O=3, backward=False):
    mesh, scene, model = scenes.config2(n_envs=E)
    plan = make_plan(mesh, E, O, backward=backward)
    return mesh, scene, model, plan


def _bufs(plan, E, O):
    torch, dev = torch_dev()
    return dict(u=torch.zeros((3, E, plan.N), device=dev), cobj=torch.zeros((E, plan.N), dtype=torch.int8, device=dev),
                na=torch.zeros((E, plan.K), dtype=torch.int32, device=dev),
                gu=torch.zeros((3, E, plan.N), device=dev), grot=torch.zeros((E, O, 9), device=dev),
                gt=torch.zeros((E, O, 3), device=dev), ga=torch.zeros((plan.K,), device=dev),
                gp=torch.zeros((17411,), device=dev), uhat=torch.zeros((3, E, plan.N), device=dev))


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def test_backward_needs_backward_scratch(oracle_lib):
    from paper_2604_20295_amd import _native
    mesh, scene, model, plan = _setup(backward=False)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    b = _bufs(plan, 4, 3)
    L = _native.lib()
    log("[gpu] validation: backward calls on a forward-only plan")
    st = L.etac_step_backward(plan.handle, C.byref(sc), C.byref(md), _p(b["gu"]), None, _p(b["grot"]),
                              _p(b["gt"]), _p(b["ga"]), _p(b["gp"]), None)
    assert st == ERR_WORKSPACE
    st = L.etac_propagate_backward(plan.handle, C.byref(md), 4, _p(b["cobj"]), _p(b["uhat"]), _p(b["gu"]), None,
                                   _p(b["uhat"]), _p(b["ga"]), _p(b["gp"]), None)
    assert st == ERR_WORKSPACE
    # the contact adjoint keeps its per-item pose partials in the backward scratch too
    st = L.etac_contact_backward(plan.handle, C.byref(sc), _p(b["uhat"]), _p(b["grot"]), _p(b["gt"]), None)
    assert st == ERR_WORKSPACE
    # the forward needs no backward scratch
    assert L.etac_step(plan.handle, C.byref(sc), C.byref(md), _p(b["u"]), _p(b["cobj"]), _p(b["na"]), None,
                       None) == OK


def test_sizes_beyond_the_plan_and_bad_models(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model, plan = _setup(E=4, O=2, backward=True)
    big = scenes.config2(n_envs=8)[1]          # 8 envs, 3 objects: more than the plan holds
    dsb, dm = DevScene(big), DevModel(model)
    b = _bufs(plan, 8, 3)
    L = _native.lib()
    md = dm.struct(plan)
    log("[gpu] validation: n_envs and max_obj beyond the plan")
    scb = _native.etac_scene(8, 2, _p(dsb.n_obj), _p(dsb.type), _p(dsb.shape), _p(dsb.rot), _p(dsb.trans))
    for fn in (L.etac_step, L.etac_step_static):
        assert fn(plan.handle, C.byref(scb), C.byref(md), _p(b["u"]), _p(b["cobj"]), _p(b["na"]), None,
                  None) == ERR_SHAPE
    assert L.etac_contact(plan.handle, C.byref(scb), _p(b["cobj"]), _p(b["uhat"]), _p(b["na"]), None) == ERR_SHAPE
    assert L.etac_step_backward(plan.handle, C.byref(scb), C.byref(md), _p(b["gu"]), None, _p(b["grot"]),
                                _p(b["gt"]), _p(b["ga"]), _p(b["gp"]), None) == ERR_SHAPE
    assert L.etac_propagate(plan.handle, C.byref(md), 8, _p(b["cobj"]), _p(b["uhat"]), _p(b["u"]), None,
                            None) == ERR_SHAPE
    # three objects per env on a plan made for two
    sco = _native.etac_scene(4, 3, _p(dsb.n_obj), _p(dsb.type), _p(dsb.shape), _p(dsb.rot), _p(dsb.trans))
    assert L.etac_step(plan.handle, C.byref(sco), C.byref(md), _p(b["u"]), _p(b["cobj"]), _p(b["na"]), None,
                       None) == ERR_SHAPE
    # models: phi NULL is allowed only in decay-only mode; unknown modes
    sc = _native.etac_scene(4, 2, _p(dsb.n_obj), _p(dsb.type), _p(dsb.shape), _p(dsb.rot), _p(dsb.trans))
    alpha = to_dev(model.alpha.astype(np.float32))
    for mode, expect in ((scenes.MODE_FULL, ERR_VALUE), (scenes.MODE_RESIDUAL_ONLY, ERR_VALUE),
                         (scenes.MODE_DECAY_ONLY, OK), (7, ERR_VALUE)):
        m = _native.etac_model(mode, _p(alpha), None)
        for fn in (L.etac_step, L.etac_step_static):
            assert fn(plan.handle, C.byref(sc), C.byref(m), _p(b["u"]), _p(b["cobj"]), _p(b["na"]), None,
                      None) == expect, (mode, fn)
        st = L.etac_step_backward(plan.handle, C.byref(sc), C.byref(m), _p(b["gu"]), None, _p(b["grot"]),
                                  _p(b["gt"]), _p(b["ga"]), _p(b["gp"]), None)
        assert st == expect, mode
    m = _native.etac_model(scenes.MODE_FULL, None, None)
    assert L.etac_step(plan.handle, C.byref(sc), C.byref(m), _p(b["u"]), _p(b["cobj"]), _p(b["na"]), None,
                       None) == ERR_NULL
    # missing outputs
    assert L.etac_step_static(plan.handle, C.byref(sc), C.byref(md), None, _p(b["cobj"]), _p(b["na"]), None,
                              None) == ERR_NULL
    torch.cuda.synchronize()


def test_autotune_refuses_stream_capture(oracle_lib):
    from paper_2604_20295_amd import _native
    torch, dev = torch_dev()
    mesh, scene, model, plan = _setup(E=4, O=3, backward=True)
    ds, dm = DevScene(scene), DevModel(model)
    sc, md = ds.struct(plan), dm.struct(plan)
    b = _bufs(plan, 4, 3)
    L = _native.lib()
    log("[gpu] validation: autotuning during stream capture")
    g = torch.cuda.CUDAGraph()
    statuses = []
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream(dev).cuda_stream
        statuses.append(L.etac_plan_autotune(plan.handle, C.byref(sc), C.byref(md), _p(b["gu"]), _p(b["u"]),
                                             _p(b["cobj"]), _p(b["na"]), None, _p(b["grot"]), _p(b["gt"]),
                                             _p(b["ga"]), _p(b["gp"]), 1, None, C.c_void_p(s)))
    assert statuses == [ERR_CAPTURE]
    g.replay()                  # the captured graph is empty
    torch.cuda.synchronize()
    assert L.etac_status_string(ERR_CAPTURE).decode().startswith("plan creation or autotuning")
