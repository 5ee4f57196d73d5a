"""The calibration loop (Eq. 3) on the GPU: its gradient against the FP64
oracle's adjoint given the same dL/dU, recovery of a teacher's decay rate,
and loss reduction of the full model on a small hand."""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL, MODE_DECAY_ONLY
from tests.gpu_util import DevModel, DevScene, log, make_plan, to_dev, torch_dev
from tests.test_gpu_backward import MARGIN, SMALL, _close, clean_scene

pytestmark = pytest.mark.gpu


def _setup(mesh, scene, O):
    from paper_2604_20295_amd.calibrate import gpu_step_fn
    ds = DevScene(scene)
    plan = make_plan(mesh, ds.E, O, backward=True)
    return plan, ds, lambda mode: gpu_step_fn(plan, ds.n_obj, ds.type, ds.shape, ds.rot, ds.trans, mode)


def test_calibration_gradient_matches_oracle(oracle_lib):
    # one loss gradient through autograd (library forward + adjoint) against
    # the oracle's adjoint of the same dL/dU, pads with all decisions clear
    import torch
    from paper_2604_20295_amd.calibrate import passive_l2
    mesh, scene, model, _ = scenes.config3()
    model = model.with_mode(MODE_FULL)
    sc, n_clean = clean_scene(oracle_lib, mesh, scene, model)
    assert n_clean >= 1
    teacher = scenes.draw_model(np.random.default_rng(77), mesh.pitch, MODE_FULL)
    target = oracle_lib.forward(mesh, sc, teacher)["u"].astype(np.float32)
    plan, ds, fn = _setup(mesh, sc, 1)
    dm = DevModel(model)
    alpha = dm.alpha.clone().requires_grad_(True)
    phi = dm.phi.clone().requires_grad_(True)
    u, cobj = fn(MODE_FULL)(alpha, phi)
    u.retain_grad()
    loss = passive_l2(u, cobj, to_dev(target))
    loss.backward()
    torch.cuda.synchronize()
    gu = u.grad.double().cpu().numpy()
    log(f"[gpu] calibration gradient, loss {float(loss.detach()):.4e}, envs {n_clean}/8")
    ref = oracle_lib.backward(mesh, sc, model, gu)
    _close(alpha.grad.cpu().numpy(), ref["grad_alpha"], "grad_alpha")
    _close(phi.grad.cpu().numpy(), ref["grad_phi"], "grad_phi")


def test_calibration_recovers_decay_rate(oracle_lib):
    import torch
    from paper_2604_20295_amd.calibrate import Calibrator, teacher_targets
    mesh, scene, model, _ = scenes.config3()
    model = model.with_mode(MODE_DECAY_ONLY)
    plan, ds, fn = _setup(mesh, scene, 1)
    dm = DevModel(model)
    target = teacher_targets(plan, ds.n_obj, ds.type, ds.shape, ds.rot, ds.trans, dm.alpha, dm.phi, MODE_DECAY_ONLY)
    cal = Calibrator(fn(MODE_DECAY_ONLY), target, dm.alpha * 1.3, dm.phi, lr_alpha=0.05, fit_phi=False,
                     lr_decay=0.95)
    l0 = cal.loss()
    for _ in range(120):
        cal.step()
    torch.cuda.synchronize()
    rel = abs(float(cal.alpha[0]) - float(model.alpha[0])) / float(model.alpha[0])
    log(f"[gpu] calibration decay rate: loss {l0:.3e} -> {cal.loss():.3e}, alpha rel err {rel:.2e}")
    assert cal.loss() < 1e-2 * l0
    assert rel < 1e-3


def test_calibration_full_model_reduces_loss(oracle_lib):
    import torch
    from paper_2604_20295_amd.calibrate import Calibrator, teacher_targets
    mesh, scene, model = scenes.config2(n_envs=96, mode=MODE_FULL, **SMALL)
    teacher = scenes.draw_model(np.random.default_rng(5), mesh.pitch, MODE_FULL)
    plan, ds, fn = _setup(mesh, scene, 3)
    dt, dm = DevModel(teacher), DevModel(model)
    target = teacher_targets(plan, ds.n_obj, ds.type, ds.shape, ds.rot, ds.trans, dt.alpha, dt.phi, MODE_FULL)
    cal = Calibrator(fn(MODE_FULL), target, dm.alpha, dm.phi, lr_alpha=0.05, lr_phi=1e-3, lr_decay=0.97)
    hist = [float(cal.step()) for _ in range(60)]
    torch.cuda.synchronize()
    log(f"[gpu] calibration full model: loss {hist[0]:.4e} -> {hist[-1]:.4e}")
    assert all(np.isfinite(hist))
    assert hist[-1] < 0.5 * hist[0]


def test_calibration_with_mesh_objects_recovers_decay_rate(oracle_lib):
    # the loop on a small hand pressed by triangle-mesh objects (and
    # primitives), through ETacMeshStep: a teacher's alpha is recovered
    import torch
    from paper_2604_20295_amd import _native
    from paper_2604_20295_amd.calibrate import Calibrator, gpu_mesh_step_fn
    from scenes import trimeshes as tm
    mesh = scenes.hand_mesh(0, sizes=SMALL["sizes"])
    ms = tm.object_set(scale=SMALL["scale"])
    scene = tm.hand_mesh_scene(mesh, ms, 48, seed=6, p_mesh=0.8, scale=SMALL["scale"])
    model = scenes.draw_model(np.random.default_rng([0, 1]), mesh.pitch, MODE_DECAY_ONLY)
    ds, dm = DevScene(scene), DevModel(model)
    plan = make_plan(mesh, 48, 3, backward=True)
    dms = _native.MeshSet.from_set(ms)
    fn = gpu_mesh_step_fn(plan, dms, ds.n_obj, ds.type, ds.shape, ds.rot, ds.trans, MODE_DECAY_ONLY)
    with torch.no_grad():
        target, cobj = fn(dm.alpha, dm.phi)
        target = target.clone()
    # patches some object touches in the batch: only their alpha gets a gradient
    act = (cobj >= 0).any(0).cpu().numpy()
    touched = np.array([act[a:b].any() for a, b in zip(mesh.patch_offset[:-1], mesh.patch_offset[1:])])
    assert touched.sum() >= 8
    cal = Calibrator(fn, target, dm.alpha * 1.3, dm.phi, lr_alpha=0.05, fit_phi=False, lr_decay=0.95)
    l0 = cal.loss()
    for _ in range(120):
        cal.step()
    torch.cuda.synchronize()
    rel = float(torch.max((torch.abs(cal.alpha - dm.alpha) / dm.alpha)[torch.from_numpy(touched).to(dm.alpha.device)]))
    log(f"[gpu] calibration with mesh objects: loss {l0:.3e} -> {cal.loss():.3e}, alpha max rel err {rel:.2e} "
        f"over the {int(touched.sum())} touched patches")
    assert cal.loss() < 1e-2 * l0
    assert rel < 1e-2
