"""GPU parity of the network arithmetic across operand ranges.

The residual network runs on FP16 matrix cores with every FP32 operand split
into an FP16 pair (hi + lo).  A pair holds 22 significant bits only inside
[2^-3, 2^15], so the library scales every split operand block by a power of
two chosen from a bound of its magnitude.  These tests move the operands far
from the seeded initialisation and check the library against the FP64 oracle
on the same inputs:

* dL/dU scaled by 1e-9, 1e-20 and 1e3 (a mean-reduced loss over a large batch
  gives dL/dU of 1e-10 and below): gradients compared with a relative bound
  only;
* a function-preserving rescaling of the network's hidden layers by 1e2 and
  1e-2 (ReLU is positively homogeneous: W1, b1 and b2 x c multiply h1 and f
  by c; W3 and W4[:, :64] / c leave g' and h4 as they are), so h1 and f move
  by c while the displacements stay in mm: forward at 1e-5 mm, adjoint at
  the usual bound;
* Phi scaled as a whole by 1e-2 and 1e2: residuals shrink or grow by up to
  1e10, so the displacement bound is relative to max |U|;
* patch origins moved by 500 mm (network inputs near 500);
* Phi after 60 Adam iterations of the Eq. 3 calibration, driven by the
  oracle's own forward and adjoint.
"""
import numpy as np
import pytest

import scenes
from scenes import MODE_FULL
from tests.gpu_util import TOL_U, gpu_step, log, make_plan, max_err
from tests.test_gpu_backward import MARGIN, SMALL, _close, gpu_step_backward

pytestmark = pytest.mark.gpu

OFF = scenes.phi_offsets()


def _block(phi, name):
    o, i = {"W1": (64, 9), "W2": (64, 64), "W3": (64, 64), "W4": (64, 128), "W5": (3, 64)}[name]
    return phi[OFF[name]:OFF[name] + o * i].reshape(o, i)


def rescaled_phi(phi, c):
    """Same function, hidden activations h1 and f multiplied by c (FP32 values
    given to both sides)."""
    p = phi.astype(np.float64).copy()
    _block(p, "W1")[:] *= c                # h1 -> c h1
    p[OFF["b1"]:OFF["b1"] + 64] *= c
    p[OFF["b2"]:OFF["b2"] + 64] *= c       # with W2 unchanged: f -> c f, g -> c g
    _block(p, "W3")[:] /= c                # g' unchanged
    _block(p, "W4")[:, :64] /= c           # h4 unchanged
    return p.astype(np.float32)


def _clean(oracle_lib, mesh, scene, model, margin):
    out = oracle_lib.forward(mesh, scene, model, with_sig=True)
    keep = out["margin"] > margin
    s = scene.copy()
    s.n_obj[~keep] = 0
    return s, int((keep & (out["n_active"].sum(axis=1) > 0)).sum())


def _compare_grads(g, ref, rel=1e-4, atol=0.0):
    for name in ("grad_trans", "grad_rot", "grad_alpha", "grad_phi"):
        _close(g[name], ref[name], name, rel=rel, atol=atol)


def _forward(oracle_lib, mesh, scene, model, plan, tol):
    u, cobj, na = gpu_step(plan, scene, model)
    ref = oracle_lib.forward(mesh, scene, model)
    assert np.array_equal(cobj, ref["contact_obj"])
    assert np.array_equal(na, ref["n_active"])
    err = max_err(u, ref["u"])
    log(f"[gpu]   max|dU| {err:.3e} mm (bound {tol:.3e}), max|U| {np.abs(ref['u']).max():.3e}")
    assert np.all(np.isfinite(u))
    assert err <= tol
    return ref


@pytest.mark.parametrize("factor", [1e-9, 1e-20, 1e3])
def test_grad_u_scale(oracle_lib, factor):
    # dL/dU far from O(1): the adjoint scales its gradient operands per item
    mesh, scene, model = scenes.config2(n_envs=96, mode=MODE_FULL, **SMALL)
    sc, n_clean = _clean(oracle_lib, mesh, scene, model, MARGIN)
    log(f"[gpu] grad_u x {factor:g}: envs compared {n_clean}/96")
    assert n_clean >= 20
    w = np.random.default_rng(4).standard_normal((3, 96, mesh.n_nodes)) * factor
    w = w.astype(np.float32).astype(np.float64)
    plan = make_plan(mesh, 96, 3, backward=True)
    g = gpu_step_backward(plan, sc, model, w)
    ref = oracle_lib.backward(mesh, sc, model, w)
    # relative bound only: an absolute floor would hide a scaled-down failure
    _compare_grads(g, ref, rel=1e-4, atol=0.0)
    # the Phi gradient is not zero, and neither block of it is lost
    for name in ("W1", "W2", "W4", "W5"):
        gb, rb = _block(g["grad_phi"], name), _block(ref["grad_phi"], name)
        assert np.max(np.abs(rb)) > 0.0
        assert np.max(np.abs(gb - rb)) <= 1e-4 * np.max(np.abs(rb)), name


@pytest.mark.parametrize("c", [1e2, 1e-2])
def test_hidden_layers_rescaled(oracle_lib, c):
    mesh, scene, model = scenes.config2(n_envs=48, mode=MODE_FULL)
    m = scenes.Model(MODE_FULL, model.alpha, rescaled_phi(model.phi, c))
    log(f"[gpu] hidden layers x {c:g}: forward, 48-env hand")
    plan = make_plan(mesh, 48, 3)
    _forward(oracle_lib, mesh, scene, m, plan, TOL_U)
    mesh, scene, model = scenes.config2(n_envs=96, mode=MODE_FULL, **SMALL)
    m = scenes.Model(MODE_FULL, model.alpha, rescaled_phi(model.phi, c))
    # the rescaled network takes the unscaled one's decisions, each at c times
    # its distance from the boundary, with rounding errors c times as large:
    # the unscaled network's margins select the envs
    sc, n_clean = _clean(oracle_lib, mesh, scene, model, MARGIN)
    log(f"[gpu] hidden layers x {c:g}: adjoint, envs compared {n_clean}/96")
    assert n_clean >= 10
    w = np.random.default_rng(4).standard_normal((3, 96, mesh.n_nodes))
    plan = make_plan(mesh, 96, 3, backward=True)
    g = gpu_step_backward(plan, sc, m, w)
    _compare_grads(g, oracle_lib.backward(mesh, sc, m, w), atol=1e-6)


@pytest.mark.parametrize("c", [1e-2, 1e2])
def test_phi_scaled_whole(oracle_lib, c):
    # every weight and bias x c: residuals scale by up to c^5, so the bound is
    # relative to the largest displacement (FP32 arithmetic, ~2^-22 per split
    # product, sums of 64 terms over four layers)
    mesh, scene, model = scenes.config2(n_envs=48, mode=MODE_FULL)
    m = scenes.Model(MODE_FULL, model.alpha, (model.phi.astype(np.float64) * c).astype(np.float32))
    ref = oracle_lib.forward(mesh, scene, m)
    tol = max(TOL_U, 2e-5 * float(np.abs(ref["u"]).max()))
    log(f"[gpu] Phi x {c:g}: forward, 48-env hand")
    _forward(oracle_lib, mesh, scene, m, make_plan(mesh, 48, 3), tol)


def test_origins_500mm(oracle_lib):
    # network inputs p - o_k near 500 mm
    mesh, scene, model = scenes.config2(n_envs=48, mode=MODE_FULL)
    shift = np.array([500.0, -500.0, 500.0])
    mesh.origin = (mesh.origin.astype(np.float64) + shift).astype(np.float32)
    log("[gpu] origins + 500 mm: forward, 48-env hand")
    _forward(oracle_lib, mesh, scene, model, make_plan(mesh, 48, 3), TOL_U)
    mesh, scene, model = scenes.config2(n_envs=256, mode=MODE_FULL, **SMALL)
    mesh.origin = (mesh.origin.astype(np.float64) + shift).astype(np.float32)
    # FP32 rounding of p - o (~3e-5 mm) and the split products (~2^-22 of
    # |W1| |x|) put the pre-activations within ~2e-4 of FP64: margin 1e-3
    sc, n_clean = _clean(oracle_lib, mesh, scene, model, 1e-3)
    log(f"[gpu] origins + 500 mm: adjoint, envs compared {n_clean}/256")
    assert n_clean >= 4
    w = np.random.default_rng(7).standard_normal((3, 256, mesh.n_nodes))
    plan = make_plan(mesh, 256, 3, backward=True)
    g = gpu_step_backward(plan, sc, model, w)
    _compare_grads(g, oracle_lib.backward(mesh, sc, model, w), atol=1e-6)


def calibrated_phi(oracle_lib, iters=60):
    """Phi after `iters` Adam iterations of the Eq. 3 loss on the 8 pads
    against a teacher model, every forward and adjoint taken by the oracle."""
    import torch
    from paper_2604_20295_amd.calibrate import Calibrator
    from tests.test_calibration import _OracleStep
    mesh, scene, model, _ = scenes.config3()
    teacher = scenes.draw_model(np.random.default_rng(77), mesh.pitch, MODE_FULL)
    out = oracle_lib.forward(mesh, scene, teacher)
    target = torch.from_numpy(out["u"])
    cobj = torch.from_numpy(oracle_lib.forward(mesh, scene, model)["contact_obj"])

    def step_fn(alpha, phi):
        return _OracleStep.apply(alpha, phi, oracle_lib, mesh, scene, MODE_FULL), cobj

    cal = Calibrator(step_fn, target, torch.from_numpy(model.alpha.astype(np.float64)),
                     torch.from_numpy(model.phi.astype(np.float64)), lr_alpha=0.02, lr_phi=3e-3)
    l0 = cal.loss()
    for _ in range(iters):
        cal.step()
    l1 = cal.loss()
    phi = cal.phi.detach().numpy().astype(np.float32)
    return phi, float(np.abs(phi - model.phi).max()), l0, l1


def test_calibrated_phi(oracle_lib):
    phi, moved, l0, l1 = calibrated_phi(oracle_lib)
    log(f"[gpu] calibrated Phi: loss {l0:.4e} -> {l1:.4e}, max|dPhi| {moved:.3e}")
    assert l1 < l0
    mesh, scene, model = scenes.config2(n_envs=48, mode=MODE_FULL)
    m = scenes.Model(MODE_FULL, model.alpha, phi)
    _forward(oracle_lib, mesh, scene, m, make_plan(mesh, 48, 3), TOL_U)
    mesh, scene, model = scenes.config2(n_envs=96, mode=MODE_FULL, **SMALL)
    m = scenes.Model(MODE_FULL, model.alpha, phi)
    sc, n_clean = _clean(oracle_lib, mesh, scene, m, MARGIN)
    log(f"[gpu] calibrated Phi: adjoint, envs compared {n_clean}/96")
    assert n_clean >= 10
    w = np.random.default_rng(4).standard_normal((3, 96, mesh.n_nodes))
    plan = make_plan(mesh, 96, 3, backward=True)
    g = gpu_step_backward(plan, sc, m, w)
    _compare_grads(g, oracle_lib.backward(mesh, sc, m, w), atol=1e-6)
