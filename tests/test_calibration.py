"""The calibration loop (Eq. 3) on the CPU: the loss helper against its
analytic gradient and central differences, and the Adam loop driven by the
FP64 oracle recovering a teacher's decay rate on the pad."""
import numpy as np
import pytest
import torch

import scenes
from scenes import MODE_DECAY_ONLY
from paper_2604_20295_amd.calibrate import Calibrator, passive_l2


def test_passive_l2_gradient():
    g = torch.Generator().manual_seed(3)
    u = torch.randn(3, 4, 50, generator=g, dtype=torch.float64, requires_grad=True)
    target = torch.randn(3, 4, 50, generator=g, dtype=torch.float64)
    cobj = torch.randint(-1, 3, (4, 50), generator=g).to(torch.int8)
    loss = passive_l2(u, cobj, target)
    loss.backward()
    passive = (cobj < 0).numpy()[None]
    r = np.where(passive, (u - target).detach().numpy(), 0.0)
    assert abs(float(loss) - np.sqrt((r * r).sum())) < 1e-12
    # d||r||/du = r / ||r|| on passive entries, 0 on active ones
    assert np.allclose(u.grad.numpy(), r / np.sqrt((r * r).sum()), atol=1e-14)
    # central differences on a few entries
    for idx in [(0, 0, 0), (1, 2, 7), (2, 3, 49)]:
        h = 1e-6
        up = u.detach().clone(); up[idx] += h
        um = u.detach().clone(); um[idx] -= h
        fd = (float(passive_l2(up, cobj, target)) - float(passive_l2(um, cobj, target))) / (2 * h)
        assert abs(fd - float(u.grad[idx])) < 1e-7


class _OracleStep(torch.autograd.Function):
    """(alpha, phi) -> U through the FP64 oracle, with its adjoint."""

    @staticmethod
    def forward(ctx, alpha, phi, oracle, mesh, scene, mode):
        model = scenes.Model(mode, alpha.detach().numpy().astype(np.float32), phi.detach().numpy().astype(np.float32))
        out = oracle.forward(mesh, scene, model)
        ctx.args = (oracle, mesh, scene, model)
        ctx.cobj = out["contact_obj"]
        return torch.from_numpy(out["u"])

    @staticmethod
    def backward(ctx, gu):
        oracle, mesh, scene, model = ctx.args
        g = oracle.backward(mesh, scene, model, gu.numpy().astype(np.float64))
        return (torch.from_numpy(g["grad_alpha"]).to(torch.float64),
                torch.from_numpy(g["grad_phi"]).to(torch.float64), None, None, None, None)


def test_calibrator_recovers_decay_rate_with_oracle(oracle_lib):
    mesh, scene, model, _ = scenes.config3(seeds=range(2))
    model = model.with_mode(MODE_DECAY_ONLY)
    alpha_t = model.alpha.astype(np.float64)
    phi = torch.from_numpy(model.phi.astype(np.float64))
    # targets from the teacher
    target = torch.from_numpy(oracle_lib.forward(mesh, scene, model)["u"])
    cobj = torch.from_numpy(oracle_lib.forward(mesh, scene, model)["contact_obj"])

    def step_fn(alpha, phi_):
        u = _OracleStep.apply(alpha, phi_, oracle_lib, mesh, scene, MODE_DECAY_ONLY)
        return u, cobj

    cal = Calibrator(step_fn, target, torch.from_numpy(alpha_t * 1.3), phi, lr_alpha=0.05, fit_phi=False,
                     lr_decay=0.95)
    l0 = cal.loss()
    for _ in range(100):
        cal.step()
    rel = abs(float(cal.alpha[0]) - alpha_t[0]) / alpha_t[0]
    assert cal.loss() < 1e-3 * l0
    assert rel < 1e-4, rel
