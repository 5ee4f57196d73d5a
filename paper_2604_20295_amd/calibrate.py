"""Calibration of the propagation model against target displacements.

The paper calibrates the decay rate alpha (Eq. 1) and the residual network's
weights Phi (Eq. 2) by gradient descent on the displacement error of the
passive nodes against FEM (Sec. III-A, "Learn Propagation Dynamics From FEM",
Eq. 3): L = || U_p - U*_p ||_2, the 2-norm over every passive node of the
batch of loading frames.  Here the targets U* are synthetic (no FEM data
ships with this project): displacements of the same scenes from a "teacher"
model with other parameters.

Each iteration is one forward and one adjoint of the library (the fused
etac_step and etac_step_backward through autograd.ETacStep, with the pooling
record); the loss, its gradient dL/dU and the Adam update are a few torch
elementwise operations and reductions over the step's outputs.  alpha is
optimised through log(alpha) so that it stays positive.
"""
import torch

from . import _native
from .autograd import ETacStep


def passive_l2(u, contact_obj, target):
    """Eq. 3: the 2-norm of U - U* over the passive nodes (contact_obj < 0)
    of every env.  u, target [3][E][N]; contact_obj [E][N]."""
    mask = (contact_obj < 0).unsqueeze(0)
    r = torch.where(mask, u - target, torch.zeros_like(u))
    return torch.linalg.vector_norm(r)


def gpu_step_fn(plan, n_obj, type_, shape, rot, trans, mode):
    """(alpha, phi) -> (U, contact_obj) through the library, differentiable in
    alpha and phi."""
    def step(alpha, phi):
        u, cobj, _ = ETacStep.apply(plan, n_obj, type_, shape, rot, trans, alpha, phi, mode)
        return u, cobj
    return step


def gpu_mesh_step_fn(plan, meshset, n_obj, type_, shape, rot, trans, mode):
    """(alpha, phi) -> (U, contact_obj) through the library for scenes with
    triangle-mesh objects (autograd.ETacMeshStep), differentiable in alpha
    and phi."""
    from .autograd import ETacMeshStep

    def step(alpha, phi):
        u, cobj, _ = ETacMeshStep.apply(plan, meshset, n_obj, type_, shape, rot, trans, alpha, phi, mode)
        return u, cobj
    return step


class Calibrator:
    """Adam on (log alpha, phi) for the Eq. 3 loss of one fixed batch of
    scenes, learning rates multiplied by `lr_decay` after every step.
    `step_fn(alpha, phi) -> (U, contact_obj)` is differentiable in alpha and
    phi (gpu_step_fn for the library)."""

    def __init__(self, step_fn, target, alpha0, phi0, lr_alpha=1e-2, lr_phi=1e-3, fit_alpha=True,
                 fit_phi=True, lr_decay=1.0):
        self.step_fn = step_fn
        self.target = target
        self.log_alpha = torch.log(alpha0.detach().clone()).requires_grad_(fit_alpha)
        self.phi = phi0.detach().clone().requires_grad_(fit_phi)
        groups = []
        if fit_alpha:
            groups.append({"params": [self.log_alpha], "lr": lr_alpha})
        if fit_phi:
            groups.append({"params": [self.phi], "lr": lr_phi})
        self.opt = torch.optim.Adam(groups)
        # the Eq. 3 loss is a norm, not its square: its gradient keeps its size
        # near the optimum, so a decaying step lets Adam settle
        self.sched = torch.optim.lr_scheduler.ExponentialLR(self.opt, gamma=lr_decay)

    @property
    def alpha(self):
        return torch.exp(self.log_alpha.detach())

    def loss(self):
        """Current loss without an update."""
        with torch.no_grad():
            u, cobj = self.step_fn(torch.exp(self.log_alpha), self.phi)
            return float(passive_l2(u, cobj, self.target))

    def step(self):
        """One forward, adjoint and Adam update; returns the loss before it."""
        self.opt.zero_grad(set_to_none=True)
        u, cobj = self.step_fn(torch.exp(self.log_alpha), self.phi)
        loss = passive_l2(u, cobj, self.target)
        loss.backward()
        self.opt.step()
        self.sched.step()
        return loss.detach()


def teacher_targets(plan, n_obj, type_, shape, rot, trans, alpha, phi, mode=_native.ETAC_FULL):
    """Target displacements [3][E][N] of the scenes under a teacher model."""
    with torch.no_grad():
        u, _ = gpu_step_fn(plan, n_obj, type_, shape, rot, trans, mode)(alpha, phi)
    return u.clone()
