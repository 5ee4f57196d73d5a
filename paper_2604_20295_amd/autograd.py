"""torch.autograd binding of the ETac step.

ETacStep.apply(plan, n_obj, type, shape, rot, trans, alpha, phi, mode)
returns (u [3][E][N], contact_obj [E][N], n_active [E][K]); gradients flow to
rot [E][O][9], trans [E][O][3], alpha [K] and phi [17411].  The forward runs
etac_step, the backward runs etac_step_backward, which recomputes the contact
pass; besides the inputs only the network's pooling record (pooled features
and their arg-max nodes, 512 bytes per (env, patch) item) is saved.
ETacMeshStep does the same for scenes with triangle-mesh objects, and
ETacHandStep for the articulated hand (gradients also to the link poses).
Argument marshalling only.
"""
import torch

from . import _native


class ETacStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, n_obj, type_, shape, rot, trans, alpha, phi, mode):
        rot, trans = rot.contiguous(), trans.contiguous()
        alpha, phi = alpha.contiguous(), phi.contiguous()
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        md = plan.model_struct(mode, alpha, phi)
        E = int(type_.shape[0])
        dev = rot.device
        u = torch.empty((3, E, plan.N), dtype=torch.float32, device=dev)
        cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
        na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
        saved = _native.saved_buffer(plan, E)
        _native.etac_step(plan, sc, md, u, cobj, na, saved=saved)
        ctx.plan, ctx.mode = plan, int(mode)
        ctx.save_for_backward(n_obj, type_, shape, rot, trans, alpha, phi, saved)
        ctx.mark_non_differentiable(cobj, na)
        return u, cobj, na

    @staticmethod
    def backward(ctx, grad_u, _grad_cobj, _grad_na):
        n_obj, type_, shape, rot, trans, alpha, phi, saved = ctx.saved_tensors
        plan = ctx.plan
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        md = plan.model_struct(ctx.mode, alpha, phi)
        gu = grad_u.to(torch.float32).contiguous()
        grot = torch.empty_like(rot)
        gtr = torch.empty_like(trans)
        gal = torch.empty_like(alpha)
        gph = torch.empty_like(phi)
        _native.etac_step_backward(plan, sc, md, gu, grot, gtr, gal, gph, saved=saved)
        return None, None, None, None, grot, gtr, gal, gph, None


def etac_step(plan, n_obj, type_, shape, rot, trans, alpha, phi, mode=_native.ETAC_FULL):
    return ETacStep.apply(plan, n_obj, type_, shape, rot, trans, alpha, phi, mode)


class ETacMeshStep(torch.autograd.Function):
    """The step with triangle-mesh objects (and primitives) in the scene:
    etac_contact_mesh then etac_propagate forward; etac_propagate_backward
    then etac_contact_mesh_backward (reading contact_obj and the
    winning-triangle records) backward.  By default the backward runs the
    contact pass again, so that only the inputs and the pooling record are
    saved, as for ETacStep; with keep_contact=True the forward's contact_obj,
    u_hat and hit record (17 bytes per node) are saved instead and the
    backward skips that launch.  The plan needs ETAC_PLAN_BACKWARD."""

    @staticmethod
    def forward(ctx, plan, meshset, n_obj, type_, shape, rot, trans, alpha, phi, mode, keep_contact=False):
        rot, trans = rot.contiguous(), trans.contiguous()
        alpha, phi = alpha.contiguous(), phi.contiguous()
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        md = plan.model_struct(mode, alpha, phi)
        E = int(type_.shape[0])
        dev = rot.device
        cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
        uhat = torch.empty((3, E, plan.N), dtype=torch.float32, device=dev)
        na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
        hit = torch.empty((E, plan.N), dtype=torch.int32, device=dev)
        u = torch.empty((3, E, plan.N), dtype=torch.float32, device=dev)
        saved = _native.saved_buffer(plan, E)
        _native.etac_contact_mesh(plan, meshset, sc, cobj, uhat, na, hit)
        _native.etac_propagate(plan, md, E, cobj, uhat, u, saved=saved)
        ctx.plan, ctx.meshset, ctx.mode, ctx.keep = plan, meshset, int(mode), bool(keep_contact)
        if ctx.keep:
            ctx.save_for_backward(n_obj, type_, shape, rot, trans, alpha, phi, saved, cobj, uhat, hit)
        else:
            ctx.save_for_backward(n_obj, type_, shape, rot, trans, alpha, phi, saved)
        ctx.mark_non_differentiable(cobj, na)
        return u, cobj, na

    @staticmethod
    def backward(ctx, grad_u, _grad_cobj, _grad_na):
        n_obj, type_, shape, rot, trans, alpha, phi, saved = ctx.saved_tensors[:8]
        plan = ctx.plan
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        md = plan.model_struct(ctx.mode, alpha, phi)
        E = int(type_.shape[0])
        if ctx.keep:
            cobj, uhat, hit = ctx.saved_tensors[8:]
        else:
            dev = rot.device
            cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
            uhat = torch.empty((3, E, plan.N), dtype=torch.float32, device=dev)
            na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
            hit = torch.empty((E, plan.N), dtype=torch.int32, device=dev)
            _native.etac_contact_mesh(plan, ctx.meshset, sc, cobj, uhat, na, hit)
        gu = grad_u.to(torch.float32).contiguous()
        guhat = torch.empty_like(uhat)
        gal = torch.empty_like(alpha)
        gph = torch.empty_like(phi)
        _native.etac_propagate_backward(plan, md, E, cobj, uhat, gu, guhat, gal, gph, saved=saved)
        grot = torch.empty_like(rot)
        gtr = torch.empty_like(trans)
        _native.etac_contact_mesh_backward(plan, ctx.meshset, sc, guhat, grot, gtr, cobj, hit)
        return None, None, None, None, None, grot, gtr, gal, gph, None, None


def etac_mesh_step(plan, meshset, n_obj, type_, shape, rot, trans, alpha, phi, mode=_native.ETAC_FULL,
                   keep_contact=False):
    return ETacMeshStep.apply(plan, meshset, n_obj, type_, shape, rot, trans, alpha, phi, mode, keep_contact)


class ETacHandStep(torch.autograd.Function):
    """The articulated-hand step (plan with etac_plan_set_hand): contact with
    the objects and the other links in each patch's link frame, then Eqs.
    1-2.  Returns (u [3][E][N] in the link frames, contact_obj, n_active,
    r_contact [E]); gradients flow to the object poses, the link poses
    [E][L][9], [E][L][3], alpha and phi.  The backward recomputes contact and
    reads the forward's pooling record."""

    @staticmethod
    def forward(ctx, plan, n_obj, type_, shape, rot, trans, link_rot, link_trans, alpha, phi, mode, omega_a=1.0):
        rot, trans = rot.contiguous(), trans.contiguous()
        link_rot, link_trans = link_rot.contiguous(), link_trans.contiguous()
        alpha, phi = alpha.contiguous(), phi.contiguous()
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        lk = plan.links_struct(link_rot, link_trans)
        md = plan.model_struct(mode, alpha, phi)
        E = int(type_.shape[0])
        dev = rot.device
        u = torch.empty((3, E, plan.N), dtype=torch.float32, device=dev)
        cobj = torch.empty((E, plan.N), dtype=torch.int8, device=dev)
        na = torch.empty((E, plan.K), dtype=torch.int32, device=dev)
        r = torch.empty((E,), dtype=torch.float32, device=dev)
        rw = plan.reward_struct(E, omega_a, r_contact=r)
        saved = _native.saved_buffer(plan, E)
        _native.etac_hand_step(plan, sc, lk, md, u, cobj, na, rw, saved=saved)
        ctx.plan, ctx.mode = plan, int(mode)
        ctx.save_for_backward(n_obj, type_, shape, rot, trans, link_rot, link_trans, alpha, phi, saved)
        ctx.mark_non_differentiable(cobj, na, r)
        return u, cobj, na, r

    @staticmethod
    def backward(ctx, grad_u, _grad_cobj, _grad_na, _grad_r):
        n_obj, type_, shape, rot, trans, link_rot, link_trans, alpha, phi, saved = ctx.saved_tensors
        plan = ctx.plan
        sc = plan.scene_struct(n_obj, type_, shape, rot, trans)
        lk = plan.links_struct(link_rot, link_trans)
        md = plan.model_struct(ctx.mode, alpha, phi)
        gu = grad_u.to(torch.float32).contiguous()
        g = [torch.empty_like(x) for x in (rot, trans, link_rot, link_trans, alpha, phi)]
        _native.etac_hand_step_backward(plan, sc, lk, md, gu, *g, saved=saved)
        return (None, None, None, None) + tuple(g) + (None, None)


def etac_hand_step(plan, n_obj, type_, shape, rot, trans, link_rot, link_trans, alpha, phi, mode=_native.ETAC_FULL,
                   omega_a=1.0):
    return ETacHandStep.apply(plan, n_obj, type_, shape, rot, trans, link_rot, link_trans, alpha, phi, mode, omega_a)


def rotation_from_axis_angle(w):
    """Rodrigues' formula, differentiable: w [..., 3] -> row-major R [..., 9]."""
    th = torch.linalg.norm(w, dim=-1, keepdim=True).clamp_min(1e-12)
    k = w / th
    kx, ky, kz = k.unbind(-1)
    z = torch.zeros_like(kx)
    K = torch.stack([z, -kz, ky, kz, z, -kx, -ky, kx, z], dim=-1).reshape(*w.shape[:-1], 3, 3)
    eye = torch.eye(3, dtype=w.dtype, device=w.device).expand_as(K)
    s = torch.sin(th)[..., None]
    c = (1.0 - torch.cos(th))[..., None]
    R = eye + s * K + c * (K @ K)
    return R.reshape(*w.shape[:-1], 9)
