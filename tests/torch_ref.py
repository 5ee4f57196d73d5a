"""Independent float64 torch-CPU formulation of the ETac step, used only to
pin the oracle: its autograd (a library routine) checks the oracle's
hand-written adjoint, and its vectorised forward (cdist / matmul / amax)
checks the oracle's plain loops.  It shares no code with the oracle or the
GPU library."""
import numpy as np
import torch

from scenes import PHI_LAYERS, phi_offsets, SPHERE, BOX, CAPSULE, MODE_DECAY_ONLY, MODE_RESIDUAL_ONLY


def unpack_phi(phi):
    off = phi_offsets()
    out = {}
    for name, o, i in PHI_LAYERS:
        out[name] = phi[off[name]: off[name] + o * i].reshape(o, i)
        b = "b" + name[1:]
        out[b] = phi[off[b]: off[b] + o]
    return out


def primitive_disp(ptype, shape, R, t, p):
    """Closest-surface-point displacement of points p [n,3] that lie inside a
    primitive (torch float64, differentiable in R [3,3] and t [3]).  Returns
    (displacement [n,3], depth [n]); values are meaningful for inside points."""
    d = p - t
    shape = torch.as_tensor(np.asarray(shape, dtype=np.float64))
    if ptype == SPHERE:
        dist = torch.linalg.norm(d, dim=1, keepdim=True)
        return (shape[0] / dist - 1.0) * d, shape[0] - dist[:, 0]
    q = d @ R                                # q = R^T d per row
    if ptype == BOX:
        h = shape[:3]
        slack = h[None, :] - q.abs()
        face = torch.argmin(slack.detach(), dim=1)   # first minimum on ties
        qs = q.gather(1, face[:, None])[:, 0]
        hs = h[face]
        sg = torch.where(qs.detach() >= 0, 1.0, -1.0).to(q.dtype)
        col = R.T[face]                      # column face of R, per node
        return ((sg * hs - qs)[:, None]) * col, (hs - qs.abs())
    r, L = shape[0], shape[1]
    z = torch.clamp(q[:, 2], -L, L)
    v = torch.stack([q[:, 0], q[:, 1], q[:, 2] - z], dim=1)
    dist = torch.linalg.norm(v, dim=1, keepdim=True)
    w = v @ R.T                              # R v per row
    return (r / dist - 1.0) * w, r - dist[:, 0]


def propagate_env(pos, nrm, origin, offsets, alpha, phi, active, uhat, mode):
    """One env.  pos, nrm [N,3]; origin [K,3]; alpha [K]; phi packed; active
    bool [N]; uhat [N,3] (zero rows for passive nodes).  Returns U [N,3]."""
    W = unpack_phi(phi)
    out = []
    for k in range(len(offsets) - 1):
        sl = slice(int(offsets[k]), int(offsets[k + 1]))
        P, Nn, A, Uh = pos[sl], nrm[sl], active[sl], uhat[sl]
        n = P.shape[0]
        if not bool(A.any()):
            out.append(torch.zeros(n, 3, dtype=pos.dtype))
            continue
        Uin = torch.where(A[:, None], Uh, torch.zeros_like(Uh))
        res = torch.zeros(n, 3, dtype=pos.dtype)
        if mode != MODE_RESIDUAL_ONLY:
            Om = torch.exp(-alpha[k] * torch.cdist(P[~A], P[A]))     # (n-m) x m
            res = res.index_put((torch.nonzero(~A)[:, 0],), Om @ Uh[A])
        if mode != MODE_DECAY_ONLY:
            x = torch.cat([P - origin[k], Nn, Uin], dim=1)
            f = torch.relu(torch.relu(x @ W["W1"].T + W["b1"]) @ W["W2"].T + W["b2"])
            g = f.amax(dim=0)
            gp = torch.relu(W["W3"] @ g + W["b3"])
            z = torch.cat([f, gp[None, :].expand(n, -1)], dim=1)
            r = torch.relu(z @ W["W4"].T + W["b4"]) @ W["W5"].T + W["b5"]
            res = res + torch.where(A[:, None], torch.zeros_like(r), r)
        out.append(torch.where(A[:, None], Uh, res))
    return torch.cat(out, dim=0)


def t64(a, grad=False):
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=torch.float64, requires_grad=grad)
