"""Differentiable polygonization of a network bound.

GridHopMesh.apply(theta, net, n, lo, h, precision) returns the welded vertex
positions (V x 3) of the grid-hopping mesh of the network whose parameters
are the flat tensor theta (order W_0, b_0, W_1, b_1, ..., W_D, b_D).  Its
backward runs gh_backward: the edge-interpolation adjoint into the corner
values and the network's vector-Jacobian product, all in the library's
kernels.  The triangles (ctx.mesh.tris) are piecewise constant in theta.
"""
import numpy as np
import torch

from . import native as N
from .polygonize import Bound, Polygonizer


def unflatten(net, theta):
    """A copy of net with weights and biases read from the flat theta (host)."""
    t = theta.detach().cpu().numpy().astype(np.float32)
    ws, bs, o = [], [], 0
    for W, b in zip(net["weights"], net["biases"]):
        W = np.asarray(W)
        ws.append(t[o:o + W.size].reshape(W.shape))
        o += W.size
        bs.append(t[o:o + len(b)])
        o += len(b)
    if o != t.size:
        raise ValueError(f"theta has {t.size} entries, the network {o}")
    out = dict(net)
    out["weights"], out["biases"] = ws, bs
    return out


def flatten(net):
    parts = []
    for W, b in zip(net["weights"], net["biases"]):
        parts.append(np.asarray(W, dtype=np.float32).ravel())
        parts.append(np.asarray(b, dtype=np.float32).ravel())
    return np.concatenate(parts)


class GridHopMesh(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, net, n, lo, h, precision="fp32", margin=0.0):
        bound = Bound.mlp(unflatten(net, theta), precision, margin=margin, device=theta.device)
        poly = Polygonizer(bound, n, lo, h, device=theta.device)
        mesh = poly.run()
        ctx.poly, ctx.mesh, ctx.nparams = poly, mesh, theta.numel()
        ctx.mark_non_differentiable()
        return mesh.verts.clone()

    @staticmethod
    def backward(ctx, dverts):
        poly = ctx.poly
        desc = poly.bound.desc
        if N.gh_param_count(desc) != ctx.nparams:
            raise RuntimeError("parameter count mismatch")
        grad = torch.empty(ctx.nparams, dtype=torch.float32, device=dverts.device)
        bws = torch.empty(N.gh_backward_workspace_size(desc, poly.corner_cap), dtype=torch.uint8,
                          device=dverts.device)
        N.check(N.gh_backward(desc, poly.grid, poly.ws, poly.corner_cap, dverts.contiguous().float(), grad, bws,
                              poly.ctr), "gh_backward")
        return grad, None, None, None, None, None, None
