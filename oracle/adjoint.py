"""Gradient of a mesh-vertex loss with respect to the network's parameters,
FP64: the analytic adjoint and central finite differences.

Loss (the backward workload): L = (1/V) sum_v ||v - q(v)||^2 over the
welded vertices, q(v) the nearest of the target points, held fixed.

A vertex on lattice edge a -> b (axis e, length h) sits at
v = P_a + t h e with t = f_a/(f_a - f_b), so
  dt/df_a = -f_b/(f_a - f_b)^2,   dt/df_b = f_a/(f_a - f_b)^2,
and the cotangent of corner value f_c is the sum over the crossing edges
through c of (dL/dv . e) h dt/df_c.  With f = a_s(||p|| - r0) + a_n NN + b,
dL/dtheta = a_n sum_c gbar_c dNN(P_c)/dtheta, by back-propagation through
the network.  The candidate cells, case bytes and nearest targets are
piecewise constant in theta and get no gradient.

Parameter order (flat): W_0 (row-major, fan_out x fan_in), b_0, W_1, b_1,
..., W_D, b_D.
"""
import numpy as np
from scipy.spatial import cKDTree

from . import mc, sdb


def flat_params(net):
    out = []
    for W, b in zip(net["weights"], net["biases"]):
        out.append(np.asarray(W, dtype=np.float64).ravel())
        out.append(np.asarray(b, dtype=np.float64).ravel())
    return np.concatenate(out)


def with_params(net, theta):
    """A copy of net whose weights and biases are taken from the flat theta."""
    new = dict(net)
    ws, bs, o = [], [], 0
    for W, b in zip(net["weights"], net["biases"]):
        W = np.asarray(W)
        ws.append(theta[o:o + W.size].reshape(W.shape))
        o += W.size
        bs.append(theta[o:o + len(b)])
        o += len(b)
    new["weights"], new["biases"] = ws, bs
    return new


def edge_endpoints(n, edge_ids):
    """Lattice point ids (a, b) of each edge and its axis."""
    n1 = n + 1
    pid, axis = edge_ids // 3, edge_ids % 3
    step = np.array([n1 * n1, n1, 1])[axis]
    return pid, pid + step, axis


def point_coords(n, lo, h, pid):
    n1 = n + 1
    a, b, c = pid // (n1 * n1), (pid // n1) % n1, pid % n1
    return np.float64(lo) + np.stack([a, b, c], axis=1).astype(np.float64) * np.float64(h)


def vertex_loss(n, lo, h, edge_ids, fa, fb, targets, nearest=None):
    """L and dL/dv for vertices on the given edges with end values fa, fb."""
    pa, _, axis = edge_endpoints(n, edge_ids)
    t = fa / (fa - fb)
    V = point_coords(n, lo, h, pa)
    V[np.arange(len(t)), axis] += t * h
    if nearest is None:
        nearest = cKDTree(targets).query(V)[1]
    d = V - targets[nearest]
    L = (d * d).sum() / len(V)
    return L, 2.0 * d / len(V), nearest


def mlp_vjp(net, P, gout):
    """sum_i gout_i dNN(P_i)/dtheta, flat, by back-propagation (FP64)."""
    _, pres, acts = sdb.mlp_forward_f64(net, P, keep=True)
    Ws = [np.asarray(W, dtype=np.float64) for W in net["weights"]]
    grads = [None] * (2 * len(Ws))
    g = np.asarray(gout, dtype=np.float64)[:, None]          # dL/d(output), rows x 1
    for l in range(len(Ws) - 1, -1, -1):
        grads[2 * l] = g.T @ acts[l]                          # dW_l = g^T a_l
        grads[2 * l + 1] = g.sum(axis=0)
        if l > 0:
            g = (g @ Ws[l]) * sdb.activation_grad_f64(net, pres[l - 1])  # through the activation
    return np.concatenate([x.ravel() for x in grads])


def adjoint(net, mesh, targets):
    """(L, dL/dtheta) for a mesh from the oracle (its edge ids and corner values)."""
    n, lo, h = mesh.n, mesh.lo, mesh.h
    pa, pb, axis = edge_endpoints(n, mesh.edge_ids)
    corners = np.unique(np.concatenate([pa, pb]))
    fc = sdb.neural_f64(net, point_coords(n, lo, h, corners))
    fa, fb = fc[np.searchsorted(corners, pa)], fc[np.searchsorted(corners, pb)]
    L, dLdv, nearest = vertex_loss(n, lo, h, mesh.edge_ids, fa, fb, targets)
    den = (fa - fb) ** 2
    ge = dLdv[np.arange(len(fa)), axis] * h                   # dL/dt per vertex
    gbar = np.zeros(len(corners))
    np.add.at(gbar, np.searchsorted(corners, pa), ge * (-fb / den))
    np.add.at(gbar, np.searchsorted(corners, pb), ge * (fa / den))
    grad = np.float64(net["a_n"]) * mlp_vjp(net, point_coords(n, lo, h, corners), gbar)
    return L, grad, nearest


def loss_at(net, theta, mesh, targets, nearest):
    """L at parameters theta for the fixed edges and nearest targets of mesh;
    also the corner signs, which must not change for a valid difference."""
    n, lo, h = mesh.n, mesh.lo, mesh.h
    net2 = with_params(net, theta)
    pa, pb, _ = edge_endpoints(n, mesh.edge_ids)
    fa = sdb.neural_f64(net2, point_coords(n, lo, h, pa))
    fb = sdb.neural_f64(net2, point_coords(n, lo, h, pb))
    L, _, _ = vertex_loss(n, lo, h, mesh.edge_ids, fa, fb, targets, nearest)
    return L, np.concatenate([fa < 0, fb < 0])


def central_difference(net, mesh, targets, nearest, direction, step):
    """(L(theta + step d) - L(theta - step d)) / (2 step), or None when a corner
    sign flips between the two evaluations."""
    theta = flat_params(net)
    lp, sp = loss_at(net, theta + step * direction, mesh, targets, nearest)
    lm, sm = loss_at(net, theta - step * direction, mesh, targets, nearest)
    if not np.array_equal(sp, sm):
        return None
    return (lp - lm) / (2 * step)
