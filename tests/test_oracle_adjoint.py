"""Pins of the oracle's adjoint: the analytic FP64 gradient of the vertex
loss against central finite differences of the loss itself (mesh topology
and nearest targets fixed), on single coordinates of every layer and on
random directions; and the VJP of the network against differences."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import hop as ohop
from oracle import sdb as osdb


@pytest.fixture(scope="module")
def case():
    net = W.mlp_net(0, width=32, depth=2, n_freq=4)
    net.update({"r0": np.float32(0.5), "a_s": np.float32(0.6), "a_n": np.float32(0.08), "b": np.float32(-0.01)})
    n, lo, h = W.grid(24)
    mesh = ohop.gridhop(osdb.SDB.neural(net), n, lo, h).mesh
    targets = W.loss_targets(seed=1, n=512).astype(np.float64)
    L, grad, nearest = oadj.adjoint(net, mesh, targets)
    return net, mesh, targets, L, grad, nearest


def test_mesh_is_nontrivial(case):
    net, mesh, targets, L, grad, nearest = case
    assert len(mesh.edge_ids) > 300 and L > 0


def test_vjp_matches_differences():
    net = W.mlp_net(2, width=16, depth=2, n_freq=2)
    P = np.random.default_rng(0).uniform(-1, 1, (7, 3))
    gout = np.random.default_rng(1).standard_normal(7)
    g = oadj.mlp_vjp(net, P, gout)
    theta = oadj.flat_params(net)
    rng = np.random.default_rng(2)
    for q in rng.choice(len(theta), 25, replace=False):
        e = np.zeros_like(theta)
        e[q] = 1e-6
        fp = osdb.mlp_forward_f64(oadj.with_params(net, theta + e), P) @ gout
        fm = osdb.mlp_forward_f64(oadj.with_params(net, theta - e), P) @ gout
        assert np.isclose(g[q], (fp - fm) / 2e-6, rtol=1e-5, atol=1e-9)


def test_gradient_matches_central_differences_per_coordinate(case):
    net, mesh, targets, L, grad, nearest = case
    theta = oadj.flat_params(net)
    rng = np.random.default_rng(4)
    # coordinates from every block (weights and biases of each layer)
    sizes = [np.asarray(x).size for pair in zip(net["weights"], net["biases"]) for x in pair]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    picks = [s + rng.integers(0, z) for s, z in zip(starts, sizes) for _ in range(3)]
    checked = 0
    for q in picks:
        d = np.zeros_like(theta)
        d[q] = 1.0
        fd = oadj.central_difference(net, mesh, targets, nearest, d, 1e-6 * max(1.0, abs(theta[q])))
        if fd is None:
            continue
        checked += 1
        assert abs(fd - grad[q]) <= 1e-6 * max(1e-3, np.abs(grad).max()) + 1e-5 * abs(grad[q]), (q, fd, grad[q])
    assert checked >= len(picks) - 2


def test_gradient_matches_central_differences_on_directions(case):
    net, mesh, targets, L, grad, nearest = case
    rng = np.random.default_rng(5)
    for _ in range(4):
        d = rng.standard_normal(len(grad))
        d /= np.linalg.norm(d)
        fd = oadj.central_difference(net, mesh, targets, nearest, d, 1e-6)
        assert fd is not None
        assert abs(fd - grad @ d) <= 1e-5 * np.linalg.norm(grad)


def test_loss_gradient_wrt_vertices():
    # dL/dv of the loss itself against differences
    n, lo, h = 8, -1.0, 0.25
    eids = np.array([3 * ((2 * 9 + 3) * 9 + 4) + 1, 3 * ((5 * 9 + 1) * 9 + 2) + 2])
    fa, fb = np.array([-0.3, 0.2]), np.array([0.5, -0.7])
    tg = np.random.default_rng(0).uniform(-1, 1, (20, 3))
    L, g, near = oadj.vertex_loss(n, lo, h, eids, fa, fb, tg)
    eps = 1e-7
    fa2 = fa.copy()
    fa2[0] += eps
    L2, _, _ = oadj.vertex_loss(n, lo, h, eids, fa2, fb, tg, near)
    # dL/dfa_0 = g[0, axis] * h * dt/dfa
    dt = -fb[0] / (fa[0] - fb[0]) ** 2
    assert np.isclose((L2 - L) / eps, g[0, 1] * h * dt, rtol=1e-5)
