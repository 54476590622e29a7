"""Pins of the oracle's distance bounds against geometry and calculus.

Exact primitive distances vanish on surface points built from each shape's
parametrisation, equal hand-computed distances at chosen points, are
1-Lipschitz, and agree with a brute-force distance to a dense surface sample.
The network's input gradient is checked against central differences, and the
stored calibration against a recomputation.
"""
import json

import numpy as np
import pytest

import workloads as W
from oracle import sdb


def _one(ptype, centre, mat, params):
    return W._record(ptype, centre, mat, params)


def _surface_points(ptype, params, m=4000, seed=0):
    rng = np.random.default_rng(seed)
    u, v = rng.uniform(0, 2 * np.pi, m), rng.uniform(0, 2 * np.pi, m)
    if ptype == W.PRIM_SPHERE:
        d = rng.standard_normal((m, 3))
        return params[0] * d / np.linalg.norm(d, axis=1, keepdims=True)
    if ptype == W.PRIM_TORUS:
        R, r = params[0], params[1]
        return np.stack([(R + r * np.cos(v)) * np.cos(u), r * np.sin(v), (R + r * np.cos(v)) * np.sin(u)], axis=1)
    if ptype == W.PRIM_CAPSULE:
        a, r = params[0], params[1]
        d = rng.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        zc = rng.uniform(-a, a, m)
        p = r * d
        p[:, 2] += np.where(np.abs(d[:, 2]) > 0.99, np.sign(d[:, 2]) * a, zc * 0)
        # points on the cylinder part
        cyl = np.stack([r * np.cos(u), r * np.sin(u), zc], axis=1)
        caps = r * d + np.stack([np.zeros(m), np.zeros(m), np.sign(d[:, 2]) * a], axis=1)
        return np.concatenate([cyl, caps])
    if ptype == W.PRIM_BOX:
        b = np.asarray(params)
        p = rng.uniform(-1, 1, (m, 3)) * b
        ax = rng.integers(0, 3, m)
        p[np.arange(m), ax] = np.sign(rng.standard_normal(m)) * b[ax]
        return p
    raise ValueError


@pytest.mark.parametrize("ptype,params", [(W.PRIM_SPHERE, (0.3, 0, 0)), (W.PRIM_TORUS, (0.25, 0.07, 0)),
                                          (W.PRIM_CAPSULE, (0.2, 0.08, 0)), (W.PRIM_BOX, (0.1, 0.2, 0.15))])
def test_primitive_zero_on_its_surface(ptype, params):
    rec = _one(ptype, (0, 0, 0), np.eye(3), params)
    P = _surface_points(ptype, np.asarray(rec[13:16], dtype=np.float64))
    np.testing.assert_allclose(sdb.prim_f64(rec, P), 0.0, atol=1e-12)


def test_primitive_known_values():
    box = _one(W.PRIM_BOX, (0, 0, 0), np.eye(3), (0.5, 0.25, 0.125))
    P = np.array([[1.5, 0, 0], [1.5, 1.25, 0], [0, 0, 0], [0.4, 0, 0], [1.5, 1.25, 1.125]])
    np.testing.assert_allclose(sdb.prim_f64(box, P), [1.0, np.sqrt(2.0), -0.125, -0.1, np.sqrt(3.0)], atol=1e-7)
    bb = _one(W.PRIM_BOXBOUND, (0, 0, 0), np.eye(3), (0.5, 0.25, 0.125))
    np.testing.assert_allclose(sdb.prim_f64(bb, P), [1.0, 1.0, -0.125, -0.1, 1.0], atol=1e-7)
    tor = _one(W.PRIM_TORUS, (0, 0, 0), np.eye(3), (0.5, 0.1, 0))
    np.testing.assert_allclose(sdb.prim_f64(tor, np.array([[0.5, 0, 0], [0, 0, 0], [0, 0.3, 0.5]])),
                               [-0.1, 0.4, 0.2], atol=1e-7)
    cap = _one(W.PRIM_CAPSULE, (0, 0, 0), np.eye(3), (0.5, 0.1, 0))
    np.testing.assert_allclose(sdb.prim_f64(cap, np.array([[0, 0, 1.0], [0.3, 0, 0.2], [0, 0.4, -0.5], [0, 0.3, -0.9]])),
                               [0.4, 0.2, 0.3, 0.5 - 0.1], atol=1e-7)
    pl = W.plane_scene((0, 0, 2.0), 0.25)[0]
    np.testing.assert_allclose(sdb.prim_f64(pl, np.array([[0.3, 0.1, 1.0]])), [0.75], atol=1e-7)


def test_rotation_and_translation():
    rng = np.random.default_rng(1)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    M = W._quat_to_local(q)
    assert np.allclose(M @ M.T, np.eye(3)) and np.isclose(np.linalg.det(M), 1.0)
    c = np.array([0.1, -0.2, 0.3])
    moved = _one(W.PRIM_TORUS, c, M, (0.3, 0.05, 0))
    base = _one(W.PRIM_TORUS, (0, 0, 0), np.eye(3), (0.3, 0.05, 0))
    Q = rng.uniform(-1, 1, (500, 3))
    world = Q @ np.asarray(moved[4:13], dtype=np.float64).reshape(3, 3) + np.asarray(moved[1:4], dtype=np.float64)
    np.testing.assert_allclose(sdb.prim_f64(moved, world), sdb.prim_f64(base, Q), atol=1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_csg_union_is_one_lipschitz_and_a_bound(seed):
    recs = W.csg_scene(seed)
    rng = np.random.default_rng(seed)
    A, B = rng.uniform(-1, 1, (20000, 3)), rng.uniform(-1, 1, (20000, 3))
    fa, fb = sdb.union_f64(recs, A), sdb.union_f64(recs, B)
    assert np.all(np.abs(fa - fb) <= np.linalg.norm(A - B, axis=1) * (1 + 1e-12) + 1e-15)


def test_exact_distance_matches_brute_force_surface_sample():
    rec = _one(W.PRIM_TORUS, (0, 0, 0), np.eye(3), (0.3, 0.1, 0))
    R, r = 0.3, 0.1
    u, v = np.meshgrid(np.linspace(0, 2 * np.pi, 600), np.linspace(0, 2 * np.pi, 300))
    S = np.stack([(R + r * np.cos(v)) * np.cos(u), r * np.sin(v), (R + r * np.cos(v)) * np.sin(u)], -1).reshape(-1, 3)
    from scipy.spatial import cKDTree
    P = np.random.default_rng(3).uniform(-0.6, 0.6, (300, 3))
    d = cKDTree(S).query(P)[0]
    np.testing.assert_allclose(np.abs(sdb.prim_f64(rec, P)), d, atol=3e-3)


def test_features_layout():
    om = W.fourier_omegas(2)
    g = sdb.features_f64(np.array([[0.0, 0.0, 0.0], [0.5, -0.25, 1.0]]), om)
    assert g.shape == (2, 15)
    np.testing.assert_allclose(g[0], [0, 0, 0, 0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1])
    np.testing.assert_allclose(g[1, 9:12], np.sin(om[1] * np.array([0.5, -0.25, 1.0])), rtol=1e-6)
    assert np.isclose(om[1], 2 ** 0.25, rtol=1e-7) and len(W.fourier_omegas()) == 16


def test_network_forward_matches_neuron_loop():
    net = W.mlp_net(5, width=8, depth=2, n_freq=2)
    net["biases"] = [b + np.float32(0.1 * (i + 1)) for i, b in enumerate(net["biases"])]
    p = np.array([[0.2, -0.7, 0.4]])
    a = list(sdb.features_f64(p, net["omegas"])[0])
    for l, (Wm, bv) in enumerate(zip(net["weights"], net["biases"])):
        z = [sum(float(Wm[o, i]) * a[i] for i in range(len(a))) + float(bv[o]) for o in range(Wm.shape[0])]
        a = [np.log1p(np.exp(x)) for x in z] if l < len(net["weights"]) - 1 else z
    assert np.isclose(sdb.mlp_forward_f64(net, p)[0], a[0], rtol=1e-12)


def test_network_input_gradient_matches_differences():
    net = W.mlp_net(3, width=32, depth=3, n_freq=4)
    P = np.random.default_rng(0).uniform(-1, 1, (16, 3))
    g = sdb.mlp_input_grad_f64(net, P)
    eps = 1e-6
    for ax in range(3):
        d = np.zeros(3)
        d[ax] = eps
        fd = (sdb.mlp_forward_f64(net, P + d) - sdb.mlp_forward_f64(net, P - d)) / (2 * eps)
        np.testing.assert_allclose(g[:, ax], fd, rtol=1e-6, atol=1e-8)


def test_stored_calibration_matches_recomputation():
    key = "seed0_w64_d4_f16"
    with open(W.neural_calibration_path()) as fh:
        stored = json.load(fh)[key]
    net = W.mlp_net(0, 64, 4, 16)
    c = sdb.calibrate_network(net, W.probe_points(), W.NEURAL_AMPLITUDE, W.NEURAL_R0)
    for k in ("S", "mu_u", "sigma_u", "L_hat"):
        assert np.isclose(c[k], stored[k], rtol=1e-9), k
    # S is the product of spectral norms: check one by power iteration
    Wm = np.asarray(net["weights"][1], dtype=np.float64)
    v = np.ones(Wm.shape[1])
    for _ in range(500):
        v = Wm.T @ (Wm @ v)
        v /= np.linalg.norm(v)
    s1 = np.linalg.norm(Wm @ v)
    assert np.isclose(np.linalg.svd(Wm, compute_uv=False)[0], s1, rtol=1e-6)


def test_neural_bound_is_contracting():
    # f = g/(lambda L): on random pairs, |f(p) - f(q)| <= |p - q| / lambda (up to sampling)
    S = sdb.SDB.neural(W.neural_scene(0, 64))
    rng = np.random.default_rng(11)
    A = rng.uniform(-1, 1, (4000, 3))
    B = A + rng.normal(0, 0.02, (4000, 3))
    ratio = np.abs(S.f64(A) - S.f64(B)) / np.linalg.norm(A - B, axis=1)
    assert ratio.max() < 1.0 / W.NEURAL_LAMBDA * 1.05
    # the surface exists: both signs occur inside the cube
    f = S.f64(rng.uniform(-1, 1, (20000, 3)))
    assert 0.02 < (f < 0).mean() < 0.2


def test_literal_reading_has_no_surface():
    # NN/prod(sigma) - 0.2 on [-1,1]^3 is negative everywhere: the reading
    # with a sphere prior is needed for a non-empty mesh
    net = W.mlp_net(0, 256, 4, 16)
    S = np.prod([np.linalg.svd(np.asarray(Wm, dtype=np.float64), compute_uv=False)[0] for Wm in net["weights"]])
    P = np.random.default_rng(0).uniform(-1, 1, (4000, 3))
    f = sdb.mlp_forward_f64(net, P) / S - 0.2
    assert f.max() < 0


def test_relu_network_closed_form():
    # A ReLU layer whose units are +-p_x, +-p_y, +-p_z summed by the output
    # layer is the L1 norm |x| + |y| + |z|, with gradient sign(p) (the
    # activation of the paper's networks, Section 5.2).
    W1 = np.zeros((8, 3), np.float32)
    for u, (axis, sign) in enumerate([(0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1)]):
        W1[u, axis] = sign
    W2 = np.array([[1, 1, 1, 1, 1, 1, 0, 0]], np.float32)
    net = {"omegas": np.zeros(0, np.float32), "weights": [W1, W2],
           "biases": [np.zeros(8, np.float32), np.zeros(1, np.float32)], "activation": "relu"}
    P = np.random.default_rng(4).uniform(-1, 1, (1000, 3))
    np.testing.assert_allclose(sdb.mlp_forward_f64(net, P), np.abs(P).sum(axis=1), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(sdb.mlp_input_grad_f64(net, P), np.sign(P))
    # the same weights under softplus are not piecewise linear
    soft = dict(net, activation="softplus")
    assert np.abs(sdb.mlp_forward_f64(soft, P) - np.abs(P).sum(axis=1)).min() > 1.0


def test_paper_network_shape():
    # eight ReLU layers of width 64 on the raw coordinates: about 30,000
    # weights (Section 5.2)
    net = W.paper_net_scene()
    assert net["activation"] == "relu" and len(net["omegas"]) == 0
    assert [w.shape for w in net["weights"]] == [(64, 3)] + [(64, 64)] * 7 + [(1, 64)]
    assert sum(w.size for w in net["weights"]) == 28928


def _both(recs, P):
    """The oracle's FP64 value and its FP32 twin at the points P."""
    P = np.asarray(P, dtype=np.float64)
    f64 = sdb.union_f64(recs, P)
    f32 = sdb.union_f32(recs, *[P[:, i].astype(np.float32) for i in range(3)]).astype(np.float64)
    return f64, f32


def test_cylinder_closed_forms():
    # capped cylinder r = 0.3, a = 0.2 about z: radial, axial and rim
    # distances outside, the nearer of side and cap inside
    recs = W.cylinder_scene(0.3, 0.2)
    P = [(0.5, 0, 0), (0, 0, 0.5), (0.5, 0, 0.5), (0, 0, 0), (0.1, 0, 0.1), (0, -0.7, -0.05)]
    exp = [0.2, 0.3, np.hypot(0.2, 0.3), -0.2, -0.1, 0.4]
    for f in _both(recs, P):
        np.testing.assert_allclose(f, exp, atol=1e-6)


def test_cone_closed_forms():
    # apex at z = 0.2, half-angle 30 degrees, cut at z = -0.2
    recs = W.cone_scene(0.2, np.pi / 6)
    s, c = 0.5, np.sqrt(3) / 2
    P = [(0, 0, 0), (0, 0, 0.3), (0.5, 0, 0), (0, 0, -0.5), (0.05, 0, -0.1)]
    exp = [-0.2 * s,                 # on the axis: distance to the side line
           0.1,                      # above the apex: distance to the apex
           0.5 * c - 0.2 * s,        # beside it: perpendicular to the side
           0.3,                      # below the base: distance to the base plane
           max(0.05 * c - 0.3 * s, -0.1)]
    for f in _both(recs, P):
        np.testing.assert_allclose(f, exp, atol=1e-6)


def test_hexprism_closed_forms():
    # apothem 0.2, half-length 0.3: along a face normal the bound is the exact
    # distance |p| - r; towards a vertex (the local y axis) it is
    # |p| cos 30 - r, below the exact |p| - r / cos 30
    recs = W.hexprism_scene(0.2, 0.3)
    P = [(0.5, 0, 0), (0.25, 0.25 * np.sqrt(3), 0), (0, 0.5, 0), (0, 0, 0.4), (0, 0, 0)]
    exp = [0.3, 0.3, 0.5 * np.sqrt(3) / 2 - 0.2, 0.1, -0.2]
    for f in _both(recs, P):
        np.testing.assert_allclose(f, exp, atol=1e-6)
    assert exp[2] < 0.5 - 0.2 / (np.sqrt(3) / 2)


def test_new_primitives_are_distance_bounds():
    # |f| <= distance to the zero set, sampled: the zero set is located on
    # segments from each inside point to far outside points by bisection (to
    # 2^-59), and every sample's |f| must not exceed its distance to those
    # points, which is at least its distance to the zero set; a bound 1 %
    # too large (the planted mistake) fails on every shape
    rng = np.random.default_rng(7)
    for recs in (W.cylinder_scene(0.3, 0.2), W.cone_scene(0.25, 0.5), W.hexprism_scene(0.2, 0.3)):
        inside = np.zeros((1, 3))
        dirs = rng.standard_normal((4000, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        lo_t, hi_t = np.zeros(len(dirs)), np.full(len(dirs), 2.0)
        for _ in range(60):
            mid = 0.5 * (lo_t + hi_t)
            neg = sdb.union_f64(recs, inside + mid[:, None] * dirs) < 0
            lo_t, hi_t = np.where(neg, mid, lo_t), np.where(neg, hi_t, mid)
        surf = inside + lo_t[:, None] * dirs
        Q = rng.uniform(-1, 1, (3000, 3))
        f = sdb.union_f64(recs, Q)
        dist = np.min(np.linalg.norm(Q[:, None, :] - surf[None, :, :], axis=2), axis=1)
        assert np.all(np.abs(f) <= dist + 1e-12), np.max(np.abs(f) - dist)
        assert np.any(np.abs(1.01 * f) > dist + 1e-12)


def test_genus2_function_and_bound():
    # the polynomial of the paper's genus-2 surface (Section 5.1) at points
    # worked by hand: F(0,0,0) = 1, F(1,0,0) = 2, zeros at (0,-1,0) (z = 0
    # leaves y^4 + 2y^3 + 1, zero at y = -1) and at the poles (0,0,+-1)
    x = np.array([0.0, 1.0, 0.0, 0.0, 0.0])
    y = np.array([0.0, 0.0, -1.0, 0.0, 0.0])
    z = np.array([0.0, 0.0, 0.0, 1.0, -1.0])
    np.testing.assert_array_equal(sdb.genus2_f64(x, y, z), [1.0, 2.0, 0.0, 0.0, 0.0])
    # the gradient bound holds over the cube (central differences at random
    # points and at the corners, where the quartic terms peak)
    B = 2.2
    rng = np.random.default_rng(11)
    P = np.concatenate([rng.uniform(-B, B, (200000, 3)),
                        np.array(np.meshgrid(*3 * [[-B, B]], indexing="ij")).reshape(3, -1).T])
    e = 1e-6
    g = np.stack([(sdb.genus2_f64(*(P + e * np.eye(3)[i]).T) - sdb.genus2_f64(*(P - e * np.eye(3)[i]).T)) / (2 * e)
                  for i in range(3)], axis=1)
    L = sdb.genus2_gradient_bound(B)
    assert np.linalg.norm(g, axis=1).max() <= L
    # the scene's factor is 1 / (s L) over the cube holding the grid's local points
    rec = W.genus2_scene()[0]
    s = W.GENUS2_SCALE
    Bg = s * (1.0 + W.GENUS2_CENTRE[1])
    assert np.isclose(float(rec[13]), 1.0 / (s * sdb.genus2_gradient_bound(Bg)), rtol=1e-6)
    # which makes it 1-Lipschitz on the grid: |f(q)| <= |f(z)| + |q - z| for
    # sampled points z where f nearly vanishes
    S = sdb.SDB.prims(W.genus2_scene())
    Q = rng.uniform(-1, 1, (20000, 3))
    f = S.f64(Q)
    near = np.abs(f) < 2e-5
    zeros, fz = Q[near], np.abs(f[near])
    assert len(zeros) > 10
    for q, v in zip(Q[:500], f[:500]):
        assert abs(v) <= (np.linalg.norm(zeros - q, axis=1) + fz).min() + 1e-12
