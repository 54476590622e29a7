"""Pins of the oracle's Sierpinski tetrahedron bound (Section 5.1's fractal
scene; the paper gives no formula, so the pins come from the geometry).

S_d is the union of 4^d tetrahedra, listed here by brute force.  The
function must be negative exactly inside them, and its magnitude must equal
the distance to the boundary of the union, the least point-triangle distance
over all their faces (it is the exact signed distance, not only a bound).
The closed forms: at the centroid, depth 0 gives minus the inradius of T
(1/sqrt 3), depth 1 the inradius of the octahedral hole |x| + |y| + |z| <= 1
(1/sqrt 3 again, with the opposite sign); beyond a vertex on its axis the
distance is to that vertex at every depth."""
import numpy as np
import pytest

from oracle import sdb as S

V = S.TETRA_V


def tetrahedra(depth):
    """Vertex arrays (4 x 3) of the 4^depth tetrahedra of S_depth."""
    out = [V.copy()]
    for _ in range(depth):
        out = [(t + v) / 2.0 for t in out for v in V]
    return out


def barycentric(P, T):
    A = np.stack([T[1] - T[0], T[2] - T[0], T[3] - T[0]], axis=1)
    lam = np.linalg.solve(A, (P - T[0]).T).T
    return np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)


def seg_dist(P, A, B):
    d = B - A
    t = np.clip((P - A) @ d / (d @ d), 0.0, 1.0)
    return np.linalg.norm(P - (A + t[:, None] * d), axis=1)


def tri_dist(P, A, B, C):
    """Exact distance from points P to the triangle ABC."""
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    h = (P - A) @ n
    Q = P - h[:, None] * n
    v0, v1, v2 = B - A, C - A, Q - A
    d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
    d20, d21 = v2 @ v0, v2 @ v1
    den = d00 * d11 - d01 * d01
    b = (d11 * d20 - d01 * d21) / den
    c = (d00 * d21 - d01 * d20) / den
    inside = (b >= 0) & (c >= 0) & (b + c <= 1)
    edge = np.minimum(np.minimum(seg_dist(P, A, B), seg_dist(P, B, C)), seg_dist(P, C, A))
    return np.where(inside, np.abs(h), edge)


def exact(P, depth):
    """Membership and the exact distance to the boundary of S_depth.  The
    tetrahedra meet only at points, so inside one of them the boundary's
    nearest point is on its own faces."""
    inside = np.zeros(len(P), bool)
    dist = np.full(len(P), np.inf)
    margin = np.full(len(P), np.inf)
    for T in tetrahedra(depth):
        lam = barycentric(P, T)
        ins = lam.min(axis=1) > 0
        margin = np.minimum(margin, np.abs(lam).min(axis=1))
        for f in range(4):
            A, B, C = (T[k] for k in range(4) if k != f)
            dist = np.minimum(dist, tri_dist(P, A, B, C))
        inside |= ins
    return inside, dist, margin


def points(depth, rng, n=1500):
    """Uniform points around T and points just off the faces of S_depth."""
    P = [rng.uniform(-1.4, 1.4, (n, 3))]
    tets = tetrahedra(depth)
    for _ in range(n):
        T = tets[rng.integers(len(tets))]
        f = rng.integers(4)
        A, B, C = (T[k] for k in range(4) if k != f)
        u, v = rng.uniform(size=2)
        if u + v > 1:
            u, v = 1 - u, 1 - v
        n_ = np.cross(B - A, C - A)
        n_ /= np.linalg.norm(n_)
        P.append((A + u * (B - A) + v * (C - A) + rng.normal(0, 0.02) * n_)[None])
    return np.concatenate(P)


@pytest.mark.parametrize("depth", [0, 1, 2, 3])
def test_sign_is_membership_and_magnitude_is_distance(depth):
    rng = np.random.default_rng(depth)
    P = points(depth, rng)
    inside, dist, margin = exact(P, depth)
    f = S.sierpinski_f64(P, depth)
    ok = margin > 1e-9                        # not on a face of a tetrahedron
    assert np.array_equal(f[ok] < 0, inside[ok])
    np.testing.assert_allclose(np.abs(f), dist, rtol=0, atol=1e-12)


def test_tighter_than_hull_bounds():
    """The nearest copy's bound is at least the hull bound of that copy
    (its recursion ends in a smaller tetrahedron inside the hull)."""
    rng = np.random.default_rng(7)
    P = rng.uniform(-1.4, 1.4, (4000, 3))
    for d in (1, 3):
        b = np.argmax(P @ V.T, axis=1)
        hull = 0.5 * S.tetra_bound_f64(2 * P - V[b])
        assert np.all(S.sierpinski_f64(P, d) >= hull - 1e-12)


def test_closed_forms_at_the_centroid():
    o = np.zeros((1, 3))
    assert S.sierpinski_f64(o, 0)[0] == pytest.approx(-1 / np.sqrt(3), abs=1e-15)
    assert S.sierpinski_f64(o, 1)[0] == pytest.approx(1 / np.sqrt(3), abs=1e-15)
    # the octahedral hole's inradius is the exact distance at depth 1
    inside, dist, _ = exact(o, 1)
    assert not inside[0] and dist[0] == pytest.approx(1 / np.sqrt(3), abs=1e-12)


def test_distance_beyond_a_vertex():
    for d in range(6):
        for i in range(4):
            t = 2.0 / 3.0 + np.arange(1, 4)[:, None]      # points v_i (1 + k/3 ...), off T on the axis
            f = S.sierpinski_f64(t * V[i], d)
            np.testing.assert_allclose(f, (t[:, 0] - 1) * np.sqrt(3.0), rtol=1e-13)


def test_vertices_are_fixed_points():
    """Each vertex of T is in every S_d (the copy at it holds it again), so
    the bound is 0 there, and small and negative just inside along the
    median."""
    for d in range(5):
        f = S.sierpinski_f64(V, d)
        assert np.all(np.abs(f) < 1e-12)
        g = S.sierpinski_f64(V * (1 - 1e-3), d)
        assert np.all(g < 0) and np.all(g > -1e-3)


def _tie_gap(P, depth):
    """The smallest gap between the two largest v_i . q over the levels: a
    point with a tiny gap may take another copy in float32."""
    q = np.asarray(P, dtype=np.float64).copy()
    gap = np.full(len(q), np.inf)
    for _ in range(depth):
        d = np.sort(q @ V.T, axis=1)
        gap = np.minimum(gap, d[:, 3] - d[:, 2])
        q = 2 * q - V[np.argmax(q @ V.T, axis=1)]
    return gap


@pytest.mark.parametrize("depth", [0, 2, 6])
def test_fp32_twin_within_rounding(depth):
    rng = np.random.default_rng(10 + depth)
    P = rng.uniform(-1.3, 1.3, (20000, 3))
    a = S.sierpinski_f64(P, depth)
    b = S.sierpinski_f32(*P.T.astype(np.float32), depth).astype(np.float64)
    ok = _tie_gap(P, depth) > 1e-4
    assert ok.mean() > 0.99
    assert np.abs(a - b)[ok].max() < 2e-6


def test_record_scales_by_k():
    rec = np.zeros(16)
    rec[0] = S.PRIM_SIERPINSKI
    rec[1:4] = (0.1, -0.2, 0.05)
    rec[4:13] = (1.25 * np.eye(3)).ravel()
    rec[13], rec[14] = 1 / 1.25, 3
    rng = np.random.default_rng(3)
    P = rng.uniform(-1, 1, (500, 3))
    ref = S.sierpinski_f64(1.25 * (P - rec[1:4]), 3) / 1.25
    np.testing.assert_allclose(S.prim_f64(rec, P), ref, rtol=0, atol=1e-15)
