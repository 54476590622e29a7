"""Signed distance bounds, FP64, with an FP32 twin.

An SDB f satisfies |f(x)| <= distance from x to the zero set of f, negative
inside (Section 1, Hart's definition).  A 1-Lipschitz function is one.

Primitive distances are written from geometry:
  sphere   ||q|| - r
  box      u = |q| - b:  ||max(u, 0)|| + min(max_i u_i, 0)     (exact distance)
  boxbound max_i u_i       the max over the six face planes (Section 4.2, eq. boxdist)
  torus    sqrt((sqrt(q_x^2 + q_z^2) - R)^2 + q_y^2) - r
  capsule  ||q - (0, 0, clamp(q_z, -a, a))|| - r
  plane    n . p - d       (Section 4.1, eq. plane)
  cylinder d = (rho - r, |q_z| - a), rho = ||(q_x, q_y)||:  ||max(d, 0)|| + min(max_i d_i, 0)
           (exact distance to the capped cylinder)
  cone     max(rho cos - (a - q_z) sin, |q_z| - a): the distance to the
           cone's side line through the apex (a bound, since it reaches
           the other nappe too) and to the slab of the caps, intersected
  hexprism max(|q . n_k| - r over the three face normals n_k = (1, 0),
           (1/2, sqrt3/2), (-1/2, sqrt3/2) in the local xy plane, |q_z| - a):
           the max of the eight face planes, like the box bound
  genus2   k F(q), F = 2y(y^2 - 3x^2)(1 - z^2) + (x^2 + y^2)^2 - (9z^2 - 1)(1 - z^2),
           the paper's implicit surface of genus 2; a bound once k makes the
           gradient at most 1 over the region evaluated (Lipschitz normalisation)
  sierpinski k S_d(q): a bound of the Sierpinski tetrahedron of depth d
           (Section 5.1's fractal scene); see `sierpinski_f64`
and combined by the minimum, which is the union of the shapes (Section 4.3).
The paper's first scene holds sphere, cube, cone, cylinder, torus,
hexagonal prism and capsule, each with a simple distance bound (Section 5.1).

The FP32 twin evaluates the same expressions in numpy float32 in a fixed
order, one rounding per operation and no fused multiply-add; numpy's float32
sqrt, division, min, max and abs are correctly rounded or exact.  The float32
op order is documented beside each twin function.
"""
import numpy as np

PRIM_SPHERE, PRIM_BOX, PRIM_TORUS, PRIM_CAPSULE, PRIM_PLANE, PRIM_BOXBOUND = 0, 1, 2, 3, 4, 5
PRIM_CYLINDER, PRIM_CONE, PRIM_HEXPRISM, PRIM_GENUS2, PRIM_SIERPINSKI = 6, 7, 8, 9, 10
SIERPINSKI_MAX_DEPTH = 16

# Vertices of the regular tetrahedron T of the Sierpinski record, in local
# coordinates (centroid at the origin, circumradius sqrt 3).
TETRA_V = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])


# ------------------------------------------------------------------------- FP64
def prim_f64(rec, P):
    """Distance bound of one primitive record at points P (n x 3), FP64."""
    rec = np.asarray(rec, dtype=np.float64)
    t = int(rec[0])
    c = rec[1:4]
    M = rec[4:13].reshape(3, 3)
    a0, a1, a2 = rec[13], rec[14], rec[15]
    if t == PRIM_PLANE:
        return P @ M[0] - a0
    q = (P - c) @ M.T
    if t == PRIM_SPHERE:
        return np.linalg.norm(q, axis=1) - a0
    if t == PRIM_BOX:
        u = np.abs(q) - np.array([a0, a1, a2])
        return np.linalg.norm(np.maximum(u, 0.0), axis=1) + np.minimum(u.max(axis=1), 0.0)
    if t == PRIM_BOXBOUND:
        u = np.abs(q) - np.array([a0, a1, a2])
        return u.max(axis=1)
    if t == PRIM_TORUS:
        ring = np.hypot(q[:, 0], q[:, 2]) - a0
        return np.hypot(ring, q[:, 1]) - a1
    if t == PRIM_CAPSULE:
        w = q.copy()
        w[:, 2] = q[:, 2] - np.clip(q[:, 2], -a0, a0)
        return np.linalg.norm(w, axis=1) - a1
    if t == PRIM_CYLINDER:
        d = np.stack([np.hypot(q[:, 0], q[:, 1]) - a0, np.abs(q[:, 2]) - a1], axis=1)
        return np.linalg.norm(np.maximum(d, 0.0), axis=1) + np.minimum(d.max(axis=1), 0.0)
    if t == PRIM_CONE:
        side = np.hypot(q[:, 0], q[:, 1]) * a2 - (a0 - q[:, 2]) * a1
        return np.maximum(side, np.abs(q[:, 2]) - a0)
    if t == PRIM_HEXPRISM:
        s3 = np.sqrt(3.0) / 2.0
        faces = [np.abs(q[:, 0]), np.abs(0.5 * q[:, 0] + s3 * q[:, 1]), np.abs(s3 * q[:, 1] - 0.5 * q[:, 0])]
        return np.maximum(np.max(np.stack(faces), axis=0) - a0, np.abs(q[:, 2]) - a1)
    if t == PRIM_GENUS2:
        return a0 * genus2_f64(q[:, 0], q[:, 1], q[:, 2])
    if t == PRIM_SIERPINSKI:
        return a0 * sierpinski_f64(q, int(a1))
    raise ValueError(f"unknown primitive type {t}")


def genus2_f64(x, y, z):
    """The implicit function of the paper's genus-2 surface (Section 5.1)."""
    return 2 * y * (y * y - 3 * x * x) * (1 - z * z) + (x * x + y * y) ** 2 - (9 * z * z - 1) * (1 - z * z)


def tetra_bound_f64(q):
    """The maximum of the signed distances to the four face planes of T: the
    face opposite v_i has outward unit normal -v_i / sqrt 3 and lies at
    distance 1 / sqrt 3 from the centroid.  Exact inside T (the distance to
    the nearest face) and below the distance outside, like the box bound of
    Section 4.2."""
    return ((-q @ TETRA_V.T) - 1.0).max(axis=1) / np.sqrt(3.0)


def _segment_distance_f64(P, A, B):
    d = B - A
    t = np.clip((P - A) @ d / (d @ d), 0.0, 1.0)
    return np.linalg.norm(P - (A + t[:, None] * d), axis=1)


def _triangle_distance_f64(P, A, B, C):
    """Distance from the points P to the triangle ABC: to its plane where the
    foot of the perpendicular falls inside it, else to the nearest edge."""
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    height = (P - A) @ n
    F = P - height[:, None] * n
    u, v, w = B - A, C - A, F - A
    uu, uv, vv, wu, wv = u @ u, u @ v, v @ v, w @ u, w @ v
    den = uu * vv - uv * uv
    beta = (vv * wu - uv * wv) / den
    gamma = (uu * wv - uv * wu) / den
    inside = (beta >= 0) & (gamma >= 0) & (beta + gamma <= 1)
    edges = np.minimum(np.minimum(_segment_distance_f64(P, A, B), _segment_distance_f64(P, B, C)),
                       _segment_distance_f64(P, C, A))
    return np.where(inside, np.abs(height), edges)


def tetra_distance_f64(q):
    """The signed distance to T: inside, minus the distance to the nearest
    face plane (the face-plane bound is exact there); outside, the distance
    to the nearest of the four faces."""
    q = np.asarray(q, dtype=np.float64)
    plane = tetra_bound_f64(q)
    faces = [_triangle_distance_f64(q, *[TETRA_V[k] for k in range(4) if k != f]) for f in range(4)]
    return np.where(plane <= 0.0, plane, np.min(np.stack(faces), axis=0))


def sierpinski_f64(q, depth):
    """The signed distance to the Sierpinski tetrahedron of depth d
    (Section 5.1, fourth scene; the paper gives no formula, this one is
    written from the geometry).  S_0 = T and S_d is the union of the four
    copies (S_{d-1} + v_i) / 2.  With b the vertex nearest to q (largest
    v_i . q, lowest i on ties):
        f_0(q) = the signed distance to T
        f_d(q) = f_{d-1}(2q - v_b) / 2
    i.e. the distance to the copy at v_b, scaled back.  That copy is the
    nearest of the four: the reflection in the bisector plane of v_b and v_j
    is a symmetry of S_{d-1} and of T that swaps the copies at v_b and v_j,
    and q lies on v_b's side, so every point of copy j has its mirror image
    in copy b at most as far from q.  Each copy lies on its own vertex's side
    of every bisector and meets it at one point, and the copies meet only at
    points, so a point inside S_d is inside copy b and the distance to the
    boundary of S_d is the distance to copy b's.  By induction f_d is the
    signed distance to S_d (a bound with equality)."""
    q = np.asarray(q, dtype=np.float64)
    scale = 1.0
    for _ in range(depth):
        b = np.argmax(q @ TETRA_V.T, axis=1)
        q = 2.0 * q - TETRA_V[b]
        scale *= 0.5
    return scale * tetra_distance_f64(q)


def genus2_gradient_bound(B):
    """An upper bound of |grad F| for the genus-2 function over the cube
    |x|, |y|, |z| <= B: each partial derivative, expanded into monomials,
    is at most the sum of its coefficients' magnitudes times B^degree,
      F_x = -12xy + 12xyz^2 + 4x^3 + 4xy^2              <= 12B^2 + 8B^3 + 12B^4
      F_y = 6y^2 - 6y^2z^2 - 6x^2 + 6x^2z^2 + 4x^2y + 4y^3 <= 12B^2 + 8B^3 + 12B^4
      F_z = -4y^3z + 12x^2yz - 20z + 36z^3               <= 20B + 36B^3 + 16B^4
    and |grad F| <= the norm of the three."""
    fx = 12 * B ** 2 + 8 * B ** 3 + 12 * B ** 4
    fz = 20 * B + 36 * B ** 3 + 16 * B ** 4
    return float(np.sqrt(2 * fx * fx + fz * fz))


def union_f64(recs, P):
    """Min-union of primitive records (Section 4.3), FP64."""
    P = np.asarray(P, dtype=np.float64)
    f = prim_f64(recs[0], P)
    for r in recs[1:]:
        f = np.minimum(f, prim_f64(r, P))
    return f


# ------------------------------------------------------------------ FP32 twin
def prim_f32(rec, x, y, z):
    """One primitive at float32 coordinate arrays, GPU op order.

    d = p - c;  q_r = (M_r0*d_x + M_r1*d_y) + M_r2*d_z for r = 0, 1, 2
    sphere:  sqrt((q_x*q_x + q_y*q_y) + q_z*q_z) - r
    box:     u_i = |q_i| - b_i;  m_i = max(u_i, 0)
             sqrt((m_x*m_x + m_y*m_y) + m_z*m_z) + min(max(u_x, max(u_y, u_z)), 0)
    boxbound max(u_x, max(u_y, u_z))
    torus:   s = sqrt(q_x*q_x + q_z*q_z) - R;  sqrt(s*s + q_y*q_y) - r
    capsule: w = q_z - min(max(q_z, -a), a);  sqrt((q_x*q_x + q_y*q_y) + w*w) - r
    plane:   ((n_x*x + n_y*y) + n_z*z) - d
    cylinder: rho = sqrt(q_x*q_x + q_y*q_y);  d_x = rho - r, d_z = |q_z| - a;
             m_i = max(d_i, 0);  sqrt(m_x*m_x + m_z*m_z) + min(max(d_x, d_z), 0)
    cone:    rho = sqrt(q_x*q_x + q_y*q_y);  max(rho*c - (a - q_z)*s, |q_z| - a)
    hexprism: h_x = 0.5*q_x, h_y = S*q_y with S = float32(sqrt(3)/2);
             max(|q_x| - r, max(|h_x + h_y| - r, max(|h_y - h_x| - r, |q_z| - a)))
    genus2:  x2 = q_x*q_x (y2, z2 alike), w = 1 - z2, r2 = x2 + y2;
             ((((2*q_y)*(y2 - 3*x2))*w + r2*r2) - (9*z2 - 1)*w) * k
    sierpinski: see `sierpinski_f32`
    """
    rec = np.asarray(rec, dtype=np.float32)
    t = int(rec[0])
    M = rec[4:13]
    a0, a1, a2 = rec[13], rec[14], rec[15]
    if t == PRIM_PLANE:
        return ((M[0] * x + M[1] * y) + M[2] * z) - a0
    dx, dy, dz = x - rec[1], y - rec[2], z - rec[3]
    qx = (M[0] * dx + M[1] * dy) + M[2] * dz
    qy = (M[3] * dx + M[4] * dy) + M[5] * dz
    qz = (M[6] * dx + M[7] * dy) + M[8] * dz
    if t == PRIM_SPHERE:
        return np.sqrt((qx * qx + qy * qy) + qz * qz) - a0
    if t in (PRIM_BOX, PRIM_BOXBOUND):
        ux, uy, uz = np.abs(qx) - a0, np.abs(qy) - a1, np.abs(qz) - a2
        inner = np.maximum(ux, np.maximum(uy, uz))
        if t == PRIM_BOXBOUND:
            return inner
        mx, my, mz = np.maximum(ux, np.float32(0)), np.maximum(uy, np.float32(0)), np.maximum(uz, np.float32(0))
        return np.sqrt((mx * mx + my * my) + mz * mz) + np.minimum(inner, np.float32(0))
    if t == PRIM_TORUS:
        s = np.sqrt(qx * qx + qz * qz) - a0
        return np.sqrt(s * s + qy * qy) - a1
    if t == PRIM_CAPSULE:
        w = qz - np.minimum(np.maximum(qz, -a0), a0)
        return np.sqrt((qx * qx + qy * qy) + w * w) - a1
    if t == PRIM_CYLINDER:
        rho = np.sqrt(qx * qx + qy * qy)
        dx, dz = rho - a0, np.abs(qz) - a1
        mx, mz = np.maximum(dx, np.float32(0)), np.maximum(dz, np.float32(0))
        return np.sqrt(mx * mx + mz * mz) + np.minimum(np.maximum(dx, dz), np.float32(0))
    if t == PRIM_CONE:
        rho = np.sqrt(qx * qx + qy * qy)
        return np.maximum(rho * a2 - (a0 - qz) * a1, np.abs(qz) - a0)
    if t == PRIM_HEXPRISM:
        hx, hy = np.float32(0.5) * qx, np.float32(np.sqrt(3.0) / 2.0) * qy
        u1, u2, u3 = np.abs(qx) - a0, np.abs(hx + hy) - a0, np.abs(hy - hx) - a0
        return np.maximum(u1, np.maximum(u2, np.maximum(u3, np.abs(qz) - a1)))
    if t == PRIM_GENUS2:
        x2, y2, z2 = qx * qx, qy * qy, qz * qz
        w = np.float32(1) - z2
        r2 = x2 + y2
        f = (((np.float32(2) * qy) * (y2 - np.float32(3) * x2)) * w + r2 * r2) - (np.float32(9) * z2 - np.float32(1)) * w
        return f * a0
    if t == PRIM_SIERPINSKI:
        return sierpinski_f32(qx, qy, qz, int(a1)) * a0
    raise ValueError(f"unknown primitive type {t}")


def sierpinski_f32(x, y, z, depth):
    """`sierpinski_f64` in float32 at local coordinates, GPU op order.  With
    u = x + y, w = x - y the four values e_i = -v_i . q are
    e_0 = -(u + z), e_1 = z - w, e_2 = w + z, e_3 = u - z; the nearest
    vertex is the least e_i (lowest i on ties).  Per level q = 2q - v_b (2q
    exact, one rounding per component).  At the last q, with the e_i sorted
    E1 >= E2 >= E3 >= E4, a = E1 - 1, c = E2 - 1 (a / sqrt 3 and c / sqrt 3
    are the two largest face-plane distances) and the nearest vertex v_b,
    the distance to T is
        a * float32(1/sqrt 3)                  if E1 + 3 E2 <= 4  (inside, or beyond one face)
        sqrt(0.375 (a a + c c) + 0.25 (a c))   if (E1 + E2) + 2 E3 <= 4  (beyond an edge)
        sqrt((d_x d_x + d_y d_y) + d_z d_z), d = q - v_b   otherwise (beyond a vertex)
    (the foot of the perpendicular on the nearest face plane lies in the
    face when every other face-plane distance is at most minus a third of
    it, the foot on the nearest edge's line lies on the edge when the third
    is at most minus half the sum of the first two; the faces' normals meet
    at cos = -1/3).  The result times 2^-d (exact) is returned for the
    caller's k."""
    x = np.asarray(x, dtype=np.float32).copy()
    y = np.asarray(y, dtype=np.float32).copy()
    z = np.asarray(z, dtype=np.float32).copy()
    V = TETRA_V.astype(np.float32)
    f = np.float32

    def es(x, y, z):
        u, w = x + y, x - y
        return np.stack([-(u + z), z - w, w + z, u - z])

    for _ in range(depth):
        b = np.argmin(es(x, y, z), axis=0)       # lowest index on ties
        x, y, z = f(2) * x - V[b, 0], f(2) * y - V[b, 1], f(2) * z - V[b, 2]
    e = es(x, y, z)
    E = np.sort(e, axis=0)
    E1, E2, E3 = E[3], E[2], E[1]
    b = np.argmin(e, axis=0)
    a, c = E1 - f(1), E2 - f(1)
    face = a * f(1.0 / np.sqrt(3.0))
    with np.errstate(invalid="ignore"):
        edge = np.sqrt(f(0.375) * (a * a + c * c) + f(0.25) * (a * c))
    dx, dy, dz = x - V[b, 0], y - V[b, 1], z - V[b, 2]
    vert = np.sqrt((dx * dx + dy * dy) + dz * dz)
    t = np.where(E1 + f(3) * E2 <= f(4), face, np.where((E1 + E2) + f(2) * E3 <= f(4), edge, vert))
    return t.astype(np.float32) * f(2.0 ** -depth)


def union_f32(recs, x, y, z):
    """Min-union in float32, primitives taken in record order."""
    x = np.asarray(x, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    z = np.asarray(z, dtype=np.float32)
    f = prim_f32(recs[0], x, y, z)
    for r in recs[1:]:
        f = np.minimum(f, prim_f32(r, x, y, z))
    return f


# ---------------------------------------------------------------------- network
def features_f64(P, omegas):
    """gamma(p) = [p, then per frequency: sin(w p_x,y,z), cos(w p_x,y,z)], FP64."""
    P = np.asarray(P, dtype=np.float64)
    cols = [P]
    for w in np.asarray(omegas, dtype=np.float64):
        cols.append(np.sin(w * P))
        cols.append(np.cos(w * P))
    return np.concatenate(cols, axis=1)


def softplus(x):
    """log(1 + e^x), evaluated stably."""
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def activation_f64(net, z):
    """The hidden layers' activation: softplus (default) or ReLU max(z, 0)."""
    return np.maximum(z, 0.0) if net.get("activation", "softplus") == "relu" else softplus(z)


def activation_grad_f64(net, z):
    """Its derivative: sigmoid for softplus, the step [z > 0] for ReLU."""
    return (z > 0).astype(np.float64) if net.get("activation", "softplus") == "relu" else sigmoid(z)


def mlp_forward_f64(net, P, keep=False):
    """Raw network output NN(gamma(p)) in FP64 (eq. nnsdb); optionally the
    pre-activations and activations of every layer."""
    a = features_f64(P, net["omegas"])
    acts, pres = [a], []
    Ws, bs = net["weights"], net["biases"]
    for l in range(len(Ws)):
        z = a @ np.asarray(Ws[l], dtype=np.float64).T + np.asarray(bs[l], dtype=np.float64)
        pres.append(z)
        a = activation_f64(net, z) if l < len(Ws) - 1 else z
        acts.append(a)
    out = a[:, 0]
    return (out, pres, acts) if keep else out


def mlp_input_grad_f64(net, P):
    """d NN(gamma(p)) / d p, FP64, by the chain rule through every layer."""
    P = np.asarray(P, dtype=np.float64)
    _, pres, acts = mlp_forward_f64(net, P, keep=True)
    Ws = [np.asarray(W, dtype=np.float64) for W in net["weights"]]
    g = np.ones((P.shape[0], 1))
    for l in range(len(Ws) - 1, -1, -1):
        g = g @ Ws[l]                      # d out / d a_{l}
        if l > 0:
            g = g * activation_grad_f64(net, pres[l - 1])
    # g = d out / d gamma; chain into p
    grad = g[:, 0:3].copy()
    for kk, w in enumerate(np.asarray(net["omegas"], dtype=np.float64)):
        gs = g[:, 3 + 6 * kk: 6 + 6 * kk]
        gc = g[:, 6 + 6 * kk: 9 + 6 * kk]
        grad += gs * w * np.cos(w * P) - gc * w * np.sin(w * P)
    return grad


def neural_f64(net, P):
    """f(p) = a_s (||p|| - r0) + a_n NN(gamma(p)) + b, FP64 with the stored coefficients."""
    P = np.asarray(P, dtype=np.float64)
    nn = mlp_forward_f64(net, P)
    return (np.float64(net["a_s"]) * (np.linalg.norm(P, axis=1) - np.float64(net["r0"]))
            + np.float64(net["a_n"]) * nn + np.float64(net["b"]))


# ------------------------------------------------------------------- dispatch
class SDB:
    """A distance bound with FP64 evaluation and, for analytic scenes, an FP32 twin."""

    def __init__(self, kind, data):
        self.kind = kind
        self.data = data

    @staticmethod
    def prims(recs):
        return SDB("prims", np.asarray(recs, dtype=np.float32))

    @staticmethod
    def neural(net):
        return SDB("neural", net)

    def f64(self, P):
        if self.kind == "prims":
            return union_f64(self.data, P)
        return neural_f64(self.data, P)

    def f32(self, x, y, z):
        if self.kind != "prims":
            raise NotImplementedError("the FP32 twin exists for analytic scenes only")
        return union_f32(self.data, x, y, z)

    def scaled(self, factor):
        """factor * f: with factor > 1 this is no longer a distance bound."""
        base = self

        class _Scaled(SDB):
            def f64(s, P):
                return factor * base.f64(P)

            def f32(s, x, y, z):
                return np.float32(factor) * base.f32(x, y, z)

        return _Scaled(self.kind, self.data)


def calibrate_network(net, probe, amplitude, r0):
    """Scale constants of the neural bound, FP64.

    u = NN/S with S the product of the layers' largest singular values;
    mu_u, sigma_u the mean and standard deviation of u over the probe points;
    g = ||p|| - r0 + amplitude (u - mu_u)/sigma_u and L_hat = max |grad g|
    over the probe.  A learned bound is shrunk by a factor found empirically
    (Section 5.2); here the shrink is lambda * L_hat.
    """
    S = float(np.prod([np.linalg.svd(np.asarray(W, dtype=np.float64), compute_uv=False)[0]
                       for W in net["weights"]]))
    P = np.asarray(probe, dtype=np.float64)
    u = mlp_forward_f64(net, P) / S
    mu, sigma = float(u.mean()), float(u.std())
    grad = P / np.linalg.norm(P, axis=1, keepdims=True) + (amplitude / (sigma * S)) * mlp_input_grad_f64(net, P)
    return {"S": S, "mu_u": mu, "sigma_u": sigma, "L_hat": float(np.linalg.norm(grad, axis=1).max())}
