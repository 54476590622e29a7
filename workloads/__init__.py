"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws parameters: primitive placements and sizes, network
weights, point sets and grid descriptions.  It evaluates no distance bound,
hops no ray and polygonizes no cell; both the oracle and the HIP path take
what it returns as plain inputs.

Every floating-point parameter is rounded to float32 here, once, so that the
FP64 oracle and the FP32 GPU path see identical parameter values and differ
only in arithmetic.

Primitive record layout (float32, PRIM_STRIDE = 16 per primitive):
  [0]     type code (PRIM_*)
  [1:4]   centre c
  [4:13]  3x3 matrix M, row-major; the local point is q = M (p - c)
  [13:16] shape parameters, per type:
          sphere    (r, 0, 0)
          box       (bx, by, bz) half extents       (exact Euclidean distance)
          torus     (R, r, 0)   ring in the local xz plane, axis = local y
          capsule   (a, r, 0)   segment [-a, a] on the local z axis
          plane     (d, 0, 0)   f = n . p - d with n = first row of M, c = 0
          boxbound  (bx, by, bz) max of the six face-plane distances
          cylinder  (r, a, 0)   capped at local z = -a, a
          cone      (a, s, c)   apex at local z = a opening toward -z with
                                half-angle sin s, cos c; cut at z = -a
          hexprism  (r, a, 0)   apothem r, faces normal to local x and at
                                +-60 degrees from it; capped at z = -a, a
          genus2    (k, 0, 0)   k F(q) with the genus-2 polynomial F of the
                                paper's Section 5.1; M = s I scales it
          sierpinski (k, d, 0)  the Sierpinski tetrahedron of depth d on the
                                tetrahedron (+-1, +-1, +-1); M = s I, k = 1/s
"""
import json
import os

import numpy as np

PRIM_SPHERE, PRIM_BOX, PRIM_TORUS, PRIM_CAPSULE, PRIM_PLANE, PRIM_BOXBOUND = 0, 1, 2, 3, 4, 5
PRIM_CYLINDER, PRIM_CONE, PRIM_HEXPRISM, PRIM_GENUS2, PRIM_SIERPINSKI = 6, 7, 8, 9, 10
PRIM_STRIDE = 16

_HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------- grid
def grid(n, lo=-1.0, extent=2.0):
    """Cell grid over the cube [lo, lo + n*h]^3 with h = extent/n, as float32.

    The paper's grid is the unit cube centred at the origin, split into N^3
    cells (Section 3, eq. cells).  The workloads use lo = -1, extent = 2; for
    power-of-two n every centroid and lattice coordinate is exact in float32.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    return int(n), np.float32(lo), np.float32(np.float64(extent) / n)


# ---------------------------------------------------------------------- primitives
def _record(ptype, centre, mat, params):
    r = np.zeros(PRIM_STRIDE, dtype=np.float32)
    r[0] = ptype
    r[1:4] = np.asarray(centre, dtype=np.float64)
    r[4:13] = np.asarray(mat, dtype=np.float64).reshape(9)
    r[13:13 + len(params)] = np.asarray(params, dtype=np.float64)
    return r


def _quat_to_local(qv):
    """Rotation R from a unit quaternion (w, x, y, z); returns M = R^T (world -> local)."""
    w, x, y, z = qv
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])
    return R.T


def sphere_scene(radius=0.5, centre=(0.0, 0.0, 0.0)):
    """Exact sphere f(p) = ||p - c|| - r as a one-primitive union."""
    return _record(PRIM_SPHERE, centre, np.eye(3), (radius,))[None, :]


def plane_scene(normal, offset):
    """Plane f(p) = n . p - d with a unit normal (Section 4.1, eq. plane)."""
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    m = np.zeros((3, 3))
    m[0] = n
    return _record(PRIM_PLANE, (0.0, 0.0, 0.0), m, (offset,))[None, :]


def box_scene(half, centre=(0.0, 0.0, 0.0), bound=False):
    """Axis-aligned box: exact distance, or the max-of-planes bound of eq. boxdist."""
    return _record(PRIM_BOXBOUND if bound else PRIM_BOX, centre, np.eye(3), half)[None, :]


def cylinder_scene(r, a, centre=(0.0, 0.0, 0.0)):
    """Capped cylinder about the z axis (exact distance)."""
    return _record(PRIM_CYLINDER, centre, np.eye(3), (r, a))[None, :]


def cone_scene(a, half_angle, centre=(0.0, 0.0, 0.0)):
    """Cone with apex at centre + (0, 0, a), opening toward -z, cut at -a."""
    return _record(PRIM_CONE, centre, np.eye(3), (a, np.sin(half_angle), np.cos(half_angle)))[None, :]


def hexprism_scene(r, a, centre=(0.0, 0.0, 0.0)):
    """Hexagonal prism of apothem r about the z axis, capped at +-a."""
    return _record(PRIM_HEXPRISM, centre, np.eye(3), (r, a))[None, :]


GENUS2_SCALE = 1.8              # local q = s (p - c): the shape spans x in [-1.6, 1.6], y in [-1.82, 0.98]
GENUS2_CENTRE = (0.0, 0.42 / 1.8, 0.0)


def genus2_scene(lo=-1.0, extent=2.0):
    """The paper's implicit surface of genus 2 (Section 5.1) in the grid
    [lo, lo + extent]^3: q = s (p - c) with s = 1.8 and c = (0, 0.42/s, 0)
    centre the shape, and the factor k = 1 / (s L) makes the bound
    1-Lipschitz in p, L = sqrt(2 Fx^2 + Fz^2) with Fx = 12B^2 + 8B^3 + 12B^4
    and Fz = 20B + 36B^3 + 16B^4 bounding |grad F| (sums of the
    monomials' magnitudes) over the cube |q_i| <= B that holds every local
    point of the grid."""
    s = GENUS2_SCALE
    c = np.asarray(GENUS2_CENTRE, dtype=np.float64)
    far = np.maximum(np.abs(lo - c), np.abs(lo + extent - c)).max()
    B = s * far
    fx = 12 * B ** 2 + 8 * B ** 3 + 12 * B ** 4
    fz = 20 * B + 36 * B ** 3 + 16 * B ** 4
    k = 1.0 / (s * np.sqrt(2 * fx * fx + fz * fz))
    return _record(PRIM_GENUS2, c, s * np.eye(3), (k,))[None, :]


def sierpinski_scene(depth=6, scale=1.2, centre=(0.013, -0.021, 0.008)):
    """The Sierpinski tetrahedron of the given depth (Section 5.1's fractal
    scene): the regular tetrahedron with vertices (+-1, +-1, +-1) (an even
    number of minus signs) in local q = scale (p - centre), so its vertices
    sit at distance sqrt(3)/scale from the centre, k = 1/scale.  The centre
    is off the lattice so that no vertex falls on a lattice point."""
    s = float(scale)
    return _record(PRIM_SIERPINSKI, centre, s * np.eye(3), (1.0 / s, depth))[None, :]


def primitives_scene(seed=0):
    """The paper's first scene's seven primitives (Section 5.1: sphere,
    cube, cone, cylinder, torus, hexagonal prism, capsule), each seeded in
    its own slot of a 3 x 3 layout in the z = 0 plane (the centre slot and
    one corner stay empty), with a rotation from a normalised N(0, I_4)
    quaternion and these sizes, drawn in this order per primitive:
      sphere r ~ U[0.15, 0.25]; cube half side ~ U[0.12, 0.2];
      cone a ~ U[0.15, 0.22], half-angle ~ U[0.3, 0.6] rad;
      cylinder r ~ U[0.08, 0.16], a ~ U[0.12, 0.2];
      torus R ~ U[0.12, 0.18], r ~ U[0.03, 0.06];
      hexagonal prism apothem ~ U[0.08, 0.16], a ~ U[0.1, 0.2];
      capsule a ~ U[0.08, 0.15], r ~ U[0.05, 0.09]."""
    rng = np.random.default_rng(seed)
    slots = [(-0.6, -0.6), (0.0, -0.6), (0.6, -0.6), (-0.6, 0.0), (0.6, 0.0), (-0.6, 0.6), (0.0, 0.6)]
    recs = []
    for t, (sx, sy) in zip((PRIM_SPHERE, PRIM_BOX, PRIM_CONE, PRIM_CYLINDER, PRIM_TORUS, PRIM_HEXPRISM, PRIM_CAPSULE),
                           slots):
        qv = rng.standard_normal(4)
        M = _quat_to_local(qv / np.linalg.norm(qv))
        c = (sx, sy, 0.0)
        if t == PRIM_SPHERE:
            params = (rng.uniform(0.15, 0.25),)
        elif t == PRIM_BOX:
            params = (rng.uniform(0.12, 0.2),) * 3
        elif t == PRIM_CONE:
            a, ang = rng.uniform(0.15, 0.22), rng.uniform(0.3, 0.6)
            params = (a, np.sin(ang), np.cos(ang))
        elif t == PRIM_CYLINDER:
            params = (rng.uniform(0.08, 0.16), rng.uniform(0.12, 0.2))
        elif t == PRIM_TORUS:
            params = (rng.uniform(0.12, 0.18), rng.uniform(0.03, 0.06))
        elif t == PRIM_HEXPRISM:
            params = (rng.uniform(0.08, 0.16), rng.uniform(0.1, 0.2))
        else:
            params = (rng.uniform(0.08, 0.15), rng.uniform(0.05, 0.09))
        recs.append(_record(t, c, M, params))
    return np.stack(recs)


def csg_scene(seed=0, n_prim=12):
    """Min-union of n_prim seeded primitives (Section 4.3 union by min).

    Type of primitive i is i mod 4 (sphere, box, torus, capsule).  Per
    primitive, in this order: centre ~ U[-0.6, 0.6]^3, a quaternion from
    N(0, I_4) normalised (uniform rotation), then the size parameters:
      sphere  r ~ U[0.1, 0.3]
      box     half extents ~ U[0.05, 0.2]^3
      torus   R ~ U[0.1, 0.25], r ~ U[0.03, 0.08]
      capsule a ~ U[0.05, 0.2], r ~ U[0.03, 0.1]
    """
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n_prim):
        t = i % 4
        c = rng.uniform(-0.6, 0.6, size=3)
        qv = rng.standard_normal(4)
        qv = qv / np.linalg.norm(qv)
        m = _quat_to_local(qv)
        if t == 0:
            recs.append(_record(PRIM_SPHERE, c, m, (rng.uniform(0.1, 0.3),)))
        elif t == 1:
            recs.append(_record(PRIM_BOX, c, m, rng.uniform(0.05, 0.2, size=3)))
        elif t == 2:
            recs.append(_record(PRIM_TORUS, c, m, (rng.uniform(0.1, 0.25), rng.uniform(0.03, 0.08))))
        else:
            recs.append(_record(PRIM_CAPSULE, c, m, (rng.uniform(0.05, 0.2), rng.uniform(0.03, 0.1))))
    return np.stack(recs)


# -------------------------------------------------------------------------- network
def fourier_omegas(n_freq=16):
    """Angular frequencies w_k = 2^(k/4) rad per unit, k = 0..n_freq-1 (float32)."""
    return (2.0 ** (np.arange(n_freq) / 4.0)).astype(np.float32)


def mlp_net(seed=0, width=256, depth=4, n_freq=16, activation="softplus"):
    """Random-weight MLP  gamma(p) -> depth x [width, activation] -> 1.

    gamma(p) = [p_x, p_y, p_z, then for each k: sin(w_k p_x), sin(w_k p_y),
    sin(w_k p_z), cos(w_k p_x), cos(w_k p_y), cos(w_k p_z)], 3 + 6 n_freq
    features.  softplus: weights W_l (fan_out x fan_in) ~ N(0, 1/fan_in),
    drawn in layer order from default_rng(seed); biases zero.  relu (the
    paper's architecture, Section 5.2: ReLU layers with batch normalisation,
    which folds into each layer's weights and bias at inference): weights
    ~ N(0, 2/fan_in) drawn in layer order, then the hidden layers' biases
    ~ N(0, 0.1^2) in layer order; the output bias is zero.  All float32.
    """
    if activation not in ("softplus", "relu"):
        raise ValueError(f"unknown activation {activation!r}")
    rng = np.random.default_rng(seed)
    dims = [3 + 6 * n_freq] + [width] * depth + [1]
    weights, biases = [], []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        z = rng.standard_normal((fan_out, fan_in))
        w = z * np.sqrt(2.0 / fan_in) if activation == "relu" else z / np.sqrt(fan_in)
        weights.append(w.astype(np.float32))
        biases.append(np.zeros(fan_out, dtype=np.float32))
    if activation == "relu":
        for l in range(len(dims) - 2):
            biases[l] = (0.1 * rng.standard_normal(dims[l + 1])).astype(np.float32)
    return {"omegas": fourier_omegas(n_freq), "weights": weights, "biases": biases, "activation": activation}


def probe_points(seed=3, n=65536):
    """Uniform points in [-1, 1]^3 used to calibrate a network's scale."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, 3))


def loss_targets(seed=1, n=4096, radius=0.4):
    """Points on a sphere of the given radius: radius * z/||z||, z ~ N(0, I_3)."""
    z = np.random.default_rng(seed).standard_normal((n, 3))
    return (radius * z / np.linalg.norm(z, axis=1, keepdims=True)).astype(np.float32)


NEURAL_LAMBDA = 1.5      # shrink factor of a learned bound (Section 5.2)
NEURAL_R0 = 0.5          # radius of the sphere prior that places the surface
NEURAL_AMPLITUDE = 0.05  # amplitude of the standardised network perturbation


def neural_calibration_path():
    return os.path.join(_HERE, "neural_calibration.json")


def calibration_key(seed, width, depth, n_freq, activation="softplus"):
    return f"seed{seed}_w{width}_d{depth}_f{n_freq}" + ("" if activation == "softplus" else f"_{activation}")


def neural_scene(seed=0, width=256, depth=4, n_freq=16, activation="softplus"):
    """Neural bound  f(p) = a_s (||p|| - r0) + a_n NN(gamma(p)) + b.

    The coefficients come from a stored calibration of this exact network
    (keyed by seed/width/depth/n_freq): with u = NN/S, S the product of the
    layers' spectral norms, g = ||p|| - r0 + A (u - mu_u)/sigma_u and
    f = g / (lambda L), where mu_u, sigma_u are the mean and deviation of u
    over probe_points() and L the largest |grad g| there.  Hence
    a_s = 1/(lambda L), a_n = A/(sigma_u S lambda L), b = -A mu_u/(sigma_u lambda L).
    """
    net = mlp_net(seed, width, depth, n_freq, activation)
    key = calibration_key(seed, width, depth, n_freq, activation)
    with open(neural_calibration_path()) as fh:
        cal = json.load(fh)
    if key not in cal:
        raise KeyError(f"no calibration stored for network {key}")
    c = cal[key]
    lam_l = NEURAL_LAMBDA * c["L_hat"]
    net["r0"] = np.float32(NEURAL_R0)
    net["a_s"] = np.float32(1.0 / lam_l)
    net["a_n"] = np.float32(NEURAL_AMPLITUDE / (c["sigma_u"] * c["S"] * lam_l))
    net["b"] = np.float32(-NEURAL_AMPLITUDE * c["mu_u"] / (c["sigma_u"] * lam_l))
    net["calibration"] = c
    return net


def paper_net_scene(seed=0):
    """The paper's network shape (Section 5.2): eight ReLU layers of width 64
    on the raw coordinates (no Fourier features), random weights, under the
    same sphere prior and calibration as neural_scene: 28,928 weights."""
    return neural_scene(seed, 64, 8, 0, "relu")


# -------------------------------------------------------------------------- batch
def batch_scenes(seed=2, n_shapes=64):
    """Mixed batch: N_s ~ choice{64,128,256,512}; even s a CSG union of
    n_prim ~ U{4..16} primitives (seed 2000+s), odd s an MLP of width
    ~ choice{64,128,256} (seed 1000+s)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_shapes):
        n = int(rng.choice([64, 128, 256, 512]))
        if s % 2 == 0:
            out.append({"kind": "csg", "n": n, "seed": 2000 + s, "n_prim": int(rng.integers(4, 17))})
        else:
            out.append({"kind": "mlp", "n": n, "seed": 1000 + s, "width": int(rng.choice([64, 128, 256]))})
    return out
