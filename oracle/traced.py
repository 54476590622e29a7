"""The paper's per-column procedure taken literally: continuous sphere
tracing along each column down to the polygonization distance, one cell
marked, then on from the next cell (Section 3: eq. iter, eq. polydist and
Algorithm 1).  Test infrastructure, like the rest of this package.

For column (i, j), in the paper's order (the unit cube generalised to the
grid [lo, lo + N h]^3, so 1/N becomes h and the cube's top z = 1/2 becomes
z_top = lo + N h):

  k <- 0
  repeat
    z_s <- centroid z of cell k
    trace from z_s: t <- 0; at p = (x_i, y_j, z_s + t) take d = |f(p)|;
      stop when d <= tau = sqrt(6)/2 h (eq. polydist);
      otherwise t <- t + d (eq. iter), and stop once t >= 1.05 (z_top - z_s)
    z <- z_s + t
    k <- max(k, floor((z - z_c0) / h))   z_c0 the first centroid: the index of
                                          the last centroid at or below z
    leave the column when k > N - 1 or z > z_mid + 1.05 N h / 2
    cell (i, j, k) is a candidate;  k <- k + 1

Readings (the paper leaves them open):
  - trace_ray is not defined; here it is plain sphere tracing with the two
    stopping rules Algorithm 1 hands it (distance to the surface, travel
    limit 1.05 x the distance to the top face), returning the travel t.
  - eq. polydist asks for |f| <= tau, so d == tau stops the trace.
  - The overrun test z > 1.05/2 of the unit cube becomes z above the cube's
    mid-plane by 1.05 x half its side.
  - max(k, .): with exact arithmetic floor((z_s + t - z_c0) / h) >= k; the
    guard keeps a rounding of z_s - z_c0 just below k h from sending the
    column back to the cell it started from (it never acts on grids whose
    centroids are exact in the arithmetic used).

precision "f64": everything in float64.  precision "f32": the float32 twin
of the GPU path: float32 centroids as in `hop.centroid_f32`, the bound's
FP32 twin, t and z accumulated in float32, and the constants tau, z_top and
the overrun height computed in float64 from the float32 grid values and
rounded once to float32; the factor 1.05 is float32(1.05), the cell index
uses float32(1 / h) as the hop does.
"""
import numpy as np

from .hop import centroid_f32, centroid_f64, polygonize_cells


def _constants(n, lo, h, precision):
    lo64, h64 = float(np.float32(lo)), float(np.float32(h))
    tau = np.sqrt(6.0) / 2.0 * h64                 # eq. polydist with 1/N -> h
    z_top = lo64 + n * h64
    z_exit = lo64 + n * h64 / 2.0 + 1.05 * (n * h64 / 2.0)
    if precision == "f64":
        return dict(tau=tau, z_top=z_top, z_exit=z_exit, c105=1.05, inv_h=None, h=h64,
                    z0=float(centroid_f64(lo64, h64, 0)), dt=np.float64)
    return dict(tau=np.float32(tau), z_top=np.float32(z_top), z_exit=np.float32(z_exit), c105=np.float32(1.05),
                inv_h=np.float32(1.0 / h64), h=np.float32(h64), z0=np.float32(centroid_f32(lo, h, 0)),
                dt=np.float32)


def hop_traced(sdb, n, lo, h, precision="f64", columns=None):
    """Algorithm 1 over every column (or the given column ids i*N + j).

    Returns (candidate cell ids sorted, number of bound evaluations,
    per-column evaluation counts), the same form as `hop.hop`.
    """
    C = _constants(n, lo, h, precision)
    dt = C["dt"]
    if columns is None:
        columns = np.arange(n * n, dtype=np.int64)
    columns = np.asarray(columns, dtype=np.int64)
    ci, cj = columns // n, columns % n
    if precision == "f64":
        x, y = centroid_f64(lo, h, ci), centroid_f64(lo, h, cj)
        cz = lambda kk: centroid_f64(lo, h, kk)
    else:
        x, y = centroid_f32(lo, h, ci), centroid_f32(lo, h, cj)
        cz = lambda kk: centroid_f32(lo, h, kk)

    def f_abs(rows, z):
        if precision == "f64":
            v = sdb.f64(np.stack([x[rows], y[rows], z], axis=1))
        else:
            v = sdb.f32(x[rows], y[rows], z).astype(np.float32)
        if not np.all(np.isfinite(v)):
            raise FloatingPointError("non-finite distance bound value")
        return np.abs(v).astype(dt)

    def t_max(zs):
        return (C["c105"] * (C["z_top"] - zs)).astype(dt) if precision == "f32" else C["c105"] * (C["z_top"] - zs)

    m = len(columns)
    k = np.zeros(m, dtype=np.int64)
    zs = cz(k).astype(dt)
    t = np.zeros(m, dtype=dt)
    tmax = t_max(zs)
    evals = np.zeros(m, dtype=np.int64)
    live = np.arange(m)
    cand = []
    while live.size:
        # one trace step on every live column: evaluate at z_s + t
        z = (zs[live] + t[live]).astype(dt)
        d = f_abs(live, z)
        evals[live] += 1
        near = d <= C["tau"]
        t_next = (t[live] + d).astype(dt)
        t[live] = np.where(near, t[live], t_next)
        ended = near | (t_next >= tmax[live])
        done = live[ended]
        if done.size:
            # the trace of these columns stopped: locate its cell
            z = (zs[done] + t[done]).astype(dt)
            if precision == "f64":
                kf = np.floor((z - C["z0"]) / C["h"])
            else:
                kf = np.floor(((z - C["z0"]).astype(np.float32) * C["inv_h"]).astype(np.float32))
            kk = np.maximum(k[done], kf.astype(np.int64))
            out = (kk > n - 1) | (z > C["z_exit"])
            keep = done[~out]
            cand.append(columns[keep] * n + kk[~out])
            k[keep] = kk[~out] + 1
            zs[keep] = cz(k[keep]).astype(dt)
            t[keep] = 0
            tmax[keep] = t_max(zs[keep])
            finished = done[out]
            live = np.setdiff1d(live, finished, assume_unique=True)
    cells = np.sort(np.concatenate(cand)) if cand else np.zeros(0, np.int64)
    return cells, int(evals.sum()), evals


def gridhop_traced(sdb, n, lo, h, precision="f64"):
    """The literal procedure followed by marching cubes on its candidates
    (the same result form as `hop.gridhop`)."""
    cells, evals, col_evals = hop_traced(sdb, n, lo, h, precision)
    return polygonize_cells(sdb, n, lo, h, cells, evals, col_evals, precision)
