"""Grid hopping: sphere tracing along the N^2 cell columns of the grid,
continuing past the surface, then marching cubes on the cells reached.

Paper, Section 3: rays R_ij start at the first cell centroid of column
(i, j) (eq. cells) and advance by |f| (eq. iter); a cell is polygonized when
the bound is small enough (eq. polydist) and the march resumes at the next
cell until the ray leaves the volume (Algorithm 1).

Hop rule used here (cell-quantised form of eq. iter): at the centroid c of
cell (i, j, k), d = |f(c)| and s = floor(d / h).
  s >= 1:  the ray skips s cells, k <- k + s;
  s == 0:  k <- k + 1, and cell (i, j, k) is a candidate for marching cubes
           when d <= T = (sqrt 3 / 2 + 1/32) h;
the ray ends once k >= N.  Every point of cells k .. k+s-1 of the column lies
within h*sqrt(1/2 + (s - 1/2)^2) < s*h <= d of c, i.e. inside the open ball
of radius d around c, which holds no zero of a distance bound (Section 1:
|f| is at most the distance to the surface): the skipped cells hold no sign
change.  A cell with a sign change holds a zero on one of its edges, at most
half its diagonal, (sqrt 3 / 2) h, from c, so d <= (sqrt 3 / 2) h there; with
values computed to within e of f (corner signs and d alike) a cell whose
computed corner signs differ still has d <= (sqrt 3 / 2) h + 2e, which the
h/32 of T covers while e <= h/64 (float32 values of unit-scale bounds are
within a few 1e-6).  So no sign-change cell is missed, and cells with
T < d < h, which cannot hold the surface, are stepped over without marching
cubes.  On grids whose cells are small against the coordinates (h below
2^-12 of the largest of 1, |lo| and |lo + N h|) T is h: every cell with
s == 0 is a candidate.

Columns are independent, so the oracle advances all live columns together
(one numpy step per hop); `hop_column` is the same rule for one column as a
plain loop.
"""
import numpy as np

from . import mc


def centroid_f64(lo, h, idx):
    """Cell centroid coordinate lo + (idx + 1/2) h (eq. cells, generalised)."""
    return np.float64(lo) + (np.asarray(idx, dtype=np.float64) + 0.5) * np.float64(h)


def centroid_f32(lo, h, idx):
    """Float32 centroid: m = (idx + 0.5f) * h rounded, then lo + m rounded."""
    t = np.asarray(idx).astype(np.float32) + np.float32(0.5)
    return np.float32(lo) + t * np.float32(h)


def _threshold_factor(n, lo, h):
    """sqrt 3 / 2 + 1/32, or 1 on grids whose cells are small against the
    coordinates (h < 2^-12 max(1, |lo|, |lo + n h|)); in double."""
    lo, h = float(lo), float(h)
    scale = max(1.0, abs(lo), abs(lo + n * h))
    return np.sqrt(3.0) / 2.0 + 1.0 / 32.0 if h >= 2.0 ** -12 * scale else 1.0


def candidate_threshold_f64(n, lo, h):
    """The candidate threshold T = (sqrt 3 / 2 + 1/32) h (see the module notes)."""
    return _threshold_factor(n, lo, h) * np.float64(h)


def candidate_threshold_f32(n, lo, h):
    """The float32 threshold: the factor times float32(h) in double, rounded once."""
    h32, lo32 = np.float32(h), np.float32(lo)
    return np.float32(_threshold_factor(n, lo32, h32) * np.float64(h32))


def hop(sdb, n, lo, h, precision="f64", columns=None, shrink=0.0):
    """Run the hop rule over every column (or the given column ids i*N + j).

    Returns (candidate cell ids sorted, number of bound evaluations, per-column
    evaluation counts).  precision "f32" is the twin of the GPU float32
    formula: float32 coordinates, float32 f, s = floor(d * inv_h) in float32
    with inv_h = float32(1/h), and the step capped at N.
    shrink (FP64 only): d = max(|f| - shrink, 0) in the step and the
    candidate test, the rule for a value known only to within shrink of f;
    since |f| - shrink is still at most the distance to the surface, no
    sign-change cell is skipped or left unmarked.
    """
    if shrink and precision != "f64":
        raise ValueError("shrink applies to the FP64 hop")
    if columns is None:
        columns = np.arange(n * n, dtype=np.int64)
    columns = np.asarray(columns, dtype=np.int64)
    ci, cj = columns // n, columns % n
    if precision == "f64":
        x, y = centroid_f64(lo, h, ci), centroid_f64(lo, h, cj)
        thr = candidate_threshold_f64(n, lo, h)
    else:
        x, y = centroid_f32(lo, h, ci), centroid_f32(lo, h, cj)
        inv_h = np.float32(1.0 / np.float64(np.float32(h)))
        thr = candidate_threshold_f32(n, lo, h)
    k = np.zeros(len(columns), dtype=np.int64)
    live = np.arange(len(columns))
    evals = np.zeros(len(columns), dtype=np.int64)
    cand = []
    while live.size:
        kk = k[live]
        if precision == "f64":
            f = sdb.f64(np.stack([x[live], y[live], centroid_f64(lo, h, kk)], axis=1))
            d = np.maximum(np.abs(f) - shrink, 0.0)
            s = np.floor(d / np.float64(h))
        else:
            f = sdb.f32(x[live], y[live], centroid_f32(lo, h, kk))
            d = np.abs(f)
            s = np.floor(d * inv_h)
        if not np.all(np.isfinite(f)):
            raise FloatingPointError("non-finite distance bound value")
        evals[live] += 1
        hit = s == 0
        mark = hit & (d <= thr)
        cand.append(columns[live[mark]] * n + kk[mark])
        step = np.where(hit, 1, np.minimum(s, n)).astype(np.int64)
        k[live] = kk + step
        live = live[k[live] < n]
    cells = np.sort(np.concatenate(cand)) if cand else np.zeros(0, np.int64)
    return cells, int(evals.sum()), evals


def hop_column(f_at_centroid, n, h, lo=-1.0):
    """The hop rule along one column as a plain loop: f_at_centroid(k) -> f.
    Returns (candidate k list, evaluation count)."""
    k, evals, cand = 0, 0, []
    while k < n:
        d = abs(f_at_centroid(k))
        evals += 1
        s = int(np.floor(d / h))
        if s == 0:
            if d <= candidate_threshold_f64(n, lo, h):
                cand.append(k)
            k += 1
        else:
            k += min(s, n)
    return cand, evals


def corner_points(n, cells):
    """Distinct lattice points (i, j, k) that are corners of the given cells."""
    cells = np.asarray(cells, dtype=np.int64)
    i, j, k = cells // (n * n), (cells // n) % n, cells % n
    n1 = n + 1
    pid = np.concatenate([((i + dx) * n1 + (j + dy)) * n1 + (k + dz)
                          for (dx, dy, dz) in mc.CORNER])
    return np.unique(pid)


class HopResult:
    def __init__(self, mesh, candidates, hop_evals, corner_evals, column_evals):
        self.mesh = mesh
        self.candidates = candidates
        self.hop_evals = hop_evals
        self.corner_evals = corner_evals
        self.column_evals = column_evals

    @property
    def evals(self):
        return self.hop_evals + self.corner_evals


def gridhop(sdb, n, lo, h, precision="f64", shrink=0.0):
    """Grid hopping followed by marching cubes on the candidate cells.

    Corner values are evaluated once per distinct lattice point of the
    candidates; their count is the corner evaluation count.
    """
    cells, hop_evals, col_evals = hop(sdb, n, lo, h, precision, shrink=shrink)
    return polygonize_cells(sdb, n, lo, h, cells, hop_evals, col_evals, precision)


def polygonize_cells(sdb, n, lo, h, cells, hop_evals, col_evals, precision="f64"):
    """Marching cubes on the given candidate cells (bound evaluated once per
    distinct corner point), packaged with the counts of the step that found
    the cells."""
    pid = corner_points(n, cells)
    n1 = n + 1
    a, b, c = pid // (n1 * n1), (pid // n1) % n1, pid % n1
    if precision == "f64":
        P = np.stack([mc.lattice_coords_f64(n, lo, h, v) for v in (a, b, c)], axis=1)
        fv = sdb.f64(P) if len(pid) else np.zeros(0)
    else:
        xs = [mc.lattice_coords_f32(n, lo, h, v) for v in (a, b, c)]
        fv = sdb.f32(*xs).astype(np.float64) if len(pid) else np.zeros(0)

    def corner_value(i, j, k):
        q = (i * n1 + j) * n1 + k
        return fv[np.searchsorted(pid, q)]

    mesh = mc.polygonize(n, lo, h, cells, corner_value)
    return HopResult(mesh, cells, hop_evals, len(pid), col_evals)
