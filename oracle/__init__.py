"""Oracle: a plain, slow CPU implementation of grid hopping, written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP path
(the two meet only through the seeded inputs of the `workloads` module).

Modules
  sdb     signed distance bounds in FP64, plus an FP32 twin that applies the
          GPU path's float32 formula operation by operation
  mc      per-cell polygon construction (no lookup table) and enumeration
  hop     grid hopping over the N^2 ray columns, with evaluation counters
  traced  the paper's per-column procedure taken literally: continuous
          sphere tracing to the polygonization distance (Algorithm 1)
  cont    continuation, the paper's surface-following comparator: from seed
          cells to face neighbours across faces the surface crosses
  mesh    mesh checks: manifoldness, Euler characteristic, area, volume,
          Hausdorff distance
  adjoint analytic FP64 gradient of a vertex loss w.r.t. network parameters,
          and central finite differences
"""
