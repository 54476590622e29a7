// Marching-cubes case table, computed at compile time.
//
// The paper polygonizes each reached cell with marching cubes (Section 5)
// and leaves the per-cell construction open; this table encodes the
// following one.  Corner c = dx | dy<<1 | dz<<2 is inside when f < 0.  Cell
// edge e = 4*axis + r joins two corners that differ along `axis`; r holds
// the offsets along the two other axes, lower axis in bit 0.  On each face,
// walking the corners counter-clockwise as seen from outside the cell, every
// maximal run of inside corners contributes a segment from the edge where
// the walk enters the run to the edge where it leaves it (so an ambiguous
// face keeps its two inside corners apart).  The segments chain into closed
// loops; each loop is fanned from its smallest edge, which orients every
// triangle from the inside towards the outside.  Adjacent cells walk a
// shared face in opposite directions over the same signs, hence cut it with
// the same segments and the mesh closes up.
#pragma once

#include <stdint.h>

namespace gh {

struct McCase {
  uint64_t tri;   // triangle t, vertex v: cell edge in nibble 3*t + v
  uint32_t ntri;  // 0..5
  uint32_t edges; // bit e set when edge e crosses the surface
};

struct McTable {
  McCase c[256];
};

constexpr int mc_edge_between(int a, int b) {
  const int diff = a ^ b;
  const int axis = diff == 1 ? 0 : (diff == 2 ? 1 : 2);
  const int lo = a < b ? a : b;
  int r = 0, slot = 0;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax == axis) continue;
    r |= ((lo >> ax) & 1) << slot;
    ++slot;
  }
  return 4 * axis + r;
}

constexpr McTable make_mc_table() {
  McTable table{};
  constexpr int du[4] = {0, 1, 1, 0};
  constexpr int dv[4] = {0, 0, 1, 1};
  for (int cs = 0; cs < 256; ++cs) {
    int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    for (int axis = 0; axis < 3; ++axis) {
      const int u = (axis + 1) % 3, v = (axis + 2) % 3;  // e_u x e_v = e_axis
      for (int side = 0; side < 2; ++side) {
        int ring[4] = {0, 0, 0, 0};
        for (int p = 0; p < 4; ++p) {
          int d[3] = {0, 0, 0};
          d[axis] = side;
          d[u] = du[p];
          d[v] = dv[p];
          // counter-clockwise about +e_axis; reversed on the face whose outward normal is -e_axis
          ring[side ? p : 3 - p] = d[0] | (d[1] << 1) | (d[2] << 2);
        }
        for (int p = 0; p < 4; ++p) {
          const int prev = (p + 3) & 3;
          const bool in_p = (cs >> ring[p]) & 1, in_prev = (cs >> ring[prev]) & 1;
          if (!in_p || in_prev) continue;
          int q = p;
          while ((cs >> ring[(q + 1) & 3]) & 1) q = (q + 1) & 3;
          next[mc_edge_between(ring[prev], ring[p])] = mc_edge_between(ring[q], ring[(q + 1) & 3]);
        }
      }
    }
    bool seen[12] = {false, false, false, false, false, false, false, false, false, false, false, false};
    uint64_t packed = 0;
    uint32_t ntri = 0, edges = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (next[e0] < 0 || seen[e0]) continue;
      int loop[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      int len = 0;
      for (int e = e0; !seen[e]; e = next[e]) {
        seen[e] = true;
        edges |= 1u << e;
        loop[len++] = e;
      }
      for (int t = 1; t + 1 < len; ++t) {
        const uint64_t tri = (uint64_t)loop[0] | ((uint64_t)loop[t] << 4) | ((uint64_t)loop[t + 1] << 8);
        packed |= tri << (12 * ntri);
        ++ntri;
      }
    }
    table.c[cs].tri = packed;
    table.c[cs].ntri = ntri;
    table.c[cs].edges = edges;
  }
  return table;
}

inline constexpr McTable kMcTable = make_mc_table();

// Lower corner of each cell edge, and its axis.
constexpr int mc_edge_lower(int e) {
  const int axis = e >> 2, r = e & 3;
  int d[3] = {0, 0, 0};
  int slot = 0;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax == axis) continue;
    d[ax] = (r >> slot) & 1;
    ++slot;
  }
  return d[0] | (d[1] << 1) | (d[2] << 2);
}

static_assert(kMcTable.c[0].ntri == 0 && kMcTable.c[255].ntri == 0, "empty cases");
static_assert(kMcTable.c[1].ntri == 1 && kMcTable.c[254].ntri == 1, "single corner");
static_assert(mc_edge_lower(11) == 3 && mc_edge_lower(7) == 5 && mc_edge_lower(3) == 6, "edge corners");

}  // namespace gh
