// Index maps and element constants of the Q2 / P1disc hexahedron x dG(1)
// shared by the 3D smoother and the 3D coarse levels.
#pragma once

#include "pns_internal.h"

namespace pns {

constexpr int kNb3 = 27;             // Q2 nodes of a hexahedron
constexpr int kNv3 = 3 * kNb3;       // velocity unknowns of a cell
constexpr int kNs3 = kNv3 + 4;       // spatial unknowns of a cell (85)
constexpr int kEs3 = kNs3 * kNs3;    // entries of a spatial cell matrix

__host__ __device__ inline int64_t cell_index3(const Grid3& g, int cx, int cy, int cz) {
  return ((int64_t)cz * g.ny + cy) * g.nx + cx;
}

__device__ __forceinline__ int64_t node_index3(const Grid3& g, int cx, int cy, int cz, int a) {
  const int64_t NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  return (int64_t)(2 * cx + a % 3) + NX * ((int64_t)(2 * cy + (a / 3) % 3) + NY * (2 * cz + a / 9));
}

// canonical index of spatial local unknown l of cell (cx,cy,cz) at Radau node mu
__device__ __forceinline__ int64_t gidx3(const Grid3& g, int cx, int cy, int cz, int l, int mu) {
  if (l < kNv3) return (int64_t)mu * g.ns + (int64_t)(l / kNb3) * g.nn + node_index3(g, cx, cy, cz, l % kNb3);
  return (int64_t)mu * g.ns + g.nv + 4 * cell_index3(g, cx, cy, cz) + (l - kNv3);
}

// Patches of one colour (parity px, py, pz) are stored contiguously, colours
// in the order c = px + 2 py + 4 pz, lexicographically (x fastest) within.
__host__ __device__ inline int64_t colour_count3(const Grid3& g, int c) {
  const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
  return (int64_t)((g.nx - px + 1) / 2) * ((g.ny - py + 1) / 2) * ((g.nz - pz + 1) / 2);
}

__host__ __device__ inline int64_t patch_slot3(const Grid3& g, int cx, int cy, int cz) {
  const int c = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
  int64_t off = 0;
  for (int k = 0; k < c; ++k) off += colour_count3(g, k);
  const int64_t ncx = (g.nx - (cx & 1) + 1) / 2, ncy = (g.ny - (cy & 1) + 1) / 2;
  return off + ((int64_t)(cz >> 1) * ncy + (cy >> 1)) * ncx + (cx >> 1);
}

// 1D Q2 mass of a cell of unit length (nodes 0, 1/2, 1): [[4,2,-1],[2,16,2],[-1,2,4]] / 30
__device__ __forceinline__ double mass1(int a, int b) {
  if (a == 1 && b == 1) return 16.0 / 30.0;
  if (a == 1 || b == 1) return 2.0 / 30.0;
  return a == b ? 4.0 / 30.0 : -1.0 / 30.0;
}

__device__ __forceinline__ double cell_mass3(const Grid3& g, int a, int b) {
  return mass1(a % 3, b % 3) * g.hx * mass1((a / 3) % 3, (b / 3) % 3) * g.hy *
         mass1(a / 9, b / 9) * g.hz;
}

// canonical index of space-time local unknown l = mu * 85 + spatial index
__device__ __forceinline__ int64_t gidx_st3(const Grid3& g, int cx, int cy, int cz, int l) {
  return gidx3(g, cx, cy, cz, l % kNs3, l / kNs3);
}

// position of space-time local unknown l in a cell's slot of per-cell results
// (layout of the 3D action: velocity of node a, Radau node mu, component c at
// a * 6 + mu * 3 + c; pressure j of mu at 162 + mu * 4 + j)
__host__ __device__ inline int slot_pos3(int l) {
  const int mu = l / kNs3, s = l % kNs3;
  if (s < kNv3) return (s % kNb3) * 6 + mu * 3 + s / kNb3;
  return 162 + mu * 4 + (s - kNv3);
}

constexpr int kNst3 = 2 * kNs3;      // space-time unknowns of a cell (170)
constexpr int kE3 = kNst3 * kNst3;   // entries of a space-time cell matrix

}  // namespace pns
