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

// value and physical gradient of the Q2 basis function of node a at xi
__device__ __forceinline__ void basis3(const Grid3& g, int a, const double xi[3], double& ph,
                                       double gr[3]) {
  const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
  const double vx = q2v(ax, xi[0]), vy = q2v(ay, xi[1]), vz = q2v(az, xi[2]);
  ph = vx * vy * vz;
  gr[0] = q2d(ax, xi[0]) * g.ihx * vy * vz;
  gr[1] = vx * q2d(ay, xi[1]) * g.ihy * vz;
  gr[2] = vx * vy * q2d(az, xi[2]) * g.ihz;
}

// Dirichlet data at the boundary face points of a hexahedral mesh: per point
// (side sd = 2k + end, k the normal direction; face cell (i1, i2) along the
// directions k1 = (k+1) % 3, k2 = (k+2) % 3; point qa = q1 + 3 q2 with
// reference coordinates xi_k1 = g_q1, xi_k2 = g_q2) and time slot s (0, 1:
// Radau nodes, 2: the slab midpoint): the lifting's value (3), its symmetric
// gradient G (G00, G01, G02, G11, G12, G22) and eta(G), k(G) of frozen_coef3.
constexpr int kLift3Vals = 11;
__host__ __device__ inline int64_t lift3_index(const Grid3& g, int sd, int i1, int i2, int qa,
                                               int s) {
  const int n[3] = {g.nx, g.ny, g.nz};
  int64_t off = 0;
  for (int t = 0; t < sd; ++t) {
    const int kt = t >> 1;
    off += (int64_t)n[(kt + 1) % 3] * n[(kt + 2) % 3];
  }
  const int k = sd >> 1;
  return (((off + (int64_t)i2 * n[(k + 1) % 3] + i1) * 9 + qa) * 3 + s) * kLift3Vals;
}
__host__ __device__ inline int64_t lift3_table_doubles(const Grid3& g) {
  return lift3_index(g, 6, 0, 0, 0, 0);
}

// eta(G) and k(G) = (p-2) nu (delta^2 + |G|^2)^((p-4)/2) for a symmetric 3 x 3 G
__host__ __device__ inline void frozen_coef3(const Model& m, const double* G6, double& eta,
                                             double& k) {
  const double g2 = G6[0] * G6[0] + G6[3] * G6[3] + G6[5] * G6[5] +
                    2.0 * (G6[1] * G6[1] + G6[2] * G6[2] + G6[4] * G6[4]);
  const double D2 = m.delta2 + g2;
  const double mu = m.nu * pow(D2, m.expo);
  eta = m.nu_inf + mu;
  k = (m.p - 2.0) * mu / D2;
}

// full symmetric matrix from the table's six entries
__host__ __device__ inline void sym3(const double* G6, double G[3][3]) {
  G[0][0] = G6[0]; G[0][1] = G[1][0] = G6[1]; G[0][2] = G[2][0] = G6[2];
  G[1][1] = G6[3]; G[1][2] = G[2][1] = G6[4]; G[2][2] = G6[5];
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
