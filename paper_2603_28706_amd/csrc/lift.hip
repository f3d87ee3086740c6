// Inhomogeneous Dirichlet data (Sec. 3.2, eq. def-b-gam): the lifting ghat_D,
// a Q2 velocity field per Radau node, evaluated once at every boundary face
// point of the quadrilateral mesh — its value (the data g_D), its symmetric
// gradient G = D ghat_D from the boundary cell's nine nodes, and the frozen
// Nitsche coefficients eta(G), k(G) — for the two Radau nodes and the slab
// midpoint (the lifting interpolated linearly in time, as the surrogate
// patches freeze every coefficient there).  The action, the residual and the
// cell matrices read the table at their face points, which keeps the
// evaluation out of their register budgets.
#include "pns_internal.h"

namespace pns {
namespace {

// one thread per (side, cell along the side, Gauss point, time slot)
__global__ __launch_bounds__(256) void lift_table_kernel(Grid g, Model m,
                                                         const double* __restrict__ ghat,
                                                         double* __restrict__ table) {
  const int L = g.nx > g.ny ? g.nx : g.ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)4 * L * 9) return;
  const int s = (int)(id % 3), q = (int)((id / 3) % 3);
  const int j = (int)((id / 9) % L), side = (int)(id / (9 * L));
  const bool xface = side < 2;
  if (j >= (xface ? g.ny : g.nx)) return;
  const int cx = xface ? (side == 0 ? 0 : g.nx - 1) : j;
  const int cy = xface ? j : (side == 2 ? 0 : g.ny - 1);
  const double gq = q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]);
  const double xi = xface ? (side == 0 ? 0.0 : 1.0) : gq;
  const double et = xface ? gq : (side == 2 ? 0.0 : 1.0);
  // time weights of the two Radau nodes' fields
  const double w0 = s == 0 ? 1.0 : (s == 1 ? 0.0 : kXiMid[0]);
  const double w1 = s == 0 ? 0.0 : (s == 1 ? 1.0 : kXiMid[1]);
  const int NX = 2 * g.nx + 1;
  double v0 = 0.0, v1 = 0.0, g00 = 0.0, g01 = 0.0, g10 = 0.0, g11 = 0.0;
  for (int ay = 0; ay < 3; ++ay)
    for (int ax = 0; ax < 3; ++ax) {
      const double bx = q2v(ax, xi), by = q2v(ay, et);
      const double ph = bx * by, px = q2d(ax, xi) * g.ihx * by, py = bx * q2d(ay, et) * g.ihy;
      const int64_t gn = (int64_t)(2 * cy + ay) * NX + (2 * cx + ax);
      const double l0 = w0 * ghat[gn] + w1 * ghat[g.nv + gn];
      const double l1 = w0 * ghat[g.nn + gn] + w1 * ghat[g.nv + g.nn + gn];
      v0 += l0 * ph;
      v1 += l1 * ph;
      g00 += l0 * px;
      g01 += l0 * py;
      g10 += l1 * px;
      g11 += l1 * py;
    }
  const double G00 = g00, G01 = 0.5 * (g01 + g10), G11 = g11;
  double eta, k;
  frozen_coef(m, G00, G01, G11, eta, k);
  double* o = table + lift_index(g, side, j, q, s);
  o[0] = v0;
  o[1] = v1;
  o[2] = G00;
  o[3] = G01;
  o[4] = G11;
  o[5] = eta;
  o[6] = k;
}

}  // namespace

hipError_t launch_lift_table(const Grid& g, const Model& m, const double* ghat, double* table,
                             hipStream_t s) {
  const int L = g.nx > g.ny ? g.nx : g.ny;
  const int64_t n = (int64_t)4 * L * 9;
  hipLaunchKernelGGL(lift_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, m,
                     ghat, table);
  return hipGetLastError();
}

}  // namespace pns
