// Inhomogeneous Dirichlet data (Sec. 3.2, eq. def-b-gam): the lifting ghat_D,
// a Q2 velocity field per Radau node, evaluated once at every boundary face
// point of the quadrilateral mesh — its value (the data g_D), its symmetric
// gradient G = D ghat_D from the boundary cell's nine nodes, and the frozen
// Nitsche coefficients eta(G), k(G) — for the two Radau nodes and the slab
// midpoint (the lifting interpolated linearly in time, as the surrogate
// patches freeze every coefficient there).  The action, the residual and the
// cell matrices read the table at their face points, which keeps the
// evaluation out of their register budgets.  Hexahedra: the same table over
// the six sides, and the data term B_gamma(g_D, .) of the residual formed per
// boundary cell into the action's per-cell result slots.
#include "hex3.h"

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


// one thread per (side, face cell, Gauss point, time slot) of a hexahedral mesh
__global__ __launch_bounds__(256) void lift3_table_kernel(Grid3 g, Model m,
                                                          const double* __restrict__ ghat,
                                                          double* __restrict__ table) {
  const int64_t total = lift3_table_doubles(g) / kLift3Vals;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int s = (int)(id % 3), qa = (int)((id / 3) % 9);
  int64_t f = id / 27;
  const int n3[3] = {g.nx, g.ny, g.nz};
  int sd = 0;
  for (; sd < 5; ++sd) {
    const int kk = sd >> 1;
    const int64_t nf = (int64_t)n3[(kk + 1) % 3] * n3[(kk + 2) % 3];
    if (f < nf) break;
    f -= nf;
  }
  const int k = sd >> 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
  const int i1 = (int)(f % n3[k1]), i2 = (int)(f / n3[k1]);
  int cc[3];
  cc[k] = (sd & 1) ? n3[k] - 1 : 0;
  cc[k1] = i1;
  cc[k2] = i2;
  double xi[3];
  xi[k] = (sd & 1) ? 1.0 : 0.0;
  xi[k1] = qa % 3 == 0 ? kGP[0] : (qa % 3 == 1 ? kGP[1] : kGP[2]);
  xi[k2] = qa / 3 == 0 ? kGP[0] : (qa / 3 == 1 ? kGP[1] : kGP[2]);
  const double w0 = s == 0 ? 1.0 : (s == 1 ? 0.0 : kXiMid[0]);
  const double w1 = s == 0 ? 0.0 : (s == 1 ? 1.0 : kXiMid[1]);
  double v[3] = {0, 0, 0}, Gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < kNb3; ++a) {
    double ph, gr[3];
    basis3(g, a, xi, ph, gr);
    const int64_t node = node_index3(g, cc[0], cc[1], cc[2], a);
    for (int c = 0; c < 3; ++c) {
      const double l = w0 * ghat[(int64_t)c * g.nn + node] + w1 * ghat[g.nv + (int64_t)c * g.nn + node];
      v[c] += l * ph;
      for (int d = 0; d < 3; ++d) Gr[c][d] += l * gr[d];
    }
  }
  double* o = table + lift3_index(g, sd, i1, i2, qa, s);
  o[0] = v[0];
  o[1] = v[1];
  o[2] = v[2];
  o[3] = Gr[0][0];
  o[4] = 0.5 * (Gr[0][1] + Gr[1][0]);
  o[5] = 0.5 * (Gr[0][2] + Gr[2][0]);
  o[6] = Gr[1][1];
  o[7] = 0.5 * (Gr[1][2] + Gr[2][1]);
  o[8] = Gr[2][2];
  frozen_coef3(m, o + 3, o[9], o[10]);
}

// The data term on hexahedra: per cell, Radau node and local unknown (81
// velocity, 4 pressure; one thread each) the slot value -tau w_mu B_gamma(g_D,
// w) summed over the cell's boundary sides and their 3 x 3 face points (zero
// for interior cells), so that the action's node gather, y = b - sum, adds
// B_gamma(g_D, .) to b.  Slot layout of the action: velocity of node a,
// Radau node mu, component c at 6 a + 3 mu + c, pressure j at 162 + 4 mu + j.
__global__ __launch_bounds__(256) void lift3_rhs_kernel(Grid3 g, Model m, double tau,
                                                        const double* __restrict__ table,
                                                        double* __restrict__ E) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nc * 170) return;
  const int64_t cell = id / 170;
  const int r = (int)(id % 170);
  const int mu = r < 162 ? (r % 6) / 3 : (r - 162) / 4;
  const int comp = r < 162 ? r % 3 : -1, a = r < 162 ? r / 6 : -1, jp = r < 162 ? -1 : (r - 162) % 4;
  const int cc[3] = {(int)(cell % g.nx), (int)((cell / g.nx) % g.ny),
                     (int)(cell / ((int64_t)g.nx * g.ny))};
  const int n3[3] = {g.nx, g.ny, g.nz};
  const double h[3] = {g.hx, g.hy, g.hz};
  double acc = 0.0;
  for (int sd = 0; sd < 6; ++sd) {
    const int k = sd >> 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    if (cc[k] != ((sd & 1) ? n3[k] - 1 : 0)) continue;
    double n[3] = {0, 0, 0};
    n[k] = (sd & 1) ? 1.0 : -1.0;
    const double ihF = 1.0 / h[k];
    for (int qa = 0; qa < 9; ++qa) {
      double xi[3];
      xi[k] = (sd & 1) ? 1.0 : 0.0;
      xi[k1] = qa % 3 == 0 ? kGP[0] : (qa % 3 == 1 ? kGP[1] : kGP[2]);
      xi[k2] = qa / 3 == 0 ? kGP[0] : (qa / 3 == 1 ? kGP[1] : kGP[2]);
      const double W = tau * (mu ? kWt[1] : kWt[0]) *
                       (qa % 3 == 0 ? kGW[0] : (qa % 3 == 1 ? kGW[1] : kGW[2])) *
                       (qa / 3 == 0 ? kGW[0] : (qa / 3 == 1 ? kGW[1] : kGW[2])) * h[k1] * h[k2];
      const double* lt = table + lift3_index(g, sd, cc[k1], cc[k2], qa, mu);
      const double gv[3] = {lt[0], lt[1], lt[2]};
      double G[3][3];
      sym3(lt + 3, G);
      const double etaG = lt[9], kG = lt[10];
      const double gn = gv[0] * n[0] + gv[1] * n[1] + gv[2] * n[2];
      double b = 0.0;
      if (a >= 0) {
        // velocity test w = phi_a e_comp
        double ph, gr[3];
        basis3(g, a, xi, ph, gr);
        const double grn = gr[0] * n[0] + gr[1] * n[1] + gr[2] * n[2];
        const double grg = gr[0] * gv[0] + gr[1] * gv[1] + gr[2] * gv[2];
        // (D w n) . g and G : D w = (G grad phi)_comp
        const double dwng = 0.5 * (gv[comp] * grn + n[comp] * grg);
        const double gdw = G[comp][0] * gr[0] + G[comp][1] * gr[1] + G[comp][2] * gr[2];
        const double Gng = (G[0][0] * n[0] + G[0][1] * n[1] + G[0][2] * n[2]) * gv[0] +
                           (G[1][0] * n[0] + G[1][1] * n[1] + G[1][2] * n[2]) * gv[1] +
                           (G[2][0] * n[0] + G[2][1] * n[1] + G[2][2] * n[2]) * gv[2];
        if (m.convection) b -= 0.5 * (fabs(gn) - gn) * gv[comp] * ph;
        b -= etaG * dwng + kG * gdw * Gng;
        b += m.gamma1 * etaG * ihF * gv[comp] * ph + m.gamma2 * ihF * gn * n[comp] * ph;
      } else {
        // pressure test psi_j: 1 or xi_d - 1/2
        const double psi = jp == 0 ? 1.0 : xi[jp - 1] - 0.5;
        b += m.qsign * gn * psi;
      }
      acc += W * b;
    }
  }
  E[cell * 170 + r] = -acc;
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

hipError_t launch_lift3_table(const Grid3& g, const Model& m, const double* ghat, double* table,
                              hipStream_t s) {
  const int64_t n = lift3_table_doubles(g) / kLift3Vals;
  hipLaunchKernelGGL(lift3_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, m,
                     ghat, table);
  return hipGetLastError();
}

hipError_t launch_lift3_rhs(const Grid3& g, const Model& m, double tau, const double* table,
                            double* E, hipStream_t s) {
  const int64_t n = g.nc * 170;
  hipLaunchKernelGGL(lift3_rhs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, m,
                     tau, table, E);
  return hipGetLastError();
}

}  // namespace pns
