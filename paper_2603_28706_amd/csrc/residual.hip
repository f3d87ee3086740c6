// Nonlinear slab residual in FP64 (Sec. 5.2 eq. slab-underint, with f = 0 and
// Dirichlet data imposed by Nitsche's method, eq. def-b-gam, eq. disc-residual):
//   R_v,mu = -( sum_nu K_t[mu][nu] M_x u_nu - m_t[mu] M_x v_prev )
//            + tau w_mu (B_gamma(g_D) - A_gamma(U_mu))_v
//   R_p,mu = tau w_mu (B_gamma(g_D) - A_gamma(U_mu))_p
// with the volume form S(Du):Dw - (u (x) u):grad w - (div w) pi - (div u) w_pi
// (Sec. 3.2 eq. pns-form) and on the boundary
//   (u.n)(u.w) - (u.n)^- (u.w) - (S(Du) n).w + pi (n.w) - (DS(G)(Dw) n).u
//   + q_sign (u.n) w_pi + gamma1 eta(G) / h_F (u.w) + gamma2 / h_F (u.n)(w.n),
// the inflow factor (u.n)^- evaluated at U itself, G = D ghat_D of the lifting
// (0 without one); B_gamma(g_D) is the same boundary form at the lifting's
// trace g with its own inflow factor, so the linear Nitsche terms act on u - g.
//
// Same tiling as the Jacobian action: one workgroup of 256 threads per tile of
// 15 x 7 owned cells plus the low-side halo cells, U's velocity (both Radau
// nodes) and v_prev staged in LDS, one thread per (cell, Radau node) looping
// over the Gauss rows, velocity shares summed in LDS, boundary faces in a phase
// of their own, owned entries written once.
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int TX = 15, TY = 7;
constexpr int HX = TX + 1, HY = TY + 1;
constexpr int BX = 2 * HX + 1, BY = 2 * HY + 1;
constexpr int kCells = HX * HY;
constexpr int kThreads = 2 * kCells;
// left-trace coupling of the Radau nodes: m_t = (xi_0(0), xi_1(0))
constexpr double kMt[2] = {1.5, -0.5};

// stress S(A) = eta(|A|) A, eta = nu_inf + nu (delta^2 + |A|^2)^((p-2)/2)
__device__ __forceinline__ double viscosity(const Model& m, double a00, double a01, double a11) {
  const double D2 = m.delta2 + a00 * a00 + 2.0 * a01 * a01 + a11 * a11;
  return m.nu_inf + m.nu * pow(D2, m.expo);
}

// one point q of a boundary face of a cell (node box offset lx0 / ly0 in the tile)
template <bool ATOMIC>
__device__ __forceinline__ void residual_face_point(const Model& m, const Grid& g, double tau,
                                                    int side, int q, int mu, int cx, int cy,
                                                    const double (*Xs)[BY][BX], int lx0, int ly0,
                                                    const double* __restrict__ U,
                                                    double (*acc)[BY][BX], double* pa) {
  const bool xface = side < 2;
  const double n0 = xface ? (side == 0 ? -1.0 : 1.0) : 0.0;
  const double n1 = xface ? 0.0 : (side == 2 ? -1.0 : 1.0);
  const double gq = q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]);
  const double wq = q == 0 ? kGW[0] : (q == 1 ? kGW[1] : kGW[2]);
  const double xi = xface ? (side == 0 ? 0.0 : 1.0) : gq;
  const double et = xface ? gq : (side == 2 ? 0.0 : 1.0);
  const double ihF = xface ? g.ihx : g.ihy;
  double vx[3], vy[3], dx[3], dy[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vx[a] = q2v(a, xi);
    vy[a] = q2v(a, et);
    dx[a] = q2d(a, xi) * g.ihx;
    dy[a] = q2d(a, et) * g.ihy;
  }
  double X[2] = {0, 0}, GX[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      const double x0 = Xs[2 * mu][ly0 + ay][lx0 + ax], x1 = Xs[2 * mu + 1][ly0 + ay][lx0 + ax];
      X[0] += x0 * ph; X[1] += x1 * ph;
      GX[0][0] += x0 * px; GX[0][1] += x0 * py;
      GX[1][0] += x1 * px; GX[1][1] += x1 * py;
    }
  const double* pv = U + (int64_t)mu * g.ns + g.nv + 3 * ((int64_t)cy * g.nx + cx);
  const double pi = pv[0] + pv[1] * (xi - 0.5) + pv[2] * (et - 0.5);
  const double a00 = GX[0][0], a01 = 0.5 * (GX[0][1] + GX[1][0]), a11 = GX[1][1];
  const double eta = viscosity(m, a00, a01, a11);
  const double sW = tau * (mu ? kWt[1] : kWt[0]) * wq * (xface ? g.hy : g.hx);
  const double un = X[0] * n0 + X[1] * n1;
  // the lifting's trace and the frozen Nitsche coefficients at its gradient
  double l0 = 0.0, l1 = 0.0, Gl00 = 0.0, Gl01 = 0.0, Gl11 = 0.0, etaG = m.etaD, kG = 0.0;
  if (m.lift) {
    const double* lt = m.lift + lift_index(g, side, xface ? cy : cx, q, mu);
    l0 = lt[0];
    l1 = lt[1];
    Gl00 = lt[2];
    Gl01 = lt[3];
    Gl11 = lt[4];
    etaG = lt[5];
    kG = lt[6];
  }
  const double e0 = X[0] - l0, e1 = X[1] - l1, en = e0 * n0 + e1 * n1;  // u - g
  const double pen1 = m.gamma1 * etaG * ihF, pen2 = m.gamma2 * ihF;
  double F0 = -eta * (a00 * n0 + a01 * n1) + pi * n0 + pen1 * e0 + pen2 * en * n0;
  double F1 = -eta * (a01 * n0 + a11 * n1) + pi * n1 + pen1 * e1 + pen2 * en * n1;
  if (m.convection) {
    const double neg = 0.5 * (fabs(un) - un);
    F0 += (un - neg) * X[0];
    F1 += (un - neg) * X[1];
    const double ln = l0 * n0 + l1 * n1;   // B^c(g_D, w) of the right-hand side
    const double lneg = 0.5 * (fabs(ln) - ln);
    F0 += lneg * l0;
    F1 += lneg * l1;
  }
  F0 *= sW;
  F1 *= sW;
  // -(DS(G)(Dw) n).(u - g): coefficient of d_j w_i, -(eta(G) S + k (G:S) G)_ij,
  // S = sym((u - g) (x) n)
  const double S00 = e0 * n0, S01 = 0.5 * (e0 * n1 + e1 * n0), S11 = e1 * n1;
  const double kGS = kG * (Gl00 * S00 + 2.0 * Gl01 * S01 + Gl11 * S11);
  const double G00 = -sW * (etaG * S00 + kGS * Gl00), G01 = -sW * (etaG * S01 + kGS * Gl01);
  const double G10 = G01, G11 = -sW * (etaG * S11 + kGS * Gl11);
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      lds_add<ATOMIC>(&acc[2 * mu][ly0 + ay][lx0 + ax], F0 * ph + G00 * px + G01 * py);
      lds_add<ATOMIC>(&acc[2 * mu + 1][ly0 + ay][lx0 + ax], F1 * ph + G10 * px + G11 * py);
    }
  if (pa) {
    const double P = sW * m.qsign * en;
    lds_add<ATOMIC>(&pa[0], P);
    lds_add<ATOMIC>(&pa[1], P * (xi - 0.5));
    lds_add<ATOMIC>(&pa[2], P * (et - 0.5));
  }
}

template <bool ORDERED>
__global__ __launch_bounds__(kThreads, 2) void residual_kernel(Grid g, Model m, double tau,
                                                               const double* __restrict__ U,
                                                               const double* __restrict__ vprev,
                                                               double* __restrict__ R,
                                                               int tiles_x) {
  __shared__ double Xs[4][BY][BX];    // U velocity: [mu*2 + comp]
  __shared__ double Vs[2][BY][BX];    // v_prev: [comp]
  __shared__ double acc[4][BY][BX];   // velocity sums: [mu*2 + comp]
  __shared__ double pacc[2][kCells][3];
  const int nb = gridDim.x, bq = nb >> 3, br = nb & 7;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int tile = xcd * bq + (xcd < br ? xcd : br) + slot;
  const int cx0 = (tile % tiles_x) * TX;
  const int cy0 = (tile / tiles_x) * TY;
  const int t = threadIdx.x;
  const int NX = 2 * g.nx + 1;
  const int gx0 = 2 * (cx0 - 1), gy0 = 2 * (cy0 - 1);

  // staging: every load of the thread issued before the first LDS store
  // (addresses clamped into the mesh, values outside it replaced by zero)
  {
    constexpr int kN = 6 * BY * BX, kSlices = (kN + kThreads - 1) / kThreads;
    double v[kSlices];
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const int i = min(t + s * kThreads, kN - 1);
      const int f = i / (BY * BX), r = i % (BY * BX);
      const int ly = r / BX, lx = r % BX;
      const int gx = gx0 + lx, gy = gy0 + ly;
      const bool in = gx >= 0 && gy >= 0 && gx <= 2 * g.nx && gy <= 2 * g.ny && (f < 4 || vprev);
      const int64_t gn = (int64_t)min(max(gy, 0), 2 * g.ny) * NX + min(max(gx, 0), 2 * g.nx);
      const double* src = f < 4 ? U + (int64_t)(f >> 1) * g.ns + (int64_t)(f & 1) * g.nn
                                : (vprev ? vprev + (int64_t)(f - 4) * g.nn : U);
      const double l = src[gn];
      v[s] = in ? l : 0.0;
    }
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const int i = t + s * kThreads;
      if (i < kN) {
        const int f = i / (BY * BX), r = i % (BY * BX);
        const int ly = r / BX, lx = r % BX;
        if (f < 4) {
          Xs[f][ly][lx] = v[s];
          acc[f][ly][lx] = 0.0;
        } else {
          Vs[f - 4][ly][lx] = v[s];
        }
      }
    }
  }
  __syncthreads();

  const int color = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const int mu = lane & 1, k = lane >> 1;
  const int hx = 2 * (k % (HX / 2)) + (color & 1), hy = 2 * (k / (HX / 2)) + (color >> 1);
  const int cx = cx0 - 1 + hx, cy = cy0 - 1 + hy;
  const bool valid = cx >= 0 && cy >= 0 && cx < g.nx && cy < g.ny;
  const int lx0 = 2 * hx, ly0 = 2 * hy;
  const int lc = hy * HX + hx;
  // ordered mode: this cell's nodal sums, added class by class after the rows
  double racc[2][9];
#pragma unroll
  for (int i = 0; i < 9; ++i) racc[0][i] = racc[1][i] = 0.0;
  (void)racc;
  if (valid) {
    const int other = 1 - mu;
    const double kself = mu ? kKt[1][1] : kKt[0][0], koth = mu ? kKt[1][0] : kKt[0][1];
    const double mtm = mu ? kMt[1] : kMt[0];
    const int64_t cell = (int64_t)cy * g.nx + cx;
    const double* pv = U + (int64_t)mu * g.ns + g.nv + 3 * cell;
    const double pp0 = pv[0], pp1 = pv[1], pp2 = pv[2];
    const double sfac = tau * (mu ? kWt[1] : kWt[0]);
    const double area = g.hx * g.hy;
    double op[3] = {0, 0, 0};
#pragma unroll 1
    for (int qy = 0; qy < 3; ++qy) {
      const double gyq = qy == 0 ? kGP[0] : (qy == 1 ? kGP[1] : kGP[2]);
      const double gwy = qy == 0 ? kGW[0] : (qy == 1 ? kGW[1] : kGW[2]);
      // contraction along y: this node's velocity (values, y-derivatives), the
      // other node's velocity values and v_prev values
      double x0y[3], x0d[3], x1y[3], x1d[3], o0[3], o1[3], v0[3], v1[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        x0y[ax] = x0d[ax] = x1y[ax] = x1d[ax] = o0[ax] = o1[ax] = v0[ax] = v1[ax] = 0.0;
#pragma unroll
      for (int ay = 0; ay < 3; ++ay) {
        const double bv = q2v(ay, gyq), bd = q2d(ay, gyq);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int ly = ly0 + ay, lx = lx0 + ax;
          const double a0 = Xs[2 * mu][ly][lx], a1 = Xs[2 * mu + 1][ly][lx];
          x0y[ax] += bv * a0; x0d[ax] += bd * a0;
          x1y[ax] += bv * a1; x1d[ax] += bd * a1;
          o0[ax] += bv * Xs[2 * other][ly][lx];
          o1[ax] += bv * Xs[2 * other + 1][ly][lx];
          v0[ax] += bv * Vs[0][ly][lx];
          v1[ax] += bv * Vs[1][ly][lx];
        }
      }
      double S1a[3] = {0, 0, 0}, S2a[3] = {0, 0, 0}, S1b[3] = {0, 0, 0}, S2b[3] = {0, 0, 0};
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        double X0 = 0, X1 = 0, X0x = 0, X0y = 0, X1x = 0, X1y = 0, O0 = 0, O1 = 0, P0 = 0, P1 = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const double bv = q2v(ax, kGP[qx]), bd = q2d(ax, kGP[qx]);
          X0 += bv * x0y[ax]; X0x += bd * x0y[ax]; X0y += bv * x0d[ax];
          X1 += bv * x1y[ax]; X1x += bd * x1y[ax]; X1y += bv * x1d[ax];
          O0 += bv * o0[ax]; O1 += bv * o1[ax];
          P0 += bv * v0[ax]; P1 += bv * v1[ax];
        }
        X0x *= g.ihx; X1x *= g.ihx;
        X0y *= g.ihy; X1y *= g.ihy;
        // time derivative and jump: sum_nu K_t[mu][nu] u_nu - m_t[mu] v_prev
        const double W0 = kself * X0 + koth * O0 - mtm * P0;
        const double W1 = kself * X1 + koth * O1 - mtm * P1;
        const double a00 = X0x, a01 = 0.5 * (X0y + X1x), a11 = X1y;
        const double eta = viscosity(m, a00, a01, a11);
        const double W = area * kGW[qx] * gwy;
        const double sW = sfac * W;
        const double pi = pp0 + pp1 * (kGP[qx] - 0.5) + pp2 * (gyq - 0.5);
        double G00 = eta * a00 - pi, G01 = eta * a01, G10 = eta * a01, G11 = eta * a11 - pi;
        if (m.convection) {
          G00 -= X0 * X0;
          G01 -= X0 * X1;
          G10 -= X1 * X0;
          G11 -= X1 * X1;
        }
        G00 *= sW * g.ihx; G10 *= sW * g.ihx;
        G01 *= sW * g.ihy; G11 *= sW * g.ihy;
        const double V0 = W * W0, V1 = W * W1;
        const double P = -sW * (X0x + X1y);
        op[0] += P;
        op[1] += P * (kGP[qx] - 0.5);
        op[2] += P * (gyq - 0.5);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const double bv = q2v(ax, kGP[qx]), bd = q2d(ax, kGP[qx]);
          S1a[ax] += bv * V0 + bd * G00;
          S2a[ax] += bv * G01;
          S1b[ax] += bv * V1 + bd * G10;
          S2b[ax] += bv * G11;
        }
      }
#pragma unroll
      for (int ay = 0; ay < 3; ++ay) {
        const double bv = q2v(ay, gyq), bd = q2d(ay, gyq);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const double r0 = bv * S1a[ax] + bd * S2a[ax], r1 = bv * S1b[ax] + bd * S2b[ax];
          if (ORDERED) {
            racc[0][3 * ay + ax] += r0;
            racc[1][3 * ay + ax] += r1;
          } else {
            atomicAdd(&acc[2 * mu][ly0 + ay][lx0 + ax], r0);
            atomicAdd(&acc[2 * mu + 1][ly0 + ay][lx0 + ax], r1);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) pacc[mu][lc][j] = op[j];
  }
  if (ORDERED) {
    // the four parity classes one after the other (cells of one class share
    // no node): every node sums in a fixed order
    for (int c = 0; c < 4; ++c) {
      if (valid && color == c) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          acc[2 * mu][ly0 + i / 3][lx0 + i % 3] += racc[0][i];
          acc[2 * mu + 1][ly0 + i / 3][lx0 + i % 3] += racc[1][i];
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();

  if (cx0 == 0 || cy0 == 0 || cx0 + TX >= g.nx || cy0 + TY >= g.ny) {
    // the face cell of (side, cell j along it) in tile coordinates, or false
    auto face_cell = [&](int side, int j, int& fhx, int& fhy, int& fcx, int& fcy) {
      if (side < 2) {
        fhx = (side == 0 ? 0 : g.nx - 1) - cx0 + 1;
        fhy = j;
      } else {
        fhx = j;
        fhy = (side == 2 ? 0 : g.ny - 1) - cy0 + 1;
      }
      fcx = cx0 - 1 + fhx;
      fcy = cy0 - 1 + fhy;
      return !(fhx < 0 || fhx >= HX || fhy < 0 || fhy >= HY || fcx < 0 || fcy < 0 ||
               fcx >= g.nx || fcy >= g.ny);
    };
    if (!ORDERED) {
      for (int p = t; p < 4 * HX * 6; p += kThreads) {
        const int side = p / (HX * 6), r = p % (HX * 6);
        const int j = r / 6, q = (r >> 1) % 3, fmu = r & 1;
        int fhx, fhy, fcx, fcy;
        if (!face_cell(side, j, fhx, fhy, fcx, fcy)) continue;
        residual_face_point<true>(m, g, tau, side, q, fmu, fcx, fcy, Xs, 2 * fhx, 2 * fhy, U,
                                  acc, (fhx >= 1 && fhy >= 1) ? pacc[fmu][fhy * HX + fhx] : nullptr);
      }
    } else {
      // side by side, cells of one parity along the side at a time, the three
      // points of a cell in turn
      for (int side = 0; side < 4; ++side)
        for (int par = 0; par < 2; ++par) {
          const int j = 2 * (t >> 1) + par, fmu = t & 1;
          int fhx, fhy, fcx, fcy;
          if (t < HX * 2 && j < HX && face_cell(side, j, fhx, fhy, fcx, fcy))
            for (int q = 0; q < 3; ++q)
              residual_face_point<false>(m, g, tau, side, q, fmu, fcx, fcy, Xs, 2 * fhx, 2 * fhy,
                                         U, acc,
                                         (fhx >= 1 && fhy >= 1) ? pacc[fmu][fhy * HX + fhx]
                                                                : nullptr);
          __syncthreads();
        }
    }
    __syncthreads();
  }

  // R = -(sums) on the owned cells and nodes
  for (int i = t; i < 2 * kCells * 3; i += kThreads) {
    const int pmu = i / (kCells * 3), r = i % (kCells * 3);
    const int c = r / 3, j = r % 3;
    const int ccx = cx0 - 1 + c % HX, ccy = cy0 - 1 + c / HX;
    if (ccx >= cx0 && ccy >= cy0 && ccx < g.nx && ccy < g.ny)
      R[(int64_t)pmu * g.ns + g.nv + 3 * ((int64_t)ccy * g.nx + ccx) + j] = -pacc[pmu][c][j];
  }
  const int gx_end = (cx0 + TX >= g.nx) ? 2 * g.nx + 1 : 2 * (cx0 + TX);
  const int gy_end = (cy0 + TY >= g.ny) ? 2 * g.ny + 1 : 2 * (cy0 + TY);
  const int nox = gx_end - 2 * cx0, noy = gy_end - 2 * cy0;
  for (int i = t; i < 4 * (2 * TY + 1) * 32; i += kThreads) {
    const int s = i / ((2 * TY + 1) * 32), r = i % ((2 * TY + 1) * 32);
    const int ox = r % 32, oy = r / 32;
    if (ox < nox && oy < noy) {
      const int64_t gn = (int64_t)(2 * cy0 + oy) * NX + (2 * cx0 + ox);
      R[(int64_t)(s >> 1) * g.ns + (int64_t)(s & 1) * g.nn + gn] = -acc[s][oy + 2][ox + 2];
    }
  }
}

}  // namespace

hipError_t launch_residual(const Grid& g, const Model& m, double tau, const double* U,
                           const double* vprev, double* R, hipStream_t s) {
  const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY;
  if (m.ordered)
    hipLaunchKernelGGL(residual_kernel<true>, dim3(tx * ty), dim3(kThreads), 0, s, g, m, tau, U,
                       vprev, R, tx);
  else
    hipLaunchKernelGGL(residual_kernel<false>, dim3(tx * ty), dim3(kThreads), 0, s, g, m, tau, U,
                       vprev, R, tx);
  return hipGetLastError();
}

}  // namespace pns
