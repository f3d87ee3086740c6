// Matrix-free slab Jacobian action on the finest level (Sec. 5.2,
// eq. slab-underint-jac): y_mu = sum_nu K_t[mu][nu] M_x x_nu + tau w_mu J_mu x_mu,
// with J_mu the spatial linearisation at the Radau node mu (viscous volume term
// with the Picard / exact / clipped tangent of Sec. 4.2-4.4, convection in
// divergence form, pressure coupling, state-dependent boundary flux and the
// Nitsche terms of eq. def-b-gam).
//
// Design (gfx950, wave64):
// * one workgroup per tile of TX x TY owned cells; it also evaluates the
//   one-cell halo on the low x / low y side, so every node it owns receives all
//   of its cell contributions inside the workgroup and each output is written
//   exactly once (no global atomics, no zero fill);
// * the tile's nodal values of x and u_k (both Radau nodes) are staged in LDS
//   with coalesced row loads;
// * three threads per (cell, Radau node mu), one per row qy of the 3x3 Gauss
//   points; a wave holds the two Radau nodes of the 32 cells of one parity
//   class of the tile (cells of one class share no node, so the LDS atomics of
//   a wave never collide) for one row qy (wave-uniform); each thread contracts the nodal values along y at its row (sum
//   factorisation), evaluates values / gradients / tangent / fluxes at its
//   three points, and forms its share of the 9 nodal results by the transposed
//   contractions; the temporal mass coupling K_t[mu][nu] x_nu is formed at the
//   points from the partner lane's values (DPP lane swap);
// * the tangent scalars (Delta^2, mu, eta, clip factor, kappa) are evaluated
//   in FP64 in both precisions; everything else in the storage type T;
// * shares are summed in LDS with LDS atomics (summation order inside a tile
//   is not fixed), then the owned nodes are written coalesced.
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int TX = 15, TY = 7;            // owned cells per tile
constexpr int HX = TX + 1, HY = TY + 1;   // evaluated cells (with low-side halo)
constexpr int BX = 2 * TX + 4, BY = 2 * TY + 3;  // LDS node box (x padded to 34)
constexpr int kCells = HX * HY;           // 128
constexpr int kThreads = 6 * kCells;      // 768: (cell, mu, qy)

// FP64 elementary functions for the tangent scalars, specialised to the
// arguments that occur here (finite, positive, normal D2; |exponent argument|
// well below the overflow range), without the special-case handling of the
// general library routines.
// 1/d: hardware reciprocal seed refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}
// 1/sqrt(a), a > 0: hardware seed refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double a) {
  double r = __builtin_amdgcn_rsq(a);
  r = r * fma(-0.5 * a * r, r, 1.5);
  r = r * fma(-0.5 * a * r, r, 1.5);
  return r;
}
// log(x), x > 0 normal: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.172, series to s^21.
__device__ __forceinline__ double log_pos(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double sv = f * rcp_nr(2.0 + f);
  const double s2 = sv * sv;
  double q = 2.0 / 21.0;
  q = fma(q, s2, 2.0 / 19.0);
  q = fma(q, s2, 2.0 / 17.0);
  q = fma(q, s2, 2.0 / 15.0);
  q = fma(q, s2, 2.0 / 13.0);
  q = fma(q, s2, 2.0 / 11.0);
  q = fma(q, s2, 2.0 / 9.0);
  q = fma(q, s2, 2.0 / 7.0);
  q = fma(q, s2, 2.0 / 5.0);
  q = fma(q, s2, 2.0 / 3.0);
  const double lm = fma(sv * s2, q, 2.0 * sv);
  const double de = (double)e;
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, lm));
}
// exp(y), |y| < 700: Cody-Waite reduction y = k ln2 + r, |r| <= ln2/2, Taylor
// polynomial of degree 13 for exp(r), scaled by 2^k.
__device__ __forceinline__ double exp_small(double y) {
  const double k = rint(y * 1.44269504088896340736);
  double r = fma(-k, 6.93147180369123816490e-01, y);
  r = fma(-k, 1.90821492927058770002e-10, r);
  double q = 1.0 / 6227020800.0;
  q = fma(q, r, 1.0 / 479001600.0);
  q = fma(q, r, 1.0 / 39916800.0);
  q = fma(q, r, 1.0 / 3628800.0);
  q = fma(q, r, 1.0 / 362880.0);
  q = fma(q, r, 1.0 / 40320.0);
  q = fma(q, r, 1.0 / 5040.0);
  q = fma(q, r, 1.0 / 720.0);
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return ldexp(q, (int)k);
}

// Tangent scalars at a point, A = D(u_k):  eta = nu_inf + mu,
// mu = nu (delta^2 + |A|^2)^((p-2)/2);  T(B) = eta B + kappa (A:B) A with
// kappa = 0 (Picard), (p-2) mu / Delta^2 (exact Newton), or the clipped
// s (p-2) mu / Delta^2 = (p-2)/Delta^2 min(mu, sigma_max / |A|) (modified Newton).
template <int LIN>
__device__ __forceinline__ void tangent_coef(const Model& m, double a00, double a01, double a11,
                                             double& eta, double& kappa) {
  const double a2 = a00 * a00 + 2.0 * a01 * a01 + a11 * a11;
  const double D2 = m.delta2 + a2;
  const double mu = m.nu * exp_small(m.expo * log_pos(D2));
  eta = m.nu_inf + mu;
  if (LIN == PNS_PICARD) {
    kappa = 0.0;
  } else {
    const double c = (m.p - 2.0) * rcp_nr(D2);
    if (LIN == PNS_MODIFIED_NEWTON) {
      // a2 = 0 makes the rank-one term vanish whatever kappa is
      const double lim = a2 > 0.0 ? m.sigma_max * rsqrt_nr(a2) : mu;
      kappa = c * fmin(mu, lim);
    } else {
      kappa = c * mu;
    }
  }
}

// value held by the partner lane (lane ^ 1): the other Radau node of the cell;
// DPP quad permutation [1,0,3,2]
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_pair(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One point of a Dirichlet face of the cell: value / gradient test coefficients,
// contracted directly against the 9 nodes and added to the LDS sums.
template <typename T, int LIN, bool CONV>
__device__ __forceinline__ void face_point(const Model& m, const Grid& g, T sfac, int side, int q,
                                        const T (*Xs)[BY][BX], const T (*Us)[BY][BX], int mu,
                                        int lx0, int ly0, T p0, T p1, T p2,
                                        double (*acc)[BY][BX], double* pacc) {
  // side: 0 x=0 (n=-e_x), 1 x=1 (n=+e_x), 2 y=0 (n=-e_y), 3 y=1 (n=+e_y)
  const bool xface = side < 2;
  const double nxv = xface ? (side == 0 ? -1.0 : 1.0) : 0.0;
  const double nyv = xface ? 0.0 : (side == 2 ? -1.0 : 1.0);
  const double hF = xface ? g.hx : g.hy;
  const double flen = xface ? g.hy : g.hx;
  const double xi = xface ? (side == 0 ? 0.0 : 1.0) : kGP[q];
  const double et = xface ? kGP[q] : (side == 2 ? 0.0 : 1.0);
  const T etaD = (T)m.etaD;
  const T pen1 = (T)(m.gamma1 * m.etaD / hF);
  const T pen2 = (T)(m.gamma2 / hF);
  const T n0 = (T)nxv, n1 = (T)nyv;
  T vx[3], vy[3], dx[3], dy[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vx[a] = (T)q2v(a, xi);
    vy[a] = (T)q2v(a, et);
    dx[a] = (T)(q2d(a, xi) / g.hx);
    dy[a] = (T)(q2d(a, et) / g.hy);
  }
  T U[2] = {0, 0}, GU[2][2] = {{0, 0}, {0, 0}}, X[2] = {0, 0}, GX[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      const T u0 = Us[2 * mu][ly0 + ay][lx0 + ax], u1 = Us[2 * mu + 1][ly0 + ay][lx0 + ax];
      const T x0 = Xs[2 * mu][ly0 + ay][lx0 + ax], x1 = Xs[2 * mu + 1][ly0 + ay][lx0 + ax];
      U[0] += u0 * ph; U[1] += u1 * ph;
      GU[0][0] += u0 * px; GU[0][1] += u0 * py;
      GU[1][0] += u1 * px; GU[1][1] += u1 * py;
      X[0] += x0 * ph; X[1] += x1 * ph;
      GX[0][0] += x0 * px; GX[0][1] += x0 * py;
      GX[1][0] += x1 * px; GX[1][1] += x1 * py;
    }
  const T xp = p0 + p1 * (T)(xi - 0.5) + p2 * (T)(et - 0.5);
  const T a00 = GU[0][0], a01 = (T)0.5 * (GU[0][1] + GU[1][0]), a11 = GU[1][1];
  const T b00 = GX[0][0], b01 = (T)0.5 * (GX[0][1] + GX[1][0]), b11 = GX[1][1];
  double eta_d, kap_d;
  tangent_coef<LIN>(m, (double)a00, (double)a01, (double)a11, eta_d, kap_d);
  const T eta = (T)eta_d, kap = (T)kap_d;
  const T ab = a00 * b00 + (T)2 * a01 * b01 + a11 * b11;
  const T T00 = eta * b00 + kap * ab * a00;
  const T T01 = eta * b01 + kap * ab * a01;
  const T T11 = eta * b11 + kap * ab * a11;
  const T sW = sfac * (T)(kGW[q] * flen);
  const T un = U[0] * n0 + U[1] * n1;
  const T xn = X[0] * n0 + X[1] * n1;
  T F0 = -(T00 * n0 + T01 * n1) + xp * n0 + pen1 * X[0] + pen2 * xn * n0;
  T F1 = -(T01 * n0 + T11 * n1) + xp * n1 + pen1 * X[1] + pen2 * xn * n1;
  if (CONV) {
    const T neg = (T)0.5 * (fabs(un) - un);
    F0 += un * X[0] - neg * X[0];
    F1 += un * X[1] - neg * X[1];
    if (LIN != PNS_PICARD) {
      F0 += xn * U[0];
      F1 += xn * U[1];
    }
  }
  F0 *= sW;
  F1 *= sW;
  // -eta_D (Dw n).x  ->  coefficient of d_j w_i : -eta_D (x_i n_j + x_j n_i)/2
  const T c = -sW * etaD * (T)0.5;
  const T G00 = c * (X[0] * n0 + X[0] * n0), G01 = c * (X[0] * n1 + X[1] * n0);
  const T G10 = c * (X[1] * n0 + X[0] * n1), G11 = c * (X[1] * n1 + X[1] * n1);
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      atomicAdd(&acc[2 * mu][ly0 + ay][lx0 + ax], (double)(F0 * ph + G00 * px + G01 * py));
      atomicAdd(&acc[2 * mu + 1][ly0 + ay][lx0 + ax], (double)(F1 * ph + G10 * px + G11 * py));
    }
  const T P = sW * (T)m.qsign * xn;
  atomicAdd(&pacc[0], (double)P);
  atomicAdd(&pacc[1], (double)(P * (T)(xi - 0.5)));
  atomicAdd(&pacc[2], (double)(P * (T)(et - 0.5)));
}

template <typename T, int LIN, bool CONV, int MODE>
__global__ __launch_bounds__(kThreads) void cell_apply_kernel(Grid g, Model m, double tau,
                                                              const T* __restrict__ uk,
                                                              const T* __restrict__ x,
                                                              const T* __restrict__ b,
                                                              T* __restrict__ y, int tiles_x) {
  __shared__ T Xs[4][BY][BX];   // x: [mu*2 + comp]
  __shared__ T Us[4][BY][BX];   // u_k: [mu*2 + comp]
  __shared__ double acc[4][BY][BX];  // results: [mu*2 + comp]
  __shared__ double pacc[2][kCells][3];
  const int tile = blockIdx.x;
  const int cx0 = (tile % tiles_x) * TX;
  const int cy0 = (tile / tiles_x) * TY;
  const int t = threadIdx.x;
  const int NX = 2 * g.nx + 1;
  const int gx0 = 2 * (cx0 - 1), gy0 = 2 * (cy0 - 1);

  // stage x and u_k of the node box, zero the sums
  for (int i = t; i < 4 * BY * BX; i += kThreads) {
    const int f = i / (BY * BX), r = i % (BY * BX);
    const int ly = r / BX, lx = r % BX;
    const int gx = gx0 + lx, gy = gy0 + ly;
    T xv = 0, uv = 0;
    if (gx >= 0 && gy >= 0 && gx <= 2 * g.nx && gy <= 2 * g.ny) {
      const int64_t gn = (int64_t)gy * NX + gx;
      xv = x[(int64_t)(f >> 1) * g.ns + (int64_t)(f & 1) * g.nn + gn];
      uv = uk[(int64_t)(f >> 1) * g.nv + (int64_t)(f & 1) * g.nn + gn];
    }
    Xs[f][ly][lx] = xv;
    Us[f][ly][lx] = uv;
    acc[f][ly][lx] = 0.0;
  }
  for (int i = t; i < 2 * kCells * 3; i += kThreads) (&pacc[0][0][0])[i] = 0.0;
  __syncthreads();

  // wave w: row qy = w / 4, parity class w % 4; lane: (cell of the class, mu)
  const int qy = __builtin_amdgcn_readfirstlane(t >> 8);
  const int color = (t >> 6) & 3, lane = t & 63;
  const int mu = lane & 1, k = lane >> 1;
  const int hx = 2 * (k % (HX / 2)) + (color & 1), hy = 2 * (k / (HX / 2)) + (color >> 1);
  const int lc = hy * HX + hx;
  const int cx = cx0 - 1 + hx, cy = cy0 - 1 + hy;
  const bool valid = cx >= 0 && cy >= 0 && cx < g.nx && cy < g.ny;
  const int lx0 = 2 * hx, ly0 = 2 * hy;

  // every lane takes part in the pair exchange below, valid or not
  {
    const int other = 1 - mu;
    const T kself = (T)kKt[mu][mu], koth = (T)kKt[mu][other];
    const int64_t cell = (int64_t)(valid ? cy : 0) * g.nx + (valid ? cx : 0);
    const T* xm = x + (int64_t)mu * g.ns + g.nv + 3 * cell;
    T pp[3] = {xm[0], xm[1], xm[2]};
    const T sfac = (T)(tau * kWt[mu]);
    const T ihx = (T)(1.0 / g.hx), ihy = (T)(1.0 / g.hy);
    const T area = (T)(g.hx * g.hy);

    // contraction along y at row qy: f_y[ax] (values), f_d[ax] (y-derivatives)
    T u0y[3], u0d[3], u1y[3], u1d[3], x0y[3], x0d[3], x1y[3], x1d[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      u0y[ax] = u0d[ax] = u1y[ax] = u1d[ax] = (T)0;
      x0y[ax] = x0d[ax] = x1y[ax] = x1d[ax] = (T)0;
    }
#pragma unroll
    for (int ay = 0; ay < 3; ++ay) {
      T bv, bd;
      // row-dependent 1D basis at the Gauss point qy (select, not a table load)
      bv = qy == 0 ? (T)q2v(ay, kGP[0]) : (qy == 1 ? (T)q2v(ay, kGP[1]) : (T)q2v(ay, kGP[2]));
      bd = qy == 0 ? (T)q2d(ay, kGP[0]) : (qy == 1 ? (T)q2d(ay, kGP[1]) : (T)q2d(ay, kGP[2]));
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int ly = ly0 + ay, lx = lx0 + ax;
        const T u0 = Us[2 * mu][ly][lx], u1 = Us[2 * mu + 1][ly][lx];
        const T x0 = Xs[2 * mu][ly][lx], x1 = Xs[2 * mu + 1][ly][lx];
        u0y[ax] += bv * u0; u0d[ax] += bd * u0;
        u1y[ax] += bv * u1; u1d[ax] += bd * u1;
        x0y[ax] += bv * x0; x0d[ax] += bd * x0;
        x1y[ax] += bv * x1; x1d[ax] += bd * x1;
      }
    }
    const double gyq = qy == 0 ? kGP[0] : (qy == 1 ? kGP[1] : kGP[2]);
    const double gwy = qy == 0 ? kGW[0] : (qy == 1 ? kGW[1] : kGW[2]);
    // per-point coefficients of the tests phi (A*), d/dx phi (B*), d/dy phi (C*)
    T S1a[3] = {0, 0, 0}, S2a[3] = {0, 0, 0}, S1b[3] = {0, 0, 0}, S2b[3] = {0, 0, 0};
    T op[3] = {0, 0, 0};
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
      T U0 = 0, U1 = 0, U0x = 0, U0y = 0, U1x = 0, U1y = 0;
      T X0 = 0, X1 = 0, X0x = 0, X0y = 0, X1x = 0, X1y = 0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
        U0 += bv * u0y[ax]; U0x += bd * u0y[ax]; U0y += bv * u0d[ax];
        U1 += bv * u1y[ax]; U1x += bd * u1y[ax]; U1y += bv * u1d[ax];
        X0 += bv * x0y[ax]; X0x += bd * x0y[ax]; X0y += bv * x0d[ax];
        X1 += bv * x1y[ax]; X1x += bd * x1y[ax]; X1y += bv * x1d[ax];
      }
      // temporal mass coupling at the point: w = K_t[mu][mu] x_mu + K_t[mu][other] x_other
      const T W0 = kself * X0 + koth * swap_pair(X0);
      const T W1 = kself * X1 + koth * swap_pair(X1);
      U0x *= ihx; U1x *= ihx; X0x *= ihx; X1x *= ihx;
      U0y *= ihy; U1y *= ihy; X0y *= ihy; X1y *= ihy;
      const T a00 = U0x, a01 = (T)0.5 * (U0y + U1x), a11 = U1y;
      const T b00 = X0x, b01 = (T)0.5 * (X0y + X1x), b11 = X1y;
      double eta_d, kap_d;
      tangent_coef<LIN>(m, (double)a00, (double)a01, (double)a11, eta_d, kap_d);
      const T eta = (T)eta_d, kap = (T)kap_d;
      const T ab = a00 * b00 + (T)2 * a01 * b01 + a11 * b11;
      const T xp = pp[0] + pp[1] * (T)(kGP[qx] - 0.5) + pp[2] * (T)(gyq - 0.5);
      T G00 = eta * b00 + kap * ab * a00 - xp;
      T G01 = eta * b01 + kap * ab * a01;
      T G10 = G01;
      T G11 = eta * b11 + kap * ab * a11 - xp;
      if (CONV) {
        G00 -= X0 * U0;
        G01 -= X0 * U1;
        G10 -= X1 * U0;
        G11 -= X1 * U1;
        if (LIN != PNS_PICARD) {
          G00 -= U0 * X0;
          G01 -= U0 * X1;
          G10 -= U1 * X0;
          G11 -= U1 * X1;
        }
      }
      const T W = area * (T)(kGW[qx] * gwy);
      const T sW = sfac * W;
      G00 *= sW * ihx; G10 *= sW * ihx;
      G01 *= sW * ihy; G11 *= sW * ihy;
      const T V0 = W * W0, V1 = W * W1;
      const T P = -sW * (X0x + X1y);
      op[0] += P;
      op[1] += P * (T)(kGP[qx] - 0.5);
      op[2] += P * (T)(gyq - 0.5);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
        S1a[ax] += bv * V0 + bd * G00;
        S2a[ax] += bv * G01;
        S1b[ax] += bv * V1 + bd * G10;
        S2b[ax] += bv * G11;
      }
    }
    if (valid) {
      // this row's share of the nodal results: B[qy][ay] S1[ax] + D[qy][ay] S2[ax]
#pragma unroll
      for (int ay = 0; ay < 3; ++ay) {
        const T bv = qy == 0 ? (T)q2v(ay, kGP[0]) : (qy == 1 ? (T)q2v(ay, kGP[1]) : (T)q2v(ay, kGP[2]));
        const T bd = qy == 0 ? (T)q2d(ay, kGP[0]) : (qy == 1 ? (T)q2d(ay, kGP[1]) : (T)q2d(ay, kGP[2]));
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          atomicAdd(&acc[2 * mu][ly0 + ay][lx0 + ax], (double)(bv * S1a[ax] + bd * S2a[ax]));
          atomicAdd(&acc[2 * mu + 1][ly0 + ay][lx0 + ax], (double)(bv * S1b[ax] + bd * S2b[ax]));
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) atomicAdd(&pacc[mu][lc][j], (double)op[j]);
      // Dirichlet faces (the whole boundary): point qy of each boundary face
      if (cx == 0)
        face_point<T, LIN, CONV>(m, g, sfac, 0, qy, Xs, Us, mu, lx0, ly0, pp[0], pp[1], pp[2],
                                 acc, pacc[mu][lc]);
      if (cx == g.nx - 1)
        face_point<T, LIN, CONV>(m, g, sfac, 1, qy, Xs, Us, mu, lx0, ly0, pp[0], pp[1], pp[2],
                                 acc, pacc[mu][lc]);
      if (cy == 0)
        face_point<T, LIN, CONV>(m, g, sfac, 2, qy, Xs, Us, mu, lx0, ly0, pp[0], pp[1], pp[2],
                                 acc, pacc[mu][lc]);
      if (cy == g.ny - 1)
        face_point<T, LIN, CONV>(m, g, sfac, 3, qy, Xs, Us, mu, lx0, ly0, pp[0], pp[1], pp[2],
                                 acc, pacc[mu][lc]);
    }
  }
  __syncthreads();
  // pressure rows of owned cells
  for (int i = t; i < 2 * kCells * 3; i += kThreads) {
    const int pmu = i / (kCells * 3), r = i % (kCells * 3);
    const int c = r / 3, j = r % 3;
    const int ccx = cx0 - 1 + c % HX, ccy = cy0 - 1 + c / HX;
    if (ccx >= cx0 && ccy >= cy0 && ccx < g.nx && ccy < g.ny) {
      const int64_t idx = (int64_t)pmu * g.ns + g.nv + 3 * ((int64_t)ccy * g.nx + ccx) + j;
      const double v = pacc[pmu][c][j];
      y[idx] = MODE ? (T)((double)b[idx] - v) : (T)v;
    }
  }
  // owned velocity nodes
  const int gx_end = (cx0 + TX >= g.nx) ? 2 * g.nx + 1 : 2 * (cx0 + TX);
  const int gy_end = (cy0 + TY >= g.ny) ? 2 * g.ny + 1 : 2 * (cy0 + TY);
  const int nox = gx_end - 2 * cx0, noy = gy_end - 2 * cy0;
  for (int i = t; i < 4 * nox * noy; i += kThreads) {
    const int s = i / (nox * noy), r = i % (nox * noy);
    const int ox = r % nox, oy = r / nox;
    const int64_t gn = (int64_t)(2 * cy0 + oy) * NX + (2 * cx0 + ox);
    const int64_t idx = (int64_t)(s >> 1) * g.ns + (int64_t)(s & 1) * g.nn + gn;
    const double v = acc[s][oy + 2][ox + 2];
    y[idx] = MODE ? (T)((double)b[idx] - v) : (T)v;
  }
}

template <typename T, int LIN, bool CONV>
hipError_t launch3(const Grid& g, const Model& m, double tau, const T* uk, const T* x, const T* b,
                   T* y, int mode, hipStream_t s) {
  const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY;
  dim3 grid(tx * ty), block(kThreads);
  if (mode == 0)
    hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 0>), grid, block, 0, s, g, m, tau, uk, x, b,
                       y, tx);
  else
    hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 1>), grid, block, 0, s, g, m, tau, uk, x, b,
                       y, tx);
  return hipGetLastError();
}

template <typename T, int LIN>
hipError_t launch2(const Grid& g, const Model& m, double tau, const T* uk, const T* x, const T* b,
                   T* y, int mode, hipStream_t s) {
  return m.convection ? launch3<T, LIN, true>(g, m, tau, uk, x, b, y, mode, s)
                      : launch3<T, LIN, false>(g, m, tau, uk, x, b, y, mode, s);
}

}  // namespace

template <typename T>
hipError_t launch_cell_apply(const Grid& g, const Model& m, double tau, const T* uk, const T* x,
                             const T* b, T* y, int mode, hipStream_t s) {
  switch (m.lin) {
    case PNS_PICARD: return launch2<T, PNS_PICARD>(g, m, tau, uk, x, b, y, mode, s);
    case PNS_EXACT_NEWTON: return launch2<T, PNS_EXACT_NEWTON>(g, m, tau, uk, x, b, y, mode, s);
    default: return launch2<T, PNS_MODIFIED_NEWTON>(g, m, tau, uk, x, b, y, mode, s);
  }
}

template hipError_t launch_cell_apply<double>(const Grid&, const Model&, double, const double*,
                                              const double*, const double*, double*, int,
                                              hipStream_t);
template hipError_t launch_cell_apply<float>(const Grid&, const Model&, double, const float*,
                                             const float*, const float*, float*, int, hipStream_t);

}  // namespace pns
