// Matrix-free slab Jacobian action on the finest level (Sec. 5.2,
// eq. slab-underint-jac): y_mu = sum_nu K_t[mu][nu] M_x x_nu + tau w_mu J_mu x_mu,
// with J_mu the spatial linearisation at the Radau node mu (viscous volume term
// with the Picard / exact / clipped tangent of Sec. 4.2-4.4, convection in
// divergence form, pressure coupling, state-dependent boundary flux and the
// Nitsche terms of eq. def-b-gam).
//
// Design (gfx950, wave64):
// * one workgroup per tile of 15 x 15 owned cells; it also evaluates the
//   one-cell halo on the low x / low y side, so every node it owns receives all
//   of its cell contributions inside the workgroup: each output is written
//   exactly once (no atomics, no zero fill, deterministic);
// * two threads per cell, one per Radau node mu; the temporal mass coupling
//   is applied to the nodal values first (w = K_t[mu][0] x_0 + K_t[mu][1] x_1),
//   so each thread interpolates x_mu (values, gradients), w (values) and
//   u_k,mu (values, gradients) and tests against its own node only;
// * sum factorisation over the 3x3 Gauss points, row by row, all in registers;
//   the 1D basis tables are compile-time constants;
// * the tangent scalars (Delta^2, mu, eta, clip factor, kappa) are evaluated
//   in FP64 in both precisions; everything else in the storage type T;
// * per-node contributions are summed in LDS in four colour phases (cells of
//   one parity class share no node), then written coalesced.
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int TX = 15;                 // owned cells per tile and direction
constexpr int HX = TX + 1;             // evaluated cells (with low-side halo)
constexpr int BX = 2 * TX + 3;         // LDS node box per direction
constexpr int kThreads = 2 * HX * HX;  // 512

template <int LIN>
__device__ __forceinline__ void tangent_coef(const Model& m, double a00, double a01, double a11,
                                             double& eta, double& kappa) {
  const double a2 = a00 * a00 + 2.0 * a01 * a01 + a11 * a11;
  const double D2 = m.delta2 + a2;
  const double mu = m.nu * pow(D2, m.expo);
  eta = m.nu_inf + mu;
  if (LIN == PNS_PICARD) {
    kappa = 0.0;
  } else {
    double k = (m.p - 2.0) * mu / D2;
    if (LIN == PNS_MODIFIED_NEWTON) {
      const double sig = mu * sqrt(a2);
      const double s = sig > 0.0 ? fmin(1.0, m.sigma_max / sig) : 0.0;
      k *= s;
    }
    kappa = k;
  }
}

// Boundary face contribution of one cell (Dirichlet faces): value/gradient test
// coefficients at the 3 face points, contracted directly against the 9 nodes.
template <typename T, int LIN, bool CONV>
__device__ void face_terms(const Model& m, const Grid& g, T sfac, int side, const T* u0, const T* u1,
                           const T* x0, const T* x1, const T* pp, T* o0, T* o1, T* op) {
  // side: 0 x=0 (n=-e_x), 1 x=1 (n=+e_x), 2 y=0 (n=-e_y), 3 y=1 (n=+e_y)
  const bool xface = side < 2;
  const double nxv = xface ? (side == 0 ? -1.0 : 1.0) : 0.0;
  const double nyv = xface ? 0.0 : (side == 2 ? -1.0 : 1.0);
  const double hF = xface ? g.hx : g.hy;
  const double flen = xface ? g.hy : g.hx;
  const T etaD = (T)m.etaD;
  const T pen1 = (T)(m.gamma1 * m.etaD / hF);
  const T pen2 = (T)(m.gamma2 / hF);
  const T n0 = (T)nxv, n1 = (T)nyv;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double xi = xface ? (side == 0 ? 0.0 : 1.0) : kGP[q];
    const double et = xface ? kGP[q] : (side == 2 ? 0.0 : 1.0);
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
        const int a = ax + 3 * ay;
        const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
        U[0] += u0[a] * ph; U[1] += u1[a] * ph;
        GU[0][0] += u0[a] * px; GU[0][1] += u0[a] * py;
        GU[1][0] += u1[a] * px; GU[1][1] += u1[a] * py;
        X[0] += x0[a] * ph; X[1] += x1[a] * ph;
        GX[0][0] += x0[a] * px; GX[0][1] += x0[a] * py;
        GX[1][0] += x1[a] * px; GX[1][1] += x1[a] * py;
      }
    const T xp = pp[0] + pp[1] * (T)(xi - 0.5) + pp[2] * (T)(et - 0.5);
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
        const int a = ax + 3 * ay;
        const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
        o0[a] += F0 * ph + G00 * px + G01 * py;
        o1[a] += F1 * ph + G10 * px + G11 * py;
      }
    const T P = sW * (T)m.qsign * xn;
    op[0] += P;
    op[1] += P * (T)(xi - 0.5);
    op[2] += P * (T)(et - 0.5);
  }
}

template <typename T, int LIN, bool CONV, int MODE>
__global__ __launch_bounds__(kThreads) void cell_apply_kernel(Grid g, Model m, double tau,
                                                              const T* __restrict__ uk,
                                                              const T* __restrict__ x,
                                                              const T* __restrict__ b,
                                                              T* __restrict__ y, int tiles_x) {
  __shared__ T acc[4][BX][BX];  // [mu*2 + comp][local node y][local node x]
  const int tile = blockIdx.x;
  const int cx0 = (tile % tiles_x) * TX;
  const int cy0 = (tile / tiles_x) * TX;
  const int t = threadIdx.x;
  const int mu = t & 1;
  const int lc = t >> 1;
  const int cx = cx0 - 1 + lc % HX;
  const int cy = cy0 - 1 + lc / HX;
  const bool valid = cx >= 0 && cy >= 0 && cx < g.nx && cy < g.ny;
  const int NX = 2 * g.nx + 1;

  for (int i = t; i < 4 * BX * BX; i += kThreads) (&acc[0][0][0])[i] = (T)0;

  T o0[9], o1[9], op[3];
#pragma unroll
  for (int a = 0; a < 9; ++a) o0[a] = o1[a] = (T)0;
  op[0] = op[1] = op[2] = (T)0;

  const int64_t cell = (int64_t)cy * g.nx + cx;
  if (valid) {
    T u0[9], u1[9], x0[9], x1[9], w0[9], w1[9], pp[3];
    const int other = 1 - mu;
    const T kself = (T)kKt[mu][mu], koth = (T)kKt[mu][other];
    const T* um = uk + (int64_t)mu * g.nv;
    const T* xm = x + (int64_t)mu * g.ns;
    const T* xo = x + (int64_t)other * g.ns;
#pragma unroll
    for (int ay = 0; ay < 3; ++ay)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int a = ax + 3 * ay;
        const int64_t gn = (int64_t)(2 * cy + ay) * NX + (2 * cx + ax);
        u0[a] = um[gn];
        u1[a] = um[g.nn + gn];
        x0[a] = xm[gn];
        x1[a] = xm[g.nn + gn];
        w0[a] = kself * x0[a] + koth * xo[gn];
        w1[a] = kself * x1[a] + koth * xo[g.nn + gn];
      }
#pragma unroll
    for (int j = 0; j < 3; ++j) pp[j] = xm[g.nv + 3 * cell + j];

    const T sfac = (T)(tau * kWt[mu]);
    const T ihx = (T)(1.0 / g.hx), ihy = (T)(1.0 / g.hy);
    const T area = (T)(g.hx * g.hy);
    // transposed accumulators: T1[c][qx][ay], T2[c][qx][ay]
    T T1a[3][3], T2a[3][3], T1b[3][3], T2b[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) T1a[i][j] = T2a[i][j] = T1b[i][j] = T2b[i][j] = (T)0;

#pragma unroll
    for (int qy = 0; qy < 3; ++qy) {
      // contract along y at qy: f_y[ax], f_dy[ax]
      T u0y[3], u0d[3], u1y[3], u1d[3], x0y[3], x0d[3], x1y[3], x1d[3], w0y[3], w1y[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        u0y[ax] = u0d[ax] = u1y[ax] = u1d[ax] = (T)0;
        x0y[ax] = x0d[ax] = x1y[ax] = x1d[ax] = w0y[ax] = w1y[ax] = (T)0;
#pragma unroll
        for (int ay = 0; ay < 3; ++ay) {
          const T bv = (T)q2v(ay, kGP[qy]), bd = (T)q2d(ay, kGP[qy]);
          const int a = ax + 3 * ay;
          u0y[ax] += bv * u0[a]; u0d[ax] += bd * u0[a];
          u1y[ax] += bv * u1[a]; u1d[ax] += bd * u1[a];
          x0y[ax] += bv * x0[a]; x0d[ax] += bd * x0[a];
          x1y[ax] += bv * x1[a]; x1d[ax] += bd * x1[a];
          w0y[ax] += bv * w0[a]; w1y[ax] += bv * w1[a];
        }
      }
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        T U0 = 0, U1 = 0, U0x = 0, U0y = 0, U1x = 0, U1y = 0;
        T X0 = 0, X1 = 0, X0x = 0, X0y = 0, X1x = 0, X1y = 0, W0 = 0, W1 = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
          U0 += bv * u0y[ax]; U0x += bd * u0y[ax]; U0y += bv * u0d[ax];
          U1 += bv * u1y[ax]; U1x += bd * u1y[ax]; U1y += bv * u1d[ax];
          X0 += bv * x0y[ax]; X0x += bd * x0y[ax]; X0y += bv * x0d[ax];
          X1 += bv * x1y[ax]; X1x += bd * x1y[ax]; X1y += bv * x1d[ax];
          W0 += bv * w0y[ax]; W1 += bv * w1y[ax];
        }
        U0x *= ihx; U1x *= ihx; X0x *= ihx; X1x *= ihx;
        U0y *= ihy; U1y *= ihy; X0y *= ihy; X1y *= ihy;
        const T a00 = U0x, a01 = (T)0.5 * (U0y + U1x), a11 = U1y;
        const T b00 = X0x, b01 = (T)0.5 * (X0y + X1x), b11 = X1y;
        double eta_d, kap_d;
        tangent_coef<LIN>(m, (double)a00, (double)a01, (double)a11, eta_d, kap_d);
        const T eta = (T)eta_d, kap = (T)kap_d;
        const T ab = a00 * b00 + (T)2 * a01 * b01 + a11 * b11;
        const T xp = pp[0] + pp[1] * (T)(kGP[qx] - 0.5) + pp[2] * (T)(kGP[qy] - 0.5);
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
        const T W = area * (T)(kGW[qx] * kGW[qy]);
        const T sW = sfac * W;
        G00 *= sW * ihx; G10 *= sW * ihx;
        G01 *= sW * ihy; G11 *= sW * ihy;
        const T V0 = W * W0, V1 = W * W1;
        const T P = -sW * (X0x + X1y);
        op[0] += P;
        op[1] += P * (T)(kGP[qx] - 0.5);
        op[2] += P * (T)(kGP[qy] - 0.5);
#pragma unroll
        for (int ay = 0; ay < 3; ++ay) {
          const T bv = (T)q2v(ay, kGP[qy]), bd = (T)q2d(ay, kGP[qy]);
          T1a[qx][ay] += bv * V0 + bd * G01;
          T2a[qx][ay] += bv * G00;
          T1b[qx][ay] += bv * V1 + bd * G11;
          T2b[qx][ay] += bv * G10;
        }
      }
    }
#pragma unroll
    for (int ay = 0; ay < 3; ++ay)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
          const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
          s0 += bv * T1a[qx][ay] + bd * T2a[qx][ay];
          s1 += bv * T1b[qx][ay] + bd * T2b[qx][ay];
        }
        o0[ax + 3 * ay] = s0;
        o1[ax + 3 * ay] = s1;
      }
    // Dirichlet faces (the whole boundary)
    if (cx == 0) face_terms<T, LIN, CONV>(m, g, sfac, 0, u0, u1, x0, x1, pp, o0, o1, op);
    if (cx == g.nx - 1) face_terms<T, LIN, CONV>(m, g, sfac, 1, u0, u1, x0, x1, pp, o0, o1, op);
    if (cy == 0) face_terms<T, LIN, CONV>(m, g, sfac, 2, u0, u1, x0, x1, pp, o0, o1, op);
    if (cy == g.ny - 1) face_terms<T, LIN, CONV>(m, g, sfac, 3, u0, u1, x0, x1, pp, o0, o1, op);
  }
  __syncthreads();
  const int color = (cx & 1) | ((cy & 1) << 1);
  const int lx0 = 2 * (cx - (cx0 - 1)), ly0 = 2 * (cy - (cy0 - 1));
#pragma unroll 1
  for (int ph = 0; ph < 4; ++ph) {
    if (valid && color == ph) {
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          acc[mu * 2 + 0][ly0 + ay][lx0 + ax] += o0[ax + 3 * ay];
          acc[mu * 2 + 1][ly0 + ay][lx0 + ax] += o1[ax + 3 * ay];
        }
    }
    __syncthreads();
  }
  // pressure rows of owned cells
  if (valid && cx >= cx0 && cy >= cy0) {
    T* ym = y + (int64_t)mu * g.ns + g.nv + 3 * cell;
    const T* bm = b + (int64_t)mu * g.ns + g.nv + 3 * cell;
#pragma unroll
    for (int j = 0; j < 3; ++j) ym[j] = MODE ? bm[j] - op[j] : op[j];
  }
  // owned velocity nodes
  const int gx_end = (cx0 + TX >= g.nx) ? 2 * g.nx + 1 : 2 * (cx0 + TX);
  const int gy_end = (cy0 + TX >= g.ny) ? 2 * g.ny + 1 : 2 * (cy0 + TX);
  const int nox = gx_end - 2 * cx0, noy = gy_end - 2 * cy0;
  for (int i = t; i < nox * noy; i += kThreads) {
    const int ox = i % nox, oy = i / nox;
    const int64_t gn = (int64_t)(2 * cy0 + oy) * NX + (2 * cx0 + ox);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t idx = (int64_t)(s >> 1) * g.ns + (int64_t)(s & 1) * g.nn + gn;
      const T v = acc[s][oy + 2][ox + 2];
      y[idx] = MODE ? b[idx] - v : v;
    }
  }
}

template <typename T, int LIN, bool CONV>
hipError_t launch3(const Grid& g, const Model& m, double tau, const T* uk, const T* x, const T* b,
                   T* y, int mode, hipStream_t s) {
  const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TX - 1) / TX;
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
