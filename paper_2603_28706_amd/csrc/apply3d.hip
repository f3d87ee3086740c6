// Matrix-free slab Jacobian action in 3D (Q2 / P1disc hexahedra x dG(1)),
// Sec. 5.2 eq. slab-underint-jac with the forms of Sec. 3.2 (eqs. pns-form,
// def-a-gam, Defc, def-b-gam) and the tangents of Sec. 4.2-4.4:
//   y_mu = sum_nu K_t[mu][nu] M_x x_nu + tau w_mu J_mu x_mu.
//
// Design: one workgroup (one wave) per cell.  The 27 nodal values of x and
// u_k (3 components, both Radau nodes) are staged in LDS and brought to the
// 3 x 3 x 3 Gauss points by sum factorisation (contractions along x, y, z);
// one thread per (Gauss point, Radau node) forms the tangent (FP64 scalars),
// the temporal mass coupling and the test coefficients; the transposed
// contractions (z, y, x) give the 81 velocity results per Radau node and the
// 4 pressure rows are summed directly.  Cells on the boundary add their face
// terms (direct evaluation at the 9 points of each boundary face).  Results are
// added to y with global atomics (y is zero-filled, or holds b for the defect,
// before the kernel), so the summation order over cells is not fixed.
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int kF = 12;  // staged fields: x (mu*3 + c), then u_k (6 + mu*3 + c)
constexpr int kR1 = 2 * 3 * 27 * 3;  // elements of r1 (r2 follows it)
static_assert(2 * 3 * 4 * 27 <= kF * 9 * 3 * 2, "cf must fit in the s1 buffer");
static_assert(kR1 + 2 * 3 * 27 * 2 <= kF * 81, "r1 and r2 must fit in the s2 buffer");

__device__ __forceinline__ double gp(int q) { return q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]); }
__device__ __forceinline__ double gw(int q) { return q == 0 ? kGW[0] : (q == 1 ? kGW[1] : kGW[2]); }
__device__ __forceinline__ double bv(int q, int a) { return q2v(a, gp(q)); }
__device__ __forceinline__ double bd(int q, int a) { return q2d(a, gp(q)); }

// tangent scalars: eta = nu_inf + mu, kappa of the selected linearisation
template <int LIN>
__device__ __forceinline__ void tangent3(const Model& m, const double A[3][3], double& eta,
                                         double& kappa) {
  double a2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) a2 += A[i][j] * A[i][j];
  const double D2 = m.delta2 + a2;
  const double mu = m.nu * pow(D2, m.expo);
  eta = m.nu_inf + mu;
  if (LIN == PNS_PICARD) {
    kappa = 0.0;
  } else {
    const double c = (m.p - 2.0) / D2;
    if (LIN == PNS_MODIFIED_NEWTON) {
      const double lim = a2 > 0.0 ? m.sigma_max / sqrt(a2) : mu;
      kappa = c * fmin(mu, lim);
    } else {
      kappa = c * mu;
    }
  }
}

template <typename T, int LIN, bool CONV>
__global__ __launch_bounds__(64) void cell_apply3d_kernel(Grid3 g, Model m, double tau,
                                                          const T* __restrict__ uk,
                                                          const T* __restrict__ x,
                                                          T* __restrict__ y, T sign) {
  // LDS stages; s1 is dead once s2 is formed and hosts cf, s2 is dead once pt is
  // formed and hosts r1 and r2
  __shared__ T nd[kF][27];                 // nodal values, local node a = ax + 3 ay + 9 az
  __shared__ T bufA[kF * 9 * 3 * 2];       // s1 [f][az*3+ay][qx][B, D along x]; then cf
  __shared__ T bufB[kF * 81];              // s2 [f][az][qy][qx][val, d/dx, d/dy]; then r1, r2
  __shared__ T pt[kF][27][4];              // [f][q][val, d/dx, d/dy, d/dz] (reference derivatives)
  __shared__ T cp[2][27];                  // [mu][q] pressure-test coefficient
  __shared__ double outv[2][85];           // [mu][81 velocity (c*27 + a), 4 pressure]
  auto s1 = reinterpret_cast<T(*)[9][3][2]>(bufA);
  auto cf = reinterpret_cast<T(*)[3][4][27]>(bufA);          // [mu][c][V, Gx, Gy, Gz][q]
  auto s2 = reinterpret_cast<T(*)[3][3][3][3]>(bufB);
  auto r1 = reinterpret_cast<T(*)[3][3][3][3][3]>(bufB);     // [mu][c][qy][qx][az][v, x, y]
  auto r2 = reinterpret_cast<T(*)[3][3][3][3][2]>(bufB + kR1);
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % g.nx), cy = (int)((cell / g.nx) % g.ny),
            cz = (int)(cell / ((int64_t)g.nx * g.ny));
  const int t = threadIdx.x;
  const int NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  auto gnode = [&](int a) -> int64_t {
    const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    return ((int64_t)(2 * cz + az) * NY + (2 * cy + ay)) * NX + (2 * cx + ax);
  };

  // stage the nodal values
  for (int i = t; i < kF * 27; i += 64) {
    const int f = i / 27, a = i % 27;
    const int64_t gn = gnode(a);
    const int fm = f % 6, mu = fm / 3, c = fm % 3;
    nd[f][a] = f < 6 ? x[(int64_t)mu * g.ns + (int64_t)c * g.nn + gn]
                     : uk[(int64_t)mu * g.nv + (int64_t)c * g.nn + gn];
  }
  for (int i = t; i < 2 * 85; i += 64) (&outv[0][0])[i] = 0.0;
  __syncthreads();
  // contraction along x
  for (int i = t; i < kF * 9 * 3; i += 64) {
    const int f = i / 27, r = (i / 3) % 9, qx = i % 3;
    T v = 0, d = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T n = nd[f][r * 3 + ax];
      v += (T)bv(qx, ax) * n;
      d += (T)bd(qx, ax) * n;
    }
    s1[f][r][qx][0] = v;
    s1[f][r][qx][1] = d;
  }
  __syncthreads();
  // contraction along y
  for (int i = t; i < kF * 27; i += 64) {
    const int f = i / 27, az = (i / 9) % 3, qy = (i / 3) % 3, qx = i % 3;
    T v = 0, dx = 0, dy = 0;
#pragma unroll
    for (int ay = 0; ay < 3; ++ay) {
      const T b = (T)bv(qy, ay), d = (T)bd(qy, ay);
      v += b * s1[f][az * 3 + ay][qx][0];
      dx += b * s1[f][az * 3 + ay][qx][1];
      dy += d * s1[f][az * 3 + ay][qx][0];
    }
    s2[f][az][qy][qx][0] = v;
    s2[f][az][qy][qx][1] = dx;
    s2[f][az][qy][qx][2] = dy;
  }
  __syncthreads();
  // contraction along z
  for (int i = t; i < kF * 27; i += 64) {
    const int f = i / 27, q = i % 27;
    const int qz = q / 9, qy = (q / 3) % 3, qx = q % 3;
    T v = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll
    for (int az = 0; az < 3; ++az) {
      const T b = (T)bv(qz, az), d = (T)bd(qz, az);
      v += b * s2[f][az][qy][qx][0];
      dx += b * s2[f][az][qy][qx][1];
      dy += b * s2[f][az][qy][qx][2];
      dz += d * s2[f][az][qy][qx][0];
    }
    pt[f][q][0] = v;
    pt[f][q][1] = dx;
    pt[f][q][2] = dy;
    pt[f][q][3] = dz;
  }
  __syncthreads();

  // pointwise: tangent, temporal mass coupling, test coefficients
  const double ih[3] = {g.ihx, g.ihy, g.ihz};
  const double vol = g.hx * g.hy * g.hz;
  if (t < 54) {
    const int q = t >> 1, mu = t & 1, other = 1 - mu;
    const int qz = q / 9, qy = (q / 3) % 3, qx = q % 3;
    const double W = vol * gw(qx) * gw(qy) * gw(qz);
    const double sW = tau * (mu ? kWt[1] : kWt[0]) * W;
    const double kself = mu ? kKt[1][1] : kKt[0][0], koth = mu ? kKt[1][0] : kKt[0][1];
    T X[3], U[3], GX[3][3], GU[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      X[c] = pt[mu * 3 + c][q][0];
      U[c] = pt[6 + mu * 3 + c][q][0];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GX[c][j] = pt[mu * 3 + c][q][1 + j] * (T)ih[j];
        GU[c][j] = pt[6 + mu * 3 + c][q][1 + j] * (T)ih[j];
      }
    }
    double A[3][3];
    T B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        A[i][j] = 0.5 * ((double)GU[i][j] + (double)GU[j][i]);
        B[i][j] = (T)0.5 * (GX[i][j] + GX[j][i]);
      }
    double eta_d, kap_d;
    tangent3<LIN>(m, A, eta_d, kap_d);
    const T eta = (T)eta_d, kap = (T)kap_d;
    T ab = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ab += (T)A[i][j] * B[i][j];
    // pressure of x at the point
    const T* pv = x + (int64_t)mu * g.ns + g.nv + 4 * cell;
    const T xp = pv[0] + pv[1] * (T)(gp(qx) - 0.5) + pv[2] * (T)(gp(qy) - 0.5) +
                 pv[3] * (T)(gp(qz) - 0.5);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T w = (T)kself * X[i] + (T)koth * pt[other * 3 + i][q][0];
      cf[mu][i][0][q] = (T)W * w;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        // coefficient of d_j w_i: T(B)_ij - convection - xp delta_ij
        T gij = eta * B[i][j] + kap * ab * (T)A[i][j] - (i == j ? xp : (T)0);
        if (CONV) {
          gij -= X[i] * U[j];
          if (LIN != PNS_PICARD) gij -= U[i] * X[j];
        }
        cf[mu][i][1 + j][q] = (T)sW * gij * (T)ih[j];
      }
    }
    cp[mu][q] = -(T)sW * (GX[0][0] + GX[1][1] + GX[2][2]);
  }
  __syncthreads();
  // transposed contraction along z: r1 = sum_qz (Bz V + Dz Gz, Bz Gx, Bz Gy)
  for (int i = t; i < 6 * 27; i += 64) {
    const int mc = i / 27, r = i % 27, mu = mc / 3, c = mc % 3;
    const int qy = r / 9, qx = (r / 3) % 3, az = r % 3;
    T v = 0, gx = 0, gy = 0;
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      const int q = (qz * 3 + qy) * 3 + qx;
      const T b = (T)bv(qz, az), d = (T)bd(qz, az);
      v += b * cf[mu][c][0][q] + d * cf[mu][c][3][q];
      gx += b * cf[mu][c][1][q];
      gy += b * cf[mu][c][2][q];
    }
    r1[mu][c][qy][qx][az][0] = v;
    r1[mu][c][qy][qx][az][1] = gx;
    r1[mu][c][qy][qx][az][2] = gy;
  }
  // pressure rows: sum_q P psi_j
  if (t < 8) {
    const int mu = t / 4, j = t % 4;
    double s = 0.0;
    for (int q = 0; q < 27; ++q) {
      const int qj = j == 1 ? q % 3 : (j == 2 ? (q / 3) % 3 : q / 9);
      const double psi = j == 0 ? 1.0 : gp(qj) - 0.5;
      s += (double)cp[mu][q] * psi;
    }
    outv[mu][81 + j] = s;
  }
  __syncthreads();
  // along y: r2 = sum_qy (By v + Dy gy, By gx)
  for (int i = t; i < 6 * 27; i += 64) {
    const int mc = i / 27, r = i % 27, mu = mc / 3, c = mc % 3;
    const int qx = r / 9, az = (r / 3) % 3, ay = r % 3;
    T v = 0, gx = 0;
#pragma unroll
    for (int qy = 0; qy < 3; ++qy) {
      const T b = (T)bv(qy, ay), d = (T)bd(qy, ay);
      v += b * r1[mu][c][qy][qx][az][0] + d * r1[mu][c][qy][qx][az][2];
      gx += b * r1[mu][c][qy][qx][az][1];
    }
    r2[mu][c][qx][az][ay][0] = v;
    r2[mu][c][qx][az][ay][1] = gx;
  }
  __syncthreads();
  // along x: results at the 27 nodes
  for (int i = t; i < 6 * 27; i += 64) {
    const int mc = i / 27, a = i % 27, mu = mc / 3, c = mc % 3;
    const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    T v = 0;
#pragma unroll
    for (int qx = 0; qx < 3; ++qx)
      v += (T)bv(qx, ax) * r2[mu][c][qx][az][ay][0] + (T)bd(qx, ax) * r2[mu][c][qx][az][ay][1];
    outv[mu][c * 27 + a] = (double)v;
  }
  __syncthreads();

  // Dirichlet faces of boundary cells: one task per (side, face point, mu)
  const bool bx0 = cx == 0, bx1 = cx == g.nx - 1, by0 = cy == 0, by1 = cy == g.ny - 1,
             bz0 = cz == 0, bz1 = cz == g.nz - 1;
  if (bx0 || bx1 || by0 || by1 || bz0 || bz1) {
#pragma unroll 1
    for (int task = t; task < 6 * 9 * 2; task += 64) {
      const int side = task / 18, qa = (task / 2) % 9, mu = task & 1;
      const int k = side / 2, hi = side & 1;  // normal direction and end
      const bool on = k == 0 ? (hi ? bx1 : bx0) : (k == 1 ? (hi ? by1 : by0) : (hi ? bz1 : bz0));
      if (!on) continue;
      // reference coordinates of the point: fixed along k, Gauss in the two others
      // (taken cyclically after k)
      const double ga = gp(qa % 3), gb = gp(qa / 3), fix = hi ? 1.0 : 0.0;
      double xi[3], n[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xi[d] = d == k ? fix : (d == (k + 1) % 3 ? ga : gb);
        n[d] = d == k ? (hi ? 1.0 : -1.0) : 0.0;
      }
      const double hk = k == 0 ? g.hx : (k == 1 ? g.hy : g.hz);
      const double ihF = 1.0 / hk;
      const double sW = tau * (mu ? kWt[1] : kWt[0]) * gw(qa % 3) * gw(qa / 3) * (vol / hk);
      // values and gradients at the point from the 27 nodes
      double X[3] = {0, 0, 0}, U[3] = {0, 0, 0}, GX[3][3] = {}, GU[3][3] = {};
#pragma unroll 1
      for (int a = 0; a < 27; ++a) {
        const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
        const double px = q2v(ax, xi[0]), py = q2v(ay, xi[1]), pz = q2v(az, xi[2]);
        const double ph = px * py * pz;
        const double dph[3] = {q2d(ax, xi[0]) * py * pz * ih[0], px * q2d(ay, xi[1]) * pz * ih[1],
                               px * py * q2d(az, xi[2]) * ih[2]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double xv = (double)nd[mu * 3 + c][a], uv = (double)nd[6 + mu * 3 + c][a];
          X[c] += xv * ph;
          U[c] += uv * ph;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            GX[c][j] += xv * dph[j];
            GU[c][j] += uv * dph[j];
          }
        }
      }
      double A[3][3], B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          A[i][j] = 0.5 * (GU[i][j] + GU[j][i]);
          B[i][j] = 0.5 * (GX[i][j] + GX[j][i]);
        }
      double eta, kap;
      tangent3<LIN>(m, A, eta, kap);
      double ab = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ab += A[i][j] * B[i][j];
      const T* pv = x + (int64_t)mu * g.ns + g.nv + 4 * cell;
      const double xp = (double)pv[0] + (double)pv[1] * (xi[0] - 0.5) +
                        (double)pv[2] * (xi[1] - 0.5) + (double)pv[3] * (xi[2] - 0.5);
      const double un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
      const double xn = X[0] * n[0] + X[1] * n[1] + X[2] * n[2];
      const double pen1 = m.gamma1 * m.etaD * ihF, pen2 = m.gamma2 * ihF;
      double F[3], G[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double Tn = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) Tn += (eta * B[i][j] + kap * ab * A[i][j]) * n[j];
        F[i] = -Tn + xp * n[i] + pen1 * X[i] + pen2 * xn * n[i];
        if (CONV) {
          const double neg = 0.5 * (fabs(un) - un);
          F[i] += (un - neg) * X[i];
          if (LIN != PNS_PICARD) F[i] += xn * U[i];
        }
        F[i] *= sW;
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = -sW * m.etaD * 0.5 * (X[i] * n[j] + X[j] * n[i]);
      }
#pragma unroll 1
      for (int a = 0; a < 27; ++a) {
        const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
        const double px = q2v(ax, xi[0]), py = q2v(ay, xi[1]), pz = q2v(az, xi[2]);
        const double ph = px * py * pz;
        const double dph[3] = {q2d(ax, xi[0]) * py * pz * ih[0], px * q2d(ay, xi[1]) * pz * ih[1],
                               px * py * q2d(az, xi[2]) * ih[2]};
#pragma unroll
        for (int c = 0; c < 3; ++c)
          atomicAdd(&outv[mu][c * 27 + a],
                    F[c] * ph + G[c][0] * dph[0] + G[c][1] * dph[1] + G[c][2] * dph[2]);
      }
      const double P = sW * m.qsign * xn;
      atomicAdd(&outv[mu][81], P);
#pragma unroll
      for (int j = 0; j < 3; ++j) atomicAdd(&outv[mu][82 + j], P * (xi[j] - 0.5));
    }
    __syncthreads();
  }

  // add the cell's results to y
  for (int i = t; i < 2 * 85; i += 64) {
    const int mu = i / 85, l = i % 85;
    int64_t idx;
    if (l < 81)
      idx = (int64_t)mu * g.ns + (int64_t)(l / 27) * g.nn + gnode(l % 27);
    else
      idx = (int64_t)mu * g.ns + g.nv + 4 * cell + (l - 81);
    atomicAdd(y + idx, sign * (T)outv[mu][l]);
  }
}

template <typename T>
__global__ void fill3_kernel(int64_t n, const T* __restrict__ b, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b ? b[i] : (T)0;
}

template <typename T, int LIN>
hipError_t launch3_lin(const Grid3& g, const Model& m, double tau, const T* uk, const T* x,
                       T* y, T sign, hipStream_t s) {
  const dim3 grid((unsigned)g.nc), block(64);
  if (m.convection)
    hipLaunchKernelGGL((cell_apply3d_kernel<T, LIN, true>), grid, block, 0, s, g, m, tau, uk, x, y,
                       sign);
  else
    hipLaunchKernelGGL((cell_apply3d_kernel<T, LIN, false>), grid, block, 0, s, g, m, tau, uk, x,
                       y, sign);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_cell_apply3d(const Grid3& g, const Model& m, double tau, const T* uk,
                               const T* x, const T* b, T* y, int mode, hipStream_t s) {
  // y = 0 (action) or y = b (defect), then the cells add +J x or -J x
  hipLaunchKernelGGL(fill3_kernel<T>, dim3((unsigned)((g.nst + 255) / 256)), dim3(256), 0, s,
                     g.nst, mode ? b : (const T*)nullptr, y);
  const T sign = mode ? (T)-1 : (T)1;
  switch (m.lin) {
    case PNS_PICARD: return launch3_lin<T, PNS_PICARD>(g, m, tau, uk, x, y, sign, s);
    case PNS_EXACT_NEWTON: return launch3_lin<T, PNS_EXACT_NEWTON>(g, m, tau, uk, x, y, sign, s);
    default: return launch3_lin<T, PNS_MODIFIED_NEWTON>(g, m, tau, uk, x, y, sign, s);
  }
}

template hipError_t launch_cell_apply3d<double>(const Grid3&, const Model&, double, const double*,
                                                const double*, const double*, double*, int,
                                                hipStream_t);
template hipError_t launch_cell_apply3d<float>(const Grid3&, const Model&, double, const float*,
                                               const float*, const float*, float*, int,
                                               hipStream_t);

}  // namespace pns
