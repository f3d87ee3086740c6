// Matrix-free slab Jacobian action in 3D (Q2 / P1disc hexahedra x dG(1)),
// Sec. 5.2 eq. slab-underint-jac with the forms of Sec. 3.2 (eqs. pns-form,
// def-a-gam, Defc, def-b-gam) and the tangents of Sec. 4.2-4.4:
//   y_mu = sum_nu K_t[mu][nu] M_x x_nu + tau w_mu J_mu x_mu.
//
// Three launches, no global atomics, fixed summation order: the volume kernel
// writes every cell's 170 results (81 velocity + 4 pressure per Radau node)
// into a per-cell buffer E; the face kernel adds the boundary-face terms of
// each boundary cell into that cell's slot; the gather kernel sums, for every
// node, the slots of the (up to 8) cells that share it, in a fixed order, and
// writes y = J x or y = b - J x.
//
// Volume kernel (gfx950, wave64): persistent waves, one cell per wave at a
// time, kCellsPerWg waves per workgroup working in their own LDS slices.
// * Each wave prefetches the next cell's nodal lines and pressure
//   coefficients into registers while it computes the current cell, so the
//   global-memory latency is hidden behind the arithmetic.
// * Sum factorisation by lines: each forward stage (x, then y, then z) gives
//   every lane one line of 3 values of one field and applies the 3x3 basis
//   value / derivative matrices, whose entries are compile-time constants;
//   12 fields (x and u_k, 3 components, 2 Radau nodes) x 9 lines = 108 lines.
// * One lane per (Gauss point, Radau node) forms the tangent (FP64 scalars),
//   the temporal mass coupling from the partner node's values and the test
//   coefficients; the Radau nodes take the two half-waves and the point values
//   are stored point-index fastest, so these LDS accesses are unit-stride; the
//   4 pressure rows are summed by a butterfly within each half-wave.
// * The transposed stages (z, y, x) run one line per lane (2 x 3 components x
//   9 lines = 54) and end in coalesced stores of the cell's slot of E.
// * Two LDS buffers per wave are used in turn by the stages (about 18 KB in
//   FP64); a wave orders its stages with wavefront-scope fences only (the LDS
//   operations of one wave are performed in order).
// Face kernel: one wave per boundary cell; the cell's nodal values and its
// slot of E are staged in LDS; its boundary sides are taken in turn, each by
// sum factorisation on the face (fields at the 3 x 3 face points, one lane per
// (face point, Radau node) for the integrand, transposed contractions in
// which every lane adds to its own entries of the slot); the slot is written
// back.
#include <type_traits>

#include "devmath.h"
#include "hex3.h"

namespace pns {
namespace {

constexpr int kCellsPerWg = 4;   // waves (cells in flight) per workgroup
constexpr int kF = 12;           // staged fields: x (mu*3 + c), then u_k (6 + mu*3 + c)
constexpr int kLines = kF * 9;   // forward lines per stage
constexpr int kP = kF * 27 * 4;  // buffer P: s1 (648), pt [f][4][27] (1296), r1 (486)
constexpr int kQ = kF * 27 * 3;  // buffer Q: s2 (972), cf (648), r2 (324)
// results per cell in E: velocity of node a, Radau node mu, component c at
// a*6 + mu*3 + c (the 6 values of a node are contiguous), pressure j of mu at
// 162 + mu*4 + j
constexpr int kSlot = 2 * 85;
static_assert(2 * 3 * 4 * 27 <= kQ, "cf must fit in Q");

// 1D Q2 basis at the 3 Gauss points (compile-time constants once unrolled)
__device__ __forceinline__ constexpr double Bq(int q, int a) { return q2v(a, kGP[q]); }
__device__ __forceinline__ constexpr double Dq(int q, int a) { return q2d(a, kGP[q]); }
__device__ __forceinline__ double gp_sel(int q) {
  return q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]);
}
__device__ __forceinline__ double gw_sel(int q) {
  return q == 0 ? kGW[0] : (q == 1 ? kGW[1] : kGW[2]);
}

// tangent scalars eta, kappa of the selected linearisation at A = D(u_k)
template <int LIN>
__device__ __forceinline__ void tangent3(const Model& m, const double A[3][3], double& eta,
                                         double& kappa) {
  double a2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) a2 += A[i][j] * A[i][j];
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

// Orders the LDS accesses of one wave across a stage boundary: the hardware
// performs them in order, the fence keeps the compiler from moving them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Storage of x and u_k: the compute type itself, or BF16 (the upper 16 bits
// of an FP32 value, held as uint16_t) widened to FP32 when it is loaded.
template <typename T, typename S>
__device__ __forceinline__ T ld(const S* p) {
  return (T)*p;
}
template <>
__device__ __forceinline__ float ld<float, uint16_t>(const uint16_t* p) {
  return __uint_as_float((uint32_t)*p << 16);
}

template <typename T, typename S, int LIN, bool CONV>
__global__ __launch_bounds__(64 * kCellsPerWg, 2) void cell_volume3d_kernel(
    Grid3 g, Model m, double tau, const S* __restrict__ uk, const S* __restrict__ x,
    T* __restrict__ E, int64_t nwaves) {
  __shared__ __align__(16) T Pall[kCellsPerWg][kP];
  __shared__ __align__(16) T Qall[kCellsPerWg][kQ];
  __shared__ double presall[kCellsPerWg][2][4];
  const int w = threadIdx.x >> 6;
  const int t = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * kCellsPerWg + w;
  if (wid >= nwaves) return;
  T* const P = Pall[w];
  T* const Q = Qall[w];
  double(*const pres)[4] = presall[w];
  const int64_t NX = 2 * g.nx + 1, NXY = NX * (2 * g.ny + 1);
  // Step k of every wave covers the block of nwaves consecutive cells
  // [k nwaves, (k+1) nwaves), so neighbouring cells run at the same time.
  // -1: no more cells for this wave.
  auto cell_of = [&](int64_t k) -> int64_t {
    const int64_t c = k * nwaves + wid;
    return c < g.nc ? c : -1;
  };
  auto node0 = [&](int64_t c) -> int64_t {
    const int64_t cx = c % g.nx, cy = (c / g.nx) % g.ny, cz = c / ((int64_t)g.nx * g.ny);
    return 2 * cz * NXY + 2 * cy * NX + 2 * cx;
  };
  // the lane's nodal lines l = t, t + 64 (field f, az, ay) and its pressure
  // coefficients (lanes of the point phase) of cell c, into registers
  auto load_lines = [&](int64_t c, T (&pre)[2][3]) {
    const int64_t nd0 = node0(c);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int l = t + 64 * it;
      if (l < kLines) {
        const int f = l / 9, r = l % 9, az = r / 3, ay = r % 3;
        const int fm = f % 6, mu = fm / 3, comp = fm % 3;
        const S* src = (f < 6 ? x + (int64_t)mu * g.ns : uk + (int64_t)mu * g.nv) +
                       (int64_t)comp * g.nn + nd0 + az * NXY + ay * NX;
        pre[it][0] = ld<T>(src);
        pre[it][1] = ld<T>(src + 1);
        pre[it][2] = ld<T>(src + 2);
      }
    }
  };
  auto load_pres = [&](int64_t c, T (&pp)[4]) {
    if ((t & 31) < 27) {  // the lanes of the point phase: Radau node t / 32
      const S* pv = x + (int64_t)(t >> 5) * g.ns + g.nv + 4 * c;
      pp[0] = ld<T>(pv);
      pp[1] = ld<T>(pv + 1);
      pp[2] = ld<T>(pv + 2);
      pp[3] = ld<T>(pv + 3);
    }
  };
  const T ih[3] = {(T)g.ihx, (T)g.ihy, (T)g.ihz};
  const double vol = g.hx * g.hy * g.hz;
  T pre[2][3] = {}, prep[4] = {};
  load_lines(wid, pre);
  load_pres(wid, prep);
  int64_t next = -1;
#pragma unroll 1
  for (int64_t k = 0, cell = wid; cell >= 0; ++k, cell = next) {
    next = cell_of(k + 1);

    // ---- forward x: line (f, az, ay) of nodal values -> s1[f][az][ay][qx][v, d]
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int l = t + 64 * it;
      if (l < kLines) {
        const T* n = pre[it];
        T* dst = P + l * 6;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          dst[2 * q] = (T)Bq(q, 0) * n[0] + (T)Bq(q, 1) * n[1] + (T)Bq(q, 2) * n[2];
          dst[2 * q + 1] = (T)Dq(q, 0) * n[0] + (T)Dq(q, 1) * n[1] + (T)Dq(q, 2) * n[2];
        }
      }
    }
    // the next cell's lines load while this one is computed
    if (next >= 0) load_lines(next, pre);
    wave_sync();
    // ---- forward y: line (f, az, qx) -> s2[f][az][qy][qx][v, dx, dy]
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int l = t + 64 * it;
      if (l < kLines) {
        const int f = l / 9, r = l % 9, az = r / 3, qx = r % 3;
        T v[3], d[3];
#pragma unroll
        for (int ay = 0; ay < 3; ++ay) {
          const T* s = P + ((f * 9 + az * 3 + ay) * 3 + qx) * 2;
          v[ay] = s[0];
          d[ay] = s[1];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          T* dst = Q + (((f * 3 + az) * 3 + q) * 3 + qx) * 3;
          dst[0] = (T)Bq(q, 0) * v[0] + (T)Bq(q, 1) * v[1] + (T)Bq(q, 2) * v[2];
          dst[1] = (T)Bq(q, 0) * d[0] + (T)Bq(q, 1) * d[1] + (T)Bq(q, 2) * d[2];
          dst[2] = (T)Dq(q, 0) * v[0] + (T)Dq(q, 1) * v[1] + (T)Dq(q, 2) * v[2];
        }
      }
    }
    wave_sync();
    // ---- forward z: line (f, qy, qx) -> pt[f][v, dx, dy, dz][q] (reference
    // derivatives; point index fastest so that the point phase reads unit stride)
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int l = t + 64 * it;
      if (l < kLines) {
        const int f = l / 9, r = l % 9;  // r = qy * 3 + qx
        T v[3], dx[3], dy[3];
#pragma unroll
        for (int az = 0; az < 3; ++az) {
          const T* s = Q + ((f * 3 + az) * 9 + r) * 3;
          v[az] = s[0];
          dx[az] = s[1];
          dy[az] = s[2];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          T* dst = P + f * 108 + q * 9 + r;
          dst[0] = (T)Bq(q, 0) * v[0] + (T)Bq(q, 1) * v[1] + (T)Bq(q, 2) * v[2];
          dst[27] = (T)Bq(q, 0) * dx[0] + (T)Bq(q, 1) * dx[1] + (T)Bq(q, 2) * dx[2];
          dst[54] = (T)Bq(q, 0) * dy[0] + (T)Bq(q, 1) * dy[1] + (T)Bq(q, 2) * dy[2];
          dst[81] = (T)Dq(q, 0) * v[0] + (T)Dq(q, 1) * v[1] + (T)Dq(q, 2) * v[2];
        }
      }
    }
    wave_sync();

    // ---- points: Radau node mu = half-wave, point q = lane within the half (27 of
    // 32 busy); test coefficients cf[mu][c][V, Gx, Gy, Gz][q] into Q, pressure
    // rows by a butterfly within each half
    {
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
      const int q = t & 31, mu = t >> 5, other = 1 - mu;
      if (q < 27) {
        const int qz = q / 9, qy = (q / 3) % 3, qx = q % 3;
        const double W = vol * gw_sel(qx) * gw_sel(qy) * gw_sel(qz);
        const double sW = tau * (mu ? kWt[1] : kWt[0]) * W;
        const double kself = mu ? kKt[1][1] : kKt[0][0], koth = mu ? kKt[1][0] : kKt[0][1];
        T X[3], U[3], GX[3][3], GU[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T* px = P + (mu * 3 + c) * 108 + q;
          const T* pu = P + (6 + mu * 3 + c) * 108 + q;
          X[c] = px[0];
          U[c] = pu[0];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            GX[c][j] = px[27 * (1 + j)] * ih[j];
            GU[c][j] = pu[27 * (1 + j)] * ih[j];
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
        const T kab = kap * ab;
        // pressure of x at the point
        const T xp = prep[0] + prep[1] * (T)(gp_sel(qx) - 0.5) +
                     prep[2] * (T)(gp_sel(qy) - 0.5) + prep[3] * (T)(gp_sel(qz) - 0.5);
        T xo[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) xo[i] = P[(other * 3 + i) * 108 + q];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          Q[((mu * 3 + i) * 4 + 0) * 27 + q] = (T)W * ((T)kself * X[i] + (T)koth * xo[i]);
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            // coefficient of d_j w_i: T(B)_ij - convection - xp delta_ij
            T gij = eta * B[i][j] + kab * (T)A[i][j] - (i == j ? xp : (T)0);
            if (CONV) {
              gij -= X[i] * U[j];
              if (LIN != PNS_PICARD) gij -= U[i] * X[j];
            }
            Q[((mu * 3 + i) * 4 + 1 + j) * 27 + q] = (T)sW * gij * ih[j];
          }
        }
        const double cpv = -sW * (double)(GX[0][0] + GX[1][1] + GX[2][2]);
        p4[0] = cpv;
        p4[1] = cpv * (gp_sel(qx) - 0.5);
        p4[2] = cpv * (gp_sel(qy) - 0.5);
        p4[3] = cpv * (gp_sel(qz) - 0.5);
      }
      // sum over the lanes of one Radau node (xor masks below 32 stay in the half)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int msk = 1; msk < 32; msk <<= 1) p4[j] += __shfl_xor(p4[j], msk, 64);
      }
      if (q == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) pres[mu][j] = p4[j];
      }
    }
    if (next >= 0) load_pres(next, prep);
    wave_sync();
    // ---- backward z: line (mu, c, qy, qx) -> r1[mu][c][qy][qx][az][v, gx, gy]
    if (t < 54) {
      const int mc = t / 9, r = t % 9;  // mc = mu * 3 + c, r = qy * 3 + qx
      T V[3], GXv[3], GYv[3], GZv[3];
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) {
        const int q = qz * 9 + r;
        V[qz] = Q[(mc * 4 + 0) * 27 + q];
        GXv[qz] = Q[(mc * 4 + 1) * 27 + q];
        GYv[qz] = Q[(mc * 4 + 2) * 27 + q];
        GZv[qz] = Q[(mc * 4 + 3) * 27 + q];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        T* dst = P + ((mc * 9 + r) * 3 + a) * 3;
        dst[0] = (T)Bq(0, a) * V[0] + (T)Bq(1, a) * V[1] + (T)Bq(2, a) * V[2] +
                 (T)Dq(0, a) * GZv[0] + (T)Dq(1, a) * GZv[1] + (T)Dq(2, a) * GZv[2];
        dst[1] = (T)Bq(0, a) * GXv[0] + (T)Bq(1, a) * GXv[1] + (T)Bq(2, a) * GXv[2];
        dst[2] = (T)Bq(0, a) * GYv[0] + (T)Bq(1, a) * GYv[1] + (T)Bq(2, a) * GYv[2];
      }
    }
    wave_sync();
    // ---- backward y: line (mu, c, qx, az) -> r2[mu][c][qx][az][ay][v, gx]
    if (t < 54) {
      const int mc = t / 9, qx = (t % 9) / 3, az = t % 3;
      T v[3], gx[3], gy[3];
#pragma unroll
      for (int qy = 0; qy < 3; ++qy) {
        const T* s = P + ((mc * 9 + qy * 3 + qx) * 3 + az) * 3;
        v[qy] = s[0];
        gx[qy] = s[1];
        gy[qy] = s[2];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        T* dst = Q + (((mc * 3 + qx) * 3 + az) * 3 + a) * 2;
        dst[0] = (T)Bq(0, a) * v[0] + (T)Bq(1, a) * v[1] + (T)Bq(2, a) * v[2] +
                 (T)Dq(0, a) * gy[0] + (T)Dq(1, a) * gy[1] + (T)Dq(2, a) * gy[2];
        dst[1] = (T)Bq(0, a) * gx[0] + (T)Bq(1, a) * gx[1] + (T)Bq(2, a) * gx[2];
      }
    }
    wave_sync();
    // ---- backward x: line (mu, c, az, ay) -> results at its 3 nodes, into E
    T* slot = E + cell * kSlot;
    if (t < 54) {
      const int mc = t / 9, az = (t % 9) / 3, ay = t % 3;
      const int mu = mc / 3, c = mc % 3;
      T v[3], gx[3];
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        const T* s = Q + (((mc * 3 + qx) * 3 + az) * 3 + ay) * 2;
        v[qx] = s[0];
        gx[qx] = s[1];
      }
      T* dst = slot + (az * 9 + ay * 3) * 6 + mu * 3 + c;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        dst[6 * a] = (T)Bq(0, a) * v[0] + (T)Bq(1, a) * v[1] + (T)Bq(2, a) * v[2] +
                 (T)Dq(0, a) * gx[0] + (T)Dq(1, a) * gx[1] + (T)Dq(2, a) * gx[2];
    } else if (t < 62) {
      const int mu = (t - 54) / 4, j = (t - 54) % 4;
      slot[162 + mu * 4 + j] = (T)pres[mu][j];
    }
    wave_sync();  // the buffers and pres are rewritten by the next cell
  }
}

// Face point qa (two tangential Gauss indices) of boundary side sd (normal
// direction k = sd / 2, end sd % 2) of a cell: reference coordinates (fixed
// along k, Gauss in the two other directions taken cyclically after k),
// outward normal, quadrature weight times tau w_mu times the face measure, and
// 1 / h_F with h_F the cell size normal to the face.
__device__ __forceinline__ void face_point_geometry(const Grid3& g, double tau, int sd, int qa,
                                                    int mu, double xi[3], double n[3],
                                                    double& sW, double& ihF) {
  const int k = sd >> 1, hi = sd & 1, k1 = (k + 1) % 3;
  const double ga = gp_sel(qa % 3), gb = gp_sel(qa / 3), fix = hi ? 1.0 : 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xi[d] = d == k ? fix : (d == k1 ? ga : gb);
    n[d] = d == k ? (hi ? 1.0 : -1.0) : 0.0;
  }
  const double hk = k == 0 ? g.hx : (k == 1 ? g.hy : g.hz);
  ihF = 1.0 / hk;
  sW = tau * (mu ? kWt[1] : kWt[0]) * gw_sel(qa % 3) * gw_sel(qa / 3) * (g.hx * g.hy * g.hz / hk);
}

// Boundary cells: one wave per cell of the six boundary layers.  Workgroup b
// takes face b of the boundary (faces numbered side by side, side s: normal
// direction k = s / 2, low / high end s % 2, within a side lexicographically
// over the tangential cell indices taken cyclically after k) and processes
// that face's cell if s is the cell's first boundary side, with all of the
// cell's boundary sides in turn; otherwise it exits.  Per side, sum
// factorisation on the face: the nodal values are contracted along the normal
// (face-layer value and normal derivative) and along the two tangential
// directions to the 3 x 3 face Gauss points; after the pointwise integrand
// the transposed contractions give the 81 velocity and 4 pressure results of
// each Radau node, one output line per lane, added to the cell's slot of E.
template <typename T, typename S, int LIN, bool CONV>
__global__ __launch_bounds__(64) void face3d_kernel(Grid3 g, Model m, double tau,
                                                    const S* __restrict__ uk,
                                                    const S* __restrict__ x, T* __restrict__ E) {
  __shared__ T nd[kF * 27];            // nd[f * 27 + a], local node a = ax + 3 ay + 9 az
  __shared__ double pf[kF][9][4];      // per field, face point: value, d/dx, d/dy, d/dz
  __shared__ double coef[2][9][13];    // per Radau node, face point: F (3), G (3x3), P
  __shared__ double outv[kSlot];       // the cell's slot of E, FP64
  const int n3[3] = {g.nx, g.ny, g.nz};
  int64_t f = blockIdx.x;
  int side = 0;
  for (; side < 5; ++side) {
    const int kk = side >> 1;
    const int64_t nf = (int64_t)n3[(kk + 1) % 3] * n3[(kk + 2) % 3];
    if (f < nf) break;
    f -= nf;
  }
  int cc[3];
  {
    const int k = side >> 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    cc[k] = (side & 1) ? n3[k] - 1 : 0;
    cc[k1] = (int)(f % n3[k1]);
    cc[k2] = (int)(f / n3[k1]);
  }
  const int sides = (cc[0] == 0 ? 1 : 0) | (cc[0] == g.nx - 1 ? 2 : 0) | (cc[1] == 0 ? 4 : 0) |
                    (cc[1] == g.ny - 1 ? 8 : 0) | (cc[2] == 0 ? 16 : 0) |
                    (cc[2] == g.nz - 1 ? 32 : 0);
  if (__builtin_ctz(sides) != side) return;  // the cell belongs to an earlier side
  const int64_t cell = ((int64_t)cc[2] * g.ny + cc[1]) * g.nx + cc[0];
  const int64_t NX = 2 * g.nx + 1, NXY = NX * (2 * g.ny + 1);
  const int64_t n0 = 2 * (int64_t)cc[2] * NXY + 2 * (int64_t)cc[1] * NX + 2 * (int64_t)cc[0];
  T* slot = E + cell * kSlot;
  const int t = threadIdx.x;
  for (int l = t; l < kLines; l += 64) {
    const int fl = l / 9, r = l % 9, lz = r / 3, ly = r % 3;
    const int fm = fl % 6, mu = fm / 3, comp = fm % 3;
    const S* src = (fl < 6 ? x + (int64_t)mu * g.ns : uk + (int64_t)mu * g.nv) +
                   (int64_t)comp * g.nn + n0 + lz * NXY + ly * NX;
#pragma unroll
    for (int a = 0; a < 3; ++a) nd[fl * 27 + r * 3 + a] = ld<T>(src + a);
  }
  for (int i = t; i < kSlot; i += 64) outv[i] = (double)slot[i];
  const double ihd[3] = {g.ihx, g.ihy, g.ihz};
  __syncthreads();
#pragma unroll 1
  for (int bits = sides; bits; bits &= bits - 1) {
    const int sd = __builtin_ctz(bits);
    const int k = sd >> 1, hi = sd & 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    // strides of the local node index along k, k1, k2; the face layer along k
    const int sk = k == 0 ? 1 : (k == 1 ? 3 : 9);
    const int s1 = k1 == 0 ? 1 : (k1 == 1 ? 3 : 9);
    const int s2 = k2 == 0 ? 1 : (k2 == 1 ? 3 : 9);
    const int lay = hi ? 2 : 0;
    // derivative of the 1D basis along k at the face (reference): q2d(a, 0 or 1)
    const double dn0 = hi ? 1.0 : -3.0, dn1 = hi ? -4.0 : 4.0, dn2 = hi ? 3.0 : -1.0;
    const double ihk = k == 0 ? g.ihx : (k == 1 ? g.ihy : g.ihz);
    const double ih1 = k1 == 0 ? g.ihx : (k1 == 1 ? g.ihy : g.ihz);
    const double ih2 = k2 == 0 ? g.ihx : (k2 == 1 ? g.ihy : g.ihz);
    // ---- (1) fields at the face points: lane (field, point q1 + 3 q2)
#pragma unroll 1
    for (int l = t; l < kF * 9; l += 64) {
      const int fl = l / 9, q = l % 9, q1 = q % 3, q2 = q / 3;
      const T* nf = nd + fl * 27;
      double v = 0.0, d1 = 0.0, d2 = 0.0, dk = 0.0;
#pragma unroll
      for (int b2 = 0; b2 < 3; ++b2) {
        const double B2 = q2 == 0 ? Bq(0, b2) : (q2 == 1 ? Bq(1, b2) : Bq(2, b2));
        const double D2 = q2 == 0 ? Dq(0, b2) : (q2 == 1 ? Dq(1, b2) : Dq(2, b2));
#pragma unroll
        for (int b1 = 0; b1 < 3; ++b1) {
          const double B1 = q1 == 0 ? Bq(0, b1) : (q1 == 1 ? Bq(1, b1) : Bq(2, b1));
          const double D1 = q1 == 0 ? Dq(0, b1) : (q1 == 1 ? Dq(1, b1) : Dq(2, b1));
          const int ab = b1 * s1 + b2 * s2;
          const double val = (double)nf[ab + lay * sk];
          const double dnv = dn0 * (double)nf[ab] + dn1 * (double)nf[ab + sk] +
                             dn2 * (double)nf[ab + 2 * sk];
          v += B1 * B2 * val;
          d1 += D1 * B2 * val;
          d2 += B1 * D2 * val;
          dk += B1 * B2 * dnv;
        }
      }
      d1 *= ih1;
      d2 *= ih2;
      dk *= ihk;
      pf[fl][q][0] = v;
      pf[fl][q][1] = k == 0 ? dk : (k1 == 0 ? d1 : d2);
      pf[fl][q][2] = k == 1 ? dk : (k1 == 1 ? d1 : d2);
      pf[fl][q][3] = k == 2 ? dk : (k1 == 2 ? d1 : d2);
    }
    __syncthreads();
    // ---- (2) integrand: lane (point, Radau node)
    if (t < 18) {
      const int qa = t >> 1, mu = t & 1;
      double xi[3], n[3], sW, ihF;
      face_point_geometry(g, tau, sd, qa, mu, xi, n, sW, ihF);
      double X[3], U[3], A[3][3], B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        X[i] = pf[mu * 3 + i][qa][0];
        U[i] = pf[6 + mu * 3 + i][qa][0];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          A[i][j] = 0.5 * (pf[6 + mu * 3 + i][qa][1 + j] + pf[6 + mu * 3 + j][qa][1 + i]);
          B[i][j] = 0.5 * (pf[mu * 3 + i][qa][1 + j] + pf[mu * 3 + j][qa][1 + i]);
        }
      double eta, kap;
      tangent3<LIN>(m, A, eta, kap);
      double ab = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ab += A[i][j] * B[i][j];
      const S* pv = x + (int64_t)mu * g.ns + g.nv + 4 * cell;
      const double xp = (double)ld<T>(pv) + (double)ld<T>(pv + 1) * (xi[0] - 0.5) +
                        (double)ld<T>(pv + 2) * (xi[1] - 0.5) + (double)ld<T>(pv + 3) * (xi[2] - 0.5);
      const double un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
      const double xn = X[0] * n[0] + X[1] * n[1] + X[2] * n[2];
      // frozen Nitsche coefficients at G = D ghat_D from the boundary table (no
      // data: eta_D, no rank-one part)
      double etaG = m.etaD, kG = 0.0, Gl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      if (m.lift) {
        const double* lt = m.lift + lift3_index(g, sd, cc[k1], cc[k2], qa, mu);
        sym3(lt + 3, Gl);
        etaG = lt[9];
        kG = lt[10];
      }
      double GS = 0.0;  // G : sym(x (x) n)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) GS += Gl[i][j] * X[i] * n[j];
      const double pen1 = m.gamma1 * etaG * ihF, pen2 = m.gamma2 * ihF;
      double* cf = coef[mu][qa];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double Tn = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) Tn += (eta * B[i][j] + kap * ab * A[i][j]) * n[j];
        // -(T(B) n).w + x_pi n.w, penalties, convective flux with the inflow correction
        double F = -Tn + xp * n[i] + pen1 * X[i] + pen2 * xn * n[i];
        if (CONV) {
          const double neg = 0.5 * (fabs(un) - un);
          F += (un - neg) * X[i];
          if (LIN != PNS_PICARD) F += xn * U[i];
        }
        cf[i] = sW * F;
        // symmetry term -(DS(G)(D w) n).x as a coefficient of d_j w_i:
        // -(eta(G) S + k (G:S) G)_ij with S = sym(x (x) n)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          cf[3 + 3 * i + j] = -sW * (etaG * 0.5 * (X[i] * n[j] + X[j] * n[i]) + kG * GS * Gl[i][j]);
      }
      cf[12] = sW * m.qsign * xn;  // coefficient of the pressure test
    }
    __syncthreads();
    // ---- (3) transposed: lane (mu, c, face node b1 + 3 b2) -> its 3 nodes along k;
    // lanes 54..61 the pressure rows
    if (t < 54) {
      const int mu = t / 27, c = (t / 9) % 3, b = t % 9, b1 = b % 3, b2 = b / 3;
      // component of the gradient coefficient along k, k1, k2
      const int gk = 3 + 3 * c + k, g1 = 3 + 3 * c + k1, g2 = 3 + 3 * c + k2;
      double sface = 0.0, snorm = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < 3; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < 3; ++q1) {
          const double* cf = coef[mu][q1 + 3 * q2];
          const double BB = Bq(q1, b1 == 0 ? 0 : (b1 == 1 ? 1 : 2)) *
                            Bq(q2, b2 == 0 ? 0 : (b2 == 1 ? 1 : 2));
          const double DB = Dq(q1, b1 == 0 ? 0 : (b1 == 1 ? 1 : 2)) *
                            Bq(q2, b2 == 0 ? 0 : (b2 == 1 ? 1 : 2));
          const double BD = Bq(q1, b1 == 0 ? 0 : (b1 == 1 ? 1 : 2)) *
                            Dq(q2, b2 == 0 ? 0 : (b2 == 1 ? 1 : 2));
          sface += cf[c] * BB + cf[g1] * ih1 * DB + cf[g2] * ih2 * BD;
          snorm += cf[gk] * ihk * BB;
        }
      const int ab = b1 * s1 + b2 * s2;
      double* o = outv + mu * 3 + c;
      // node index a in the slot: velocity at a*6 + mu*3 + c
      o[(ab + 0 * sk) * 6] += dn0 * snorm + (lay == 0 ? sface : 0.0);
      o[(ab + 1 * sk) * 6] += dn1 * snorm;
      o[(ab + 2 * sk) * 6] += dn2 * snorm + (lay == 2 ? sface : 0.0);
    } else if (t < 62) {
      const int mu = (t - 54) / 4, j = (t - 54) % 4;
      double sp = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < 3; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < 3; ++q1) {
          // psi_j at the point: 1 or (xi_d - 1/2), d = j - 1
          const int d = j - 1;
          const double xd = d == k ? (hi ? 1.0 : 0.0) : (d == k1 ? kGP[q1] : kGP[q2]);
          sp += coef[mu][q1 + 3 * q2][12] * (j == 0 ? 1.0 : xd - 0.5);
        }
      outv[162 + mu * 4 + j] += sp;
    }
    __syncthreads();
  }
  for (int i = t; i < kSlot; i += 64) slot[i] = (T)outv[i];
}

// y = s or y = b - s, s the sum over the cells sharing each unknown of their
// slots of E: thread i < nn takes node i (6 velocity unknowns), thread
// nn + c takes the 8 pressure unknowns of cell c.  Cells are visited in the
// order of increasing index, so the result does not depend on scheduling.
template <typename T>
__global__ void gather3_kernel(Grid3 g, const T* __restrict__ E, const T* __restrict__ b,
                               T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nn + g.nc) return;
  if (i >= g.nn) {
    const int64_t cell = i - g.nn;
#pragma unroll
    for (int mu = 0; mu < 2; ++mu)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t idx = (int64_t)mu * g.ns + g.nv + 4 * cell + j;
        const T v = E[cell * kSlot + 162 + mu * 4 + j];
        y[idx] = b ? b[idx] - v : v;
      }
    return;
  }
  const int64_t NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  const int ii[3] = {(int)(i % NX), (int)((i / NX) % NY), (int)(i / (NX * NY))};
  const int nn3[3] = {g.nx, g.ny, g.nz};
  // per direction, candidates h = 0, 1: the cell below the node (local index
  // 2) and the cell above it (local index 0); an odd node index lies inside
  // one cell (local index 1, candidate 1 only)
  int cs[3][2], as[3][2];
  bool ok[3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int v = ii[d];
    const bool odd = v & 1;
    cs[d][0] = (v >> 1) - 1;
    as[d][0] = 2;
    ok[d][0] = !odd && v > 0;
    cs[d][1] = v >> 1;
    as[d][1] = odd ? 1 : 0;
    ok[d][1] = (v >> 1) < nn3[d];
  }
  // all loads first (fixed trip count), then the sum in a fixed order
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  T2 v[8][3];
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int h0 = h & 1, h1 = (h >> 1) & 1, h2 = h >> 2;
    const bool use = ok[0][h0] && ok[1][h1] && ok[2][h2];
    const int64_t cell =
        use ? ((int64_t)cs[2][h2] * g.ny + cs[1][h1]) * g.nx + cs[0][h0] : 0;
    const int a = as[0][h0] + 3 * as[1][h1] + 9 * as[2][h2];
    // the node's 6 values are contiguous (16-byte aligned in FP64, 8 in FP32)
    const T2* sl = reinterpret_cast<const T2*>(E + cell * kSlot + a * 6);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      v[h][q] = use ? sl[q] : T2{(T)0, (T)0};
    }
  }
  T acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < 8; ++h)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      acc[2 * q] += v[h][q].x;
      acc[2 * q + 1] += v[h][q].y;
    }
#pragma unroll
  for (int mu = 0; mu < 2; ++mu)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (int64_t)mu * g.ns + (int64_t)c * g.nn + i;
      y[idx] = b ? b[idx] - acc[mu * 3 + c] : acc[mu * 3 + c];
    }
}

// waves of the kernel that are resident at once on the device (0 on error)
template <typename K>
int64_t resident_waves(K kernel) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 64 * kCellsPerWg, 0) != hipSuccess)
    return 0;
  return (int64_t)nb * cus * kCellsPerWg;
}

template <typename T, typename S, int LIN, bool CONV>
hipError_t launch3_kernels(const Grid3& g, const Model& m, double tau, const S* uk, const S* x,
                           T* E, hipStream_t s) {
  auto vkern = cell_volume3d_kernel<T, S, LIN, CONV>;
  static const int64_t resident = resident_waves(vkern);
  if (resident <= 0) return hipErrorInvalidDeviceFunction;
  const int64_t nwaves = g.nc < resident ? g.nc : resident;
  hipLaunchKernelGGL(vkern, dim3((unsigned)((nwaves + kCellsPerWg - 1) / kCellsPerWg)),
                     dim3(64 * kCellsPerWg), 0, s, g, m, tau, uk, x, E, nwaves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nfaces = 2 * ((int64_t)g.ny * g.nz + (int64_t)g.nz * g.nx + (int64_t)g.nx * g.ny);
  hipLaunchKernelGGL((face3d_kernel<T, S, LIN, CONV>), dim3((unsigned)nfaces), dim3(64), 0, s, g,
                     m, tau, uk, x, E);
  return hipGetLastError();
}

template <typename T, typename S, int LIN>
hipError_t launch3_lin(const Grid3& g, const Model& m, double tau, const S* uk, const S* x, T* E,
                       hipStream_t s) {
  return m.convection ? launch3_kernels<T, S, LIN, true>(g, m, tau, uk, x, E, s)
                      : launch3_kernels<T, S, LIN, false>(g, m, tau, uk, x, E, s);
}

template <typename T, typename S>
hipError_t apply3d_any(const Grid3& g, const Model& m, double tau, const S* uk, const S* x,
                       const T* b, T* y, T* E, int mode, hipStream_t s) {
  hipError_t e;
  switch (m.lin) {
    case PNS_PICARD: e = launch3_lin<T, S, PNS_PICARD>(g, m, tau, uk, x, E, s); break;
    case PNS_EXACT_NEWTON: e = launch3_lin<T, S, PNS_EXACT_NEWTON>(g, m, tau, uk, x, E, s); break;
    default: e = launch3_lin<T, S, PNS_MODIFIED_NEWTON>(g, m, tau, uk, x, E, s); break;
  }
  if (e != hipSuccess) return e;
  const int64_t nt = g.nn + g.nc;
  hipLaunchKernelGGL(gather3_kernel<T>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, g,
                     (const T*)E, mode ? b : (const T*)nullptr, y);
  return hipGetLastError();
}

// FP64 -> BF16 with round to nearest even, correctly rounded for finite
// values in the FP32 range: the value is first rounded to FP32 by round to
// odd (truncate, then set the last bit when the truncation was inexact), which
// keeps every bit the final rounding to 8 significant bits needs, then rounded
// to nearest even on its upper 16 bits.
__global__ void to_bf16_kernel(int64_t n, const double* __restrict__ in, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = in[i];
  const float f = __double2float_rz(v);
  uint32_t u = __float_as_uint(f);
  if ((double)f != v) u |= 1u;
  u += 0x7fffu + ((u >> 16) & 1u);
  out[i] = (uint16_t)(u >> 16);
}

}  // namespace

template <typename T>
hipError_t launch_cell_apply3d(const Grid3& g, const Model& m, double tau, const T* uk,
                               const T* x, const T* b, T* y, T* E, int mode, hipStream_t s) {
  return apply3d_any<T, T>(g, m, tau, uk, x, b, y, E, mode, s);
}

hipError_t launch_cell_apply3d_bf16(const Grid3& g, const Model& m, double tau, const uint16_t* uk,
                                    const uint16_t* x, const float* b, float* y, float* E,
                                    int mode, hipStream_t s) {
  return apply3d_any<float, uint16_t>(g, m, tau, uk, x, b, y, E, mode, s);
}

hipError_t launch_to_bf16(int64_t n, const double* in, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather3(const Grid3& g, const T* E, const T* b, T* y, hipStream_t s) {
  const int64_t nt = g.nn + g.nc;
  hipLaunchKernelGGL(gather3_kernel<T>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, g, E,
                     b, y);
  return hipGetLastError();
}

template hipError_t launch_gather3<double>(const Grid3&, const double*, const double*, double*,
                                           hipStream_t);
template hipError_t launch_gather3<float>(const Grid3&, const float*, const float*, float*,
                                          hipStream_t);
template hipError_t launch_cell_apply3d<double>(const Grid3&, const Model&, double, const double*,
                                                const double*, const double*, double*, double*,
                                                int, hipStream_t);
template hipError_t launch_cell_apply3d<float>(const Grid3&, const Model&, double, const float*,
                                               const float*, const float*, float*, float*, int,
                                               hipStream_t);

}  // namespace pns
