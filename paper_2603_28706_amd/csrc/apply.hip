// Matrix-free slab Jacobian action on the finest level (Sec. 5.2,
// eq. slab-underint-jac): y_mu = sum_nu K_t[mu][nu] M_x x_nu + tau w_mu J_mu x_mu,
// with J_mu the spatial linearisation at the Radau node mu (viscous volume term
// with the Picard / exact / clipped tangent of Sec. 4.2-4.4, convection in
// divergence form, pressure coupling, state-dependent boundary flux and the
// Nitsche terms of eq. def-b-gam).
//
// Design (gfx950, wave64):
// * one workgroup of 256 threads per tile of 16 x 8 evaluated cells; tiles
//   are dealt to the XCDs in contiguous runs.  Two tilings (chosen per variant
//   by how many workgroups share a CU): 15 x 7 owned cells plus a one-cell
//   halo on the low x / low y side, so every owned node is complete in its
//   tile and written once; or 16 x 8 owned cells without halo, each cell
//   evaluated once (at 256 x 256: 512 tiles, one per slot of two workgroups
//   per CU), nodes of shared tile edges written as per-tile partial sums and
//   completed by a second kernel in a fixed order;
// * the tile's nodal values of x and u_k (both Radau nodes) are staged in LDS
//   with coalesced row loads;
// * one thread per (cell, Radau node mu); a wave holds the two Radau nodes of
//   the 32 cells of one parity class of the tile (cells of one class share no
//   node, so the LDS atomics of a wave never collide); for each row qy of the
//   3x3 Gauss points a thread contracts the nodal values along y (sum
//   factorisation), evaluates values / gradients / tangent at the three points
//   of the row, and forms the row's share of the 9 nodal results by the
//   transposed contractions; the temporal mass coupling K_t[mu][nu] x_nu is
//   formed at the points from the partner lane's values (DPP lane swap);
// * the tangent scalars (Delta^2, mu, eta, clip factor, kappa) are evaluated
//   in FP64 in both precisions; everything else in the storage type T;
// * velocity shares are summed in LDS with LDS atomics (summation order inside
//   a tile is not fixed); the pressure rows of a cell are complete in its
//   thread and stored to LDS;
// * the boundary-face terms run in a phase of their own after a barrier, one
//   thread per face point of the tile (only tiles at the boundary), which keeps
//   their registers out of the volume part: three workgroups share a CU;
// * the owned cells' pressure rows and the tile's complete nodes are written
//   coalesced from LDS (without halo: the partial sums of shared edge nodes to
//   the edge buffer).
#include "devmath.h"
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int HX = 16, HY = 8;            // evaluated cells per tile
constexpr int BX = 2 * HX + 1, BY = 2 * HY + 1;  // LDS node box (33 x 17)
constexpr int kCells = HX * HY;           // 128
constexpr int kThreads = 2 * kCells;      // 256: (cell, mu)
// perimeter of the node box: bottom row (33), top row (33), left and right
// columns without the corners (15 each)
constexpr int kPerim = 2 * BX + 2 * (BY - 2);  // 96

__host__ __device__ inline int perim_index(int lx, int ly) {
  if (ly == 0) return lx;
  if (ly == BY - 1) return BX + lx;
  if (lx == 0) return 2 * BX + ly - 1;
  return 2 * BX + (BY - 2) + ly - 1;  // lx == BX - 1
}
// Waves per SIMD the register allocation must allow: several workgroups share
// a CU, so the staging, compute and write-out phases of different tiles
// overlap.  3 (<= 168 VGPRs) fits without spills except for the FP64 variant
// that recomputes the tangent, which gets 2.
template <typename T, bool CACHED>
constexpr int waves_per_simd() {
  return (sizeof(T) == 8 && !CACHED) ? 2 : 3;
}
// Tiling of a variant.  With three workgroups per CU (768 slots) the tiles of
// 15 x 7 owned cells plus a one-cell halo on the low x / low y side (666 tiles
// at 256 x 256) fit in one round and every node is complete inside its tile.
// With two per CU (512 slots) those tiles would take two rounds, so the tile
// is 16 x 8 owned cells without halo (512 tiles at 256 x 256, 22 % less
// arithmetic) and the nodes of shared tile edges are completed by a second
// kernel from per-tile partial sums.
template <typename T, bool CACHED>
constexpr bool halo_tiles() {
  return waves_per_simd<T, CACHED>() == 3;
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

// 1D basis values / derivatives at the Gauss point qy of a wave-uniform row
template <typename T>
__device__ __forceinline__ T row_sel(int qy, double a, double b, double c) {
  return qy == 0 ? (T)a : (qy == 1 ? (T)b : (T)c);
}
template <typename T>
__device__ __forceinline__ T row_v(int qy, int a) {
  return row_sel<T>(qy, q2v(a, kGP[0]), q2v(a, kGP[1]), q2v(a, kGP[2]));
}
template <typename T>
__device__ __forceinline__ T row_d(int qy, int a) {
  return row_sel<T>(qy, q2d(a, kGP[0]), q2d(a, kGP[1]), q2d(a, kGP[2]));
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

// One point q of a Dirichlet boundary face of a cell (the whole boundary of the
// rectangle is Dirichlet): convective boundary flux, the consistency / symmetry
// terms with the tangent and the pressure, the lagged inflow term and the two
// penalties (eq. def-b-gam).  The test coefficients are contracted against the
// 9 nodes of the cell and added to the tile's LDS sums (velocity: acc, at the
// cell's node box offset lx0 / ly0; pressure: pa, or nothing for pa == nullptr).
// u_k is read from the tile's LDS copy Us when the variant stages one, else
// from memory.
template <typename T, int LIN, bool CONV, bool ATOMIC, bool LDS_U>
__device__ __forceinline__ void face_point(const Model& m, const Grid& g, double tau, int side,
                                           int q, int mu, int cx, int cy, const T (*Xs)[BY][BX],
                                           const T (*Us)[BY][BX], int lx0, int ly0,
                                           const T* __restrict__ uk, const T* __restrict__ x,
                                           double (*acc)[BY][BX], double* pa) {
  // side: 0 x=0 (n=-e_x), 1 x=1 (n=+e_x), 2 y=0 (n=-e_y), 3 y=1 (n=+e_y)
  const bool xface = side < 2;
  const double nxv = xface ? (side == 0 ? -1.0 : 1.0) : 0.0;
  const double nyv = xface ? 0.0 : (side == 2 ? -1.0 : 1.0);
  // per-lane q, mu: selects instead of indexed constant tables
  const double gq = q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]);
  const double wq = q == 0 ? kGW[0] : (q == 1 ? kGW[1] : kGW[2]);
  const double xi = xface ? (side == 0 ? 0.0 : 1.0) : gq;
  const double et = xface ? gq : (side == 2 ? 0.0 : 1.0);
  const double ihF = xface ? g.ihx : g.ihy;  // 1 / h_F, h_F the cell size normal to the face
  // frozen Nitsche coefficients at G = D ghat_D from the boundary table (no
  // data: eta_D, no rank-one part)
  const int64_t cell = (int64_t)cy * g.nx + cx;
  // the pressure coefficients of x first: their load overlaps the rest
  const T* pv = x + (int64_t)mu * g.ns + g.nv + 3 * cell;
  const T xp0 = pv[0], xp1 = pv[1], xp2 = pv[2];
  double Gl00 = 0.0, Gl01 = 0.0, Gl11 = 0.0, etaG = m.etaD, kG = 0.0;
  if (m.lift) {
    const double* lt = m.lift + lift_index(g, side, xface ? cy : cx, q, mu);
    Gl00 = lt[2];
    Gl01 = lt[3];
    Gl11 = lt[4];
    etaG = lt[5];
    kG = lt[6];
  }
  const T pen1 = (T)(m.gamma1 * etaG * ihF);
  const T pen2 = (T)(m.gamma2 * ihF);
  const T n0 = (T)nxv, n1 = (T)nyv;
  const int NX = 2 * g.nx + 1;
  const T* um = uk + (int64_t)mu * g.nv;
  T vx[3], vy[3], dx[3], dy[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vx[a] = (T)q2v(a, xi);
    vy[a] = (T)q2v(a, et);
    dx[a] = (T)(q2d(a, xi) * g.ihx);
    dy[a] = (T)(q2d(a, et) * g.ihy);
  }
  // u_k first and the tangent from it, then x: keeps the loads in flight (and
  // their registers) to one field at a time
  T U[2] = {0, 0}, GU[2][2] = {{0, 0}, {0, 0}}, X[2] = {0, 0}, GX[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      T u0, u1;
      if (LDS_U) {
        u0 = Us[2 * mu][ly0 + ay][lx0 + ax];
        u1 = Us[2 * mu + 1][ly0 + ay][lx0 + ax];
      } else {
        const int64_t gn = (int64_t)(2 * cy + ay) * NX + (2 * cx + ax);
        u0 = um[gn];
        u1 = um[g.nn + gn];
      }
      U[0] += u0 * ph; U[1] += u1 * ph;
      GU[0][0] += u0 * px; GU[0][1] += u0 * py;
      GU[1][0] += u1 * px; GU[1][1] += u1 * py;
    }
  const T a00 = GU[0][0], a01 = (T)0.5 * (GU[0][1] + GU[1][0]), a11 = GU[1][1];
  double eta_d, kap_d;
  tangent_coef<LIN>(m, (double)a00, (double)a01, (double)a11, eta_d, kap_d);
  const T eta = (T)eta_d, kap = (T)kap_d;
  // zero offset that the compiler must take as depending on the tangent
  int lofs = 0;
  asm volatile("" : "+v"(lofs) : "v"(kap_d));
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      const T x0 = Xs[2 * mu][ly0 + ay][lx0 + ax + lofs];
      const T x1 = Xs[2 * mu + 1][ly0 + ay][lx0 + ax + lofs];
      X[0] += x0 * ph; X[1] += x1 * ph;
      GX[0][0] += x0 * px; GX[0][1] += x0 * py;
      GX[1][0] += x1 * px; GX[1][1] += x1 * py;
    }
  const T xp = xp0 + xp1 * (T)(xi - 0.5) + xp2 * (T)(et - 0.5);
  const T b00 = GX[0][0], b01 = (T)0.5 * (GX[0][1] + GX[1][0]), b11 = GX[1][1];
  const T ab = a00 * b00 + (T)2 * a01 * b01 + a11 * b11;
  const T T00 = eta * b00 + kap * ab * a00;
  const T T01 = eta * b01 + kap * ab * a01;
  const T T11 = eta * b11 + kap * ab * a11;
  // tau w_mu times the face quadrature weight
  const T sW = (T)(tau * (mu ? kWt[1] : kWt[0]) * wq * (xface ? g.hy : g.hx));
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
  // -(DS(G)(Dw) n).x = -Dw : DS(G)(sym(x (x) n))  ->  coefficient of d_j w_i:
  // -(eta(G) S + k (G:S) G)_ij with S = sym(x (x) n)
  const T S00 = X[0] * n0, S01 = (T)0.5 * (X[0] * n1 + X[1] * n0), S11 = X[1] * n1;
  const T kGS = (T)kG * ((T)Gl00 * S00 + (T)2 * (T)Gl01 * S01 + (T)Gl11 * S11);
  const T eG = (T)etaG;
  const T G00 = -sW * (eG * S00 + kGS * (T)Gl00), G01 = -sW * (eG * S01 + kGS * (T)Gl01);
  const T G10 = G01, G11 = -sW * (eG * S11 + kGS * (T)Gl11);
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ph = vx[ax] * vy[ay], px = dx[ax] * vy[ay], py = vx[ax] * dy[ay];
      lds_add<ATOMIC>(&acc[2 * mu][ly0 + ay][lx0 + ax], (double)(F0 * ph + G00 * px + G01 * py));
      lds_add<ATOMIC>(&acc[2 * mu + 1][ly0 + ay][lx0 + ax],
                      (double)(F1 * ph + G10 * px + G11 * py));
    }
  if (pa) {
    const T P = sW * (T)m.qsign * xn;
    lds_add<ATOMIC>(&pa[0], (double)P);
    lds_add<ATOMIC>(&pa[1], (double)(P * (T)(xi - 0.5)));
    lds_add<ATOMIC>(&pa[2], (double)(P * (T)(et - 0.5)));
  }
}

// Per-point coefficients of the volume term, cached once per linearisation
// state (index ((cell*2 + mu)*9 + qy*3 + qx)*6):
//   c0 = sW eta,  (c1, c2, c3) = sqrt(-sW kappa) (A00, A01, A11),  (c4, c5) = sW u,
// with sW = tau w_mu W_q, so that sW T(B) = c0 B - (a':B) a' (kappa <= 0 for
// p <= 2) and the convective flux uses sW u directly.  Tangent scalars in FP64.
constexpr int kCacheVals = 6;

template <typename T, int LIN>
__global__ __launch_bounds__(256) void tangent_cache_kernel(Grid g, Model m, double tau,
                                                            const double* __restrict__ uk,
                                                            T* __restrict__ cache) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nc * 18) return;
  const int q = (int)(id % 9);
  const int mu = (int)((id / 9) % 2);
  const int64_t cell = id / 18;
  const int cx = (int)(cell % g.nx), cy = (int)(cell / g.nx);
  const int qx = q % 3, qy = q / 3;
  const double* um = uk + (int64_t)mu * g.nv;
  const int NX = 2 * g.nx + 1;
  double U0 = 0, U1 = 0, g00 = 0, g01 = 0, g10 = 0, g11 = 0;
  for (int a = 0; a < 9; ++a) {
    const int ax = a % 3, ay = a / 3;
    const int64_t gn = (int64_t)(2 * cy + ay) * NX + (2 * cx + ax);
    const double u0 = um[gn], u1 = um[g.nn + gn];
    const double ph = q2v(ax, kGP[qx]) * q2v(ay, kGP[qy]);
    const double px = q2d(ax, kGP[qx]) / g.hx * q2v(ay, kGP[qy]);
    const double py = q2v(ax, kGP[qx]) * q2d(ay, kGP[qy]) / g.hy;
    U0 += u0 * ph; U1 += u1 * ph;
    g00 += u0 * px; g01 += u0 * py; g10 += u1 * px; g11 += u1 * py;
  }
  const double a00 = g00, a01 = 0.5 * (g01 + g10), a11 = g11;
  double eta, kap;
  tangent_coef<LIN>(m, a00, a01, a11, eta, kap);
  const double sW = tau * kWt[mu] * kGW[qx] * kGW[qy] * g.hx * g.hy;
  const double sk = sqrt(fmax(-sW * kap, 0.0));
  T* c = cache + id * kCacheVals;
  c[0] = (T)(sW * eta);
  c[1] = (T)(sk * a00);
  c[2] = (T)(sk * a01);
  c[3] = (T)(sk * a11);
  c[4] = (T)(sW * U0);
  c[5] = (T)(sW * U1);
}

// ORDERED: the cell contributions of a tile sum in a fixed order (parity
// classes one after the other, faces side by side) instead of with LDS atomics
template <typename T, int LIN, bool CONV, int MODE, bool CACHED, bool ORDERED>
__global__ __launch_bounds__(kThreads, (waves_per_simd<T, CACHED>())) void cell_apply_kernel(Grid g, Model m, double tau,
                                                              const T* __restrict__ uk,
                                                              const T* __restrict__ cache,
                                                              const T* __restrict__ x,
                                                              const T* __restrict__ b,
                                                              T* __restrict__ y,
                                                              double* __restrict__ edge,
                                                              int tiles_x) {
  __shared__ T Xs[4][BY][BX];                  // x: [mu*2 + comp]
  __shared__ T Us[CACHED ? 1 : 4][BY][BX];     // u_k: [mu*2 + comp] (recomputing variant)
  __shared__ double acc[4][BY][BX];            // velocity results: [mu*2 + comp]
  __shared__ double pacc[2][kCells][3];        // pressure results: [mu][cell][j]
  // Workgroups are dealt round-robin to the 8 XCDs: give each XCD a contiguous
  // run of tiles, so that neighbouring tiles (shared halo nodes, shared cache
  // lines at the tile edges) meet in the same L2.
  const int nb = gridDim.x, bq = nb >> 3, br = nb & 7;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int tile = xcd * bq + (xcd < br ? xcd : br) + slot;
  constexpr bool HALO = halo_tiles<T, CACHED>();
  constexpr int OFF = HALO ? 1 : 0;  // halo cells on the low side
  const int cx0 = (tile % tiles_x) * (HX - OFF);  // first owned cell
  const int cy0 = (tile / tiles_x) * (HY - OFF);
  const int t = threadIdx.x;
  const int NX = 2 * g.nx + 1;
  const int gx0 = 2 * (cx0 - OFF), gy0 = 2 * (cy0 - OFF);  // node box origin

  // stage x (and u_k) of the node box, zero the sums.  Every load of the
  // thread is issued before the first LDS store (addresses clamped into the
  // mesh, values outside it replaced by zero), so the thread waits for one
  // memory round trip instead of one per box slice.
  {
    constexpr int kSlices = (4 * BY * BX + kThreads - 1) / kThreads;
    T xv[kSlices], uv[kSlices];
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const int i = min(t + s * kThreads, 4 * BY * BX - 1);
      const int f = i / (BY * BX), r = i % (BY * BX);
      const int ly = r / BX, lx = r % BX;
      const int gx = gx0 + lx, gy = gy0 + ly;
      const bool in = gx >= 0 && gy >= 0 && gx <= 2 * g.nx && gy <= 2 * g.ny;
      const int64_t gn = (int64_t)min(max(gy, 0), 2 * g.ny) * NX + min(max(gx, 0), 2 * g.nx);
      const T xl = x[(int64_t)(f >> 1) * g.ns + (int64_t)(f & 1) * g.nn + gn];
      xv[s] = in ? xl : (T)0;
      if (!CACHED) {
        const T ul = uk[(int64_t)(f >> 1) * g.nv + (int64_t)(f & 1) * g.nn + gn];
        uv[s] = in ? ul : (T)0;
      }
    }
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const int i = t + s * kThreads;
      if (i < 4 * BY * BX) {
        const int f = i / (BY * BX), r = i % (BY * BX);
        const int ly = r / BX, lx = r % BX;
        Xs[f][ly][lx] = xv[s];
        if (!CACHED) Us[f][ly][lx] = uv[s];
        acc[f][ly][lx] = 0.0;
      }
    }
  }
  __syncthreads();

  // wave = parity class (cells of one class share no node); lane = (cell, mu)
  const int color = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const int mu = lane & 1, k = lane >> 1;
  const int hx = 2 * (k % (HX / 2)) + (color & 1), hy = 2 * (k / (HX / 2)) + (color >> 1);
  const int cx = cx0 - OFF + hx, cy = cy0 - OFF + hy;
  const bool valid = cx >= 0 && cy >= 0 && cx < g.nx && cy < g.ny;
  const int lx0 = 2 * hx, ly0 = 2 * hy;

  // every lane takes part in the pair exchange below, valid or not
  {
    const T kself = (T)(mu ? kKt[1][1] : kKt[0][0]), koth = (T)(mu ? kKt[1][0] : kKt[0][1]);
    const int64_t cell = (int64_t)(valid ? cy : 0) * g.nx + (valid ? cx : 0);
    const T* xm = x + (int64_t)mu * g.ns + g.nv + 3 * cell;
    const T pp[3] = {xm[0], xm[1], xm[2]};
    const T sfac = (T)(tau * (mu ? kWt[1] : kWt[0]));
    const T ihx = (T)g.ihx, ihy = (T)g.ihy;
    const T area = (T)(g.hx * g.hy);
    T op[3] = {0, 0, 0};  // pressure results of this (cell, mu)

#pragma unroll 1
    for (int qy = 0; qy < 3; ++qy) {
      const T* cq = cache + ((cell * 2 + mu) * 9 + qy * 3) * kCacheVals;
      // contraction along y at row qy: f_y[ax] (values), f_d[ax] (y-derivatives)
      T u0y[3], u0d[3], u1y[3], u1d[3], x0y[3], x0d[3], x1y[3], x1d[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        u0y[ax] = u0d[ax] = u1y[ax] = u1d[ax] = (T)0;
        x0y[ax] = x0d[ax] = x1y[ax] = x1d[ax] = (T)0;
      }
      // the node values are the same for every row; reloading them from LDS per
      // row (an opaque zero offset keeps the loads inside the loop) is cheaper
      // than holding all of them in registers across the rows
      int lofs = 0;
      asm volatile("" : "+v"(lofs));
#pragma unroll
      for (int ay = 0; ay < 3; ++ay) {
        const T bv = row_v<T>(qy, ay), bd = row_d<T>(qy, ay);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int ly = ly0 + ay, lx = lx0 + ax + lofs;
          const T x0 = Xs[2 * mu][ly][lx], x1 = Xs[2 * mu + 1][ly][lx];
          x0y[ax] += bv * x0; x0d[ax] += bd * x0;
          x1y[ax] += bv * x1; x1d[ax] += bd * x1;
          if (!CACHED) {
            const T u0 = Us[2 * mu][ly][lx], u1 = Us[2 * mu + 1][ly][lx];
            u0y[ax] += bv * u0; u0d[ax] += bd * u0;
            u1y[ax] += bv * u1; u1d[ax] += bd * u1;
          }
        }
      }
      const T gyq = row_sel<T>(qy, kGP[0] - 0.5, kGP[1] - 0.5, kGP[2] - 0.5);
      const T gwy = row_sel<T>(qy, kGW[0], kGW[1], kGW[2]);
      // per-point coefficients of the tests phi (S1 value / x-derivative, S2 y-derivative)
      T S1a[3] = {0, 0, 0}, S2a[3] = {0, 0, 0}, S1b[3] = {0, 0, 0}, S2b[3] = {0, 0, 0};
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        T X0 = 0, X1 = 0, X0x = 0, X0y = 0, X1x = 0, X1y = 0;
        T U0 = 0, U1 = 0, U0x = 0, U0y = 0, U1x = 0, U1y = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
          X0 += bv * x0y[ax]; X0x += bd * x0y[ax]; X0y += bv * x0d[ax];
          X1 += bv * x1y[ax]; X1x += bd * x1y[ax]; X1y += bv * x1d[ax];
          if (!CACHED) {
            U0 += bv * u0y[ax]; U0x += bd * u0y[ax]; U0y += bv * u0d[ax];
            U1 += bv * u1y[ax]; U1x += bd * u1y[ax]; U1y += bv * u1d[ax];
          }
        }
        // temporal mass coupling at the point: w = K_t[mu][mu] x_mu + K_t[mu][other] x_other
        const T W0 = kself * X0 + koth * swap_pair(X0);
        const T W1 = kself * X1 + koth * swap_pair(X1);
        X0x *= ihx; X1x *= ihx;
        X0y *= ihy; X1y *= ihy;
        const T b00 = X0x, b01 = (T)0.5 * (X0y + X1x), b11 = X1y;
        const T W = area * (T)kGW[qx] * gwy;
        const T sW = sfac * W;
        const T xp = pp[0] + pp[1] * (T)(kGP[qx] - 0.5) + pp[2] * gyq;
        T G00, G01, G10, G11;  // sW * (T(B) - convective flux - xp I)
        if (CACHED) {
          const T c0 = cq[qx * kCacheVals + 0], c1 = cq[qx * kCacheVals + 1];
          const T c2 = cq[qx * kCacheVals + 2], c3 = cq[qx * kCacheVals + 3];
          const T c4 = cq[qx * kCacheVals + 4], c5 = cq[qx * kCacheVals + 5];
          const T ab = c1 * b00 + (T)2 * c2 * b01 + c3 * b11;
          const T sxp = sW * xp;
          G00 = c0 * b00 - ab * c1 - sxp;
          G01 = c0 * b01 - ab * c2;
          G10 = G01;
          G11 = c0 * b11 - ab * c3 - sxp;
          if (CONV) {
            G00 -= X0 * c4;
            G01 -= X0 * c5;
            G10 -= X1 * c4;
            G11 -= X1 * c5;
            if (LIN != PNS_PICARD) {
              G00 -= c4 * X0;
              G01 -= c4 * X1;
              G10 -= c5 * X0;
              G11 -= c5 * X1;
            }
          }
        } else {
          U0x *= ihx; U1x *= ihx;
          U0y *= ihy; U1y *= ihy;
          const T a00 = U0x, a01 = (T)0.5 * (U0y + U1x), a11 = U1y;
          double eta_d, kap_d;
          tangent_coef<LIN>(m, (double)a00, (double)a01, (double)a11, eta_d, kap_d);
          const T eta = (T)eta_d, kap = (T)kap_d;
          const T ab = a00 * b00 + (T)2 * a01 * b01 + a11 * b11;
          G00 = eta * b00 + kap * ab * a00 - xp;
          G01 = eta * b01 + kap * ab * a01;
          G10 = G01;
          G11 = eta * b11 + kap * ab * a11 - xp;
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
          G00 *= sW; G01 *= sW; G10 *= sW; G11 *= sW;
        }
        G00 *= ihx; G10 *= ihx;
        G01 *= ihy; G11 *= ihy;
        const T V0 = W * W0, V1 = W * W1;
        const T P = -sW * (X0x + X1y);
        op[0] += P;
        op[1] += P * (T)(kGP[qx] - 0.5);
        op[2] += P * gyq;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const T bv = (T)q2v(ax, kGP[qx]), bd = (T)q2d(ax, kGP[qx]);
          S1a[ax] += bv * V0 + bd * G00;
          S2a[ax] += bv * G01;
          S1b[ax] += bv * V1 + bd * G10;
          S2b[ax] += bv * G11;
        }
      }
      // this row's share of the nodal results: B[qy][ay] S1[ax] + D[qy][ay] S2[ax];
      // in the ordered mode the four parity classes add one after the other
      // (cells of one class share no node), so every node sums in a fixed order
      if (ORDERED) {
        for (int c = 0; c < 4; ++c) {
          if (valid && color == c) {
#pragma unroll
            for (int ay = 0; ay < 3; ++ay) {
              const T bv = row_v<T>(qy, ay), bd = row_d<T>(qy, ay);
#pragma unroll
              for (int ax = 0; ax < 3; ++ax) {
                acc[2 * mu][ly0 + ay][lx0 + ax] += (double)(bv * S1a[ax] + bd * S2a[ax]);
                acc[2 * mu + 1][ly0 + ay][lx0 + ax] += (double)(bv * S1b[ax] + bd * S2b[ax]);
              }
            }
          }
          __syncthreads();
        }
      } else if (valid) {
#pragma unroll
        for (int ay = 0; ay < 3; ++ay) {
          const T bv = row_v<T>(qy, ay), bd = row_d<T>(qy, ay);
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            atomicAdd(&acc[2 * mu][ly0 + ay][lx0 + ax], (double)(bv * S1a[ax] + bd * S2a[ax]));
            atomicAdd(&acc[2 * mu + 1][ly0 + ay][lx0 + ax], (double)(bv * S1b[ax] + bd * S2b[ax]));
          }
        }
      }
    }
    if (valid) {
      // every volume contribution to the pressure rows of the cell is in this thread
      const int lc = hy * HX + hx;
#pragma unroll
      for (int j = 0; j < 3; ++j) pacc[mu][lc][j] = (double)op[j];
    }
  }
  __syncthreads();

  // Boundary faces of the evaluated cells, in a phase of their own (one
  // thread per face point), so that their registers do not add to the volume
  // part's.  Only tiles at the boundary of the rectangle have any.
  const int hxe = min(HX - OFF, g.nx - cx0), hye = min(HY - OFF, g.ny - cy0);  // owned cells
  if (cx0 == 0 || cy0 == 0 || cx0 + hxe == g.nx || cy0 + hye == g.ny) {
    // the face cell of point p (side, cell j along it): tile coordinates, or
    // false if it is not evaluated here
    auto face_cell = [&](int side, int j, int& fhx, int& fhy, int& fcx, int& fcy) {
      if (side < 2) {
        fhx = (side == 0 ? 0 : g.nx - 1) - cx0 + OFF;
        fhy = j;
      } else {
        fhx = j;
        fhy = (side == 2 ? 0 : g.ny - 1) - cy0 + OFF;
      }
      fcx = cx0 - OFF + fhx;
      fcy = cy0 - OFF + fhy;
      return !(fhx < 0 || fhx >= HX || fhy < 0 || fhy >= HY || fcx < 0 || fcy < 0 ||
               fcx >= g.nx || fcy >= g.ny);
    };
    if (!ORDERED) {
      // the points of the sides this tile touches, numbered consecutively
      // (HY x 3 x 2 on an x side, HX x 3 x 2 on a y side), one per thread
      // unless the tile touches more than two sides
      const bool touch[4] = {cx0 == 0, cx0 + hxe == g.nx, cy0 == 0, cy0 + hye == g.ny};
      int first[5];
      first[0] = 0;
#pragma unroll
      for (int sd = 0; sd < 4; ++sd) first[sd + 1] = first[sd] + (touch[sd] ? (sd < 2 ? HY : HX) * 6 : 0);
      for (int p = t; p < first[4]; p += kThreads) {
        const int side = p < first[1] ? 0 : (p < first[2] ? 1 : (p < first[3] ? 2 : 3));
        const int r = p - first[side];
        const int j = r / 6, q = (r >> 1) % 3, fmu = r & 1;
        int fhx, fhy, fcx, fcy;
        if (!face_cell(side, j, fhx, fhy, fcx, fcy)) continue;
        // a halo cell contributes to the tile's nodes but not to its pressure rows
        const bool own = fhx >= OFF && fhy >= OFF;
        face_point<T, LIN, CONV, true, !CACHED>(m, g, tau, side, q, fmu, fcx, fcy, Xs, Us,
                                                2 * fhx, 2 * fhy, uk, x, acc,
                                                own ? pacc[fmu][fhy * HX + fhx] : nullptr);
      }
    } else {
      // fixed order: side by side, cells of one parity along the side at a
      // time (neighbours share nodes), the three points of a cell in turn
      for (int side = 0; side < 4; ++side)
        for (int par = 0; par < 2; ++par) {
          const int j = 2 * (t >> 1) + par, fmu = t & 1;
          int fhx, fhy, fcx, fcy;
          if (t < HX * 2 && j < HX && face_cell(side, j, fhx, fhy, fcx, fcy)) {
            const bool own = fhx >= OFF && fhy >= OFF;
            for (int q = 0; q < 3; ++q)
              face_point<T, LIN, CONV, false, !CACHED>(m, g, tau, side, q, fmu, fcx, fcy, Xs,
                                                       Us, 2 * fhx, 2 * fhy, uk, x, acc,
                                                       own ? pacc[fmu][fhy * HX + fhx] : nullptr);
          }
          __syncthreads();
        }
    }
    __syncthreads();
  }

  // Write-out.  In the defect the thread's loads of b for every slice are
  // issued before the first store (invalid slices read b[0]), so it waits for
  // one memory round trip instead of one per slice.
  // pressure rows of the owned cells
  {
    constexpr int kP = (2 * kCells * 3 + kThreads - 1) / kThreads;
    int64_t pidx[kP];
    T pb[kP];
#pragma unroll
    for (int s = 0; s < kP; ++s) {
      const int i = t + s * kThreads;
      const int pmu = i / (kCells * 3), r = i % (kCells * 3);
      const int c = r / 3, j = r % 3;
      const int ccx = cx0 - OFF + c % HX, ccy = cy0 - OFF + c / HX;
      const bool own = i < 2 * kCells * 3 && ccx >= cx0 && ccy >= cy0 && ccx < g.nx && ccy < g.ny;
      pidx[s] = own ? (int64_t)pmu * g.ns + g.nv + 3 * ((int64_t)ccy * g.nx + ccx) + j : -1;
      if (MODE) pb[s] = b[own ? pidx[s] : 0];
    }
#pragma unroll
    for (int s = 0; s < kP; ++s) {
      if (pidx[s] >= 0) {
        const int r = (t + s * kThreads) % (kCells * 3);
        const double v = pacc[(t + s * kThreads) / (kCells * 3)][r / 3][r % 3];
        y[pidx[s]] = MODE ? (T)((double)pb[s] - v) : (T)v;
      }
    }
  }
  if constexpr (HALO) {
    // owned velocity nodes, complete: rows of at most 31 nodes in a 32-wide
    // frame starting at the first owned cell's low corner
    const int gx_end = (cx0 + hxe >= g.nx) ? 2 * g.nx + 1 : 2 * (cx0 + hxe);
    const int gy_end = (cy0 + hye >= g.ny) ? 2 * g.ny + 1 : 2 * (cy0 + hye);
    const int nox = gx_end - 2 * cx0, noy = gy_end - 2 * cy0;
    constexpr int kN = 4 * (2 * HY - 1) * 32, kV = (kN + kThreads - 1) / kThreads;
    int64_t vidx[kV];
    T vb[kV];
#pragma unroll
    for (int sl = 0; sl < kV; ++sl) {
      const int i = t + sl * kThreads;
      const int s = i / ((2 * HY - 1) * 32), r = i % ((2 * HY - 1) * 32);
      const int ox = r % 32, oy = r / 32;
      const bool own = i < kN && ox < nox && oy < noy;
      const int64_t gn = (int64_t)(2 * cy0 + oy) * NX + (2 * cx0 + ox);
      vidx[sl] = own ? (int64_t)(s >> 1) * g.ns + (int64_t)(s & 1) * g.nn + gn : -1;
      if (MODE) vb[sl] = b[own ? vidx[sl] : 0];
    }
#pragma unroll
    for (int sl = 0; sl < kV; ++sl) {
      if (vidx[sl] >= 0) {
        const int i = t + sl * kThreads;
        const int s = i / ((2 * HY - 1) * 32), r = i % ((2 * HY - 1) * 32);
        const double v = acc[s][r / 32 + 2][r % 32 + 2];
        y[vidx[sl]] = MODE ? (T)((double)vb[sl] - v) : (T)v;
      }
    }
  } else {
    // velocity nodes: unshared ones complete, to y; those on an edge shared
    // with another tile as partial sums, to the tile's slice of the edge buffer
    double* te = edge + (int64_t)tile * 4 * kPerim;
    const bool shl = cx0 > 0, shr = cx0 + hxe < g.nx, shb = cy0 > 0, sht = cy0 + hye < g.ny;
    constexpr int kN = 4 * BY * BX, kV = (kN + kThreads - 1) / kThreads;
    int64_t vidx[kV];  // y index, -1: shared edge node or outside the owned box
    T vb[kV];
#pragma unroll
    for (int sl = 0; sl < kV; ++sl) {
      const int i = t + sl * kThreads;
      const int s = i / (BY * BX), r = i % (BY * BX);
      const int ly = r / BX, lx = r % BX;
      const bool in = i < kN && lx <= 2 * hxe && ly <= 2 * hye;
      const bool shared = (lx == 0 && shl) || (lx == 2 * hxe && shr) || (ly == 0 && shb) ||
                          (ly == 2 * hye && sht);
      const int64_t gn = (int64_t)(gy0 + ly) * NX + (gx0 + lx);
      vidx[sl] = in && !shared ? (int64_t)(s >> 1) * g.ns + (int64_t)(s & 1) * g.nn + gn : -1;
      if (MODE) vb[sl] = b[vidx[sl] >= 0 ? vidx[sl] : 0];
    }
#pragma unroll
    for (int sl = 0; sl < kV; ++sl) {
      const int i = t + sl * kThreads;
      const int s = i / (BY * BX), r = i % (BY * BX);
      const int ly = r / BX, lx = r % BX;
      if (i >= kN || lx > 2 * hxe || ly > 2 * hye) continue;
      const double v = acc[s][ly][lx];
      if (vidx[sl] < 0) {
        te[s * kPerim + perim_index(lx, ly)] = v;
      } else {
        y[vidx[sl]] = MODE ? (T)((double)vb[sl] - v) : (T)v;
      }
    }
  }
}

// Tiles without halo: nodes on tile edges shared by 2 or 4 tiles get
// y = the sum of the tiles' partial sums (tiles in increasing order), or
// b - sum.  One thread per node of a shared tile boundary and velocity field:
// the vertical boundaries first, then the horizontal ones, whose nodes on a
// vertical boundary were done there.  Index arithmetic in 32 bits (the node
// count of the shared boundaries is far below 2^31); the up to four partial
// sums and b are loaded before the first of them is used, so their latencies
// overlap.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void edge_sum_kernel(Grid g, const double* __restrict__ edge,
                                                       const T* __restrict__ b,
                                                       T* __restrict__ y, int tiles_x,
                                                       int tiles_y) {
  const unsigned id = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  const unsigned nvl = tiles_x - 1, nhl = tiles_y - 1;  // shared boundaries
  const unsigned nvert = nvl * NY;
  const unsigned nhor = nhl * NX;
  const int s = (int)(id & 3);
  const unsigned nid = id >> 2;
  if (nid >= nvert + nhor) return;
  int gx, gy;
  const bool onv_line = nid < nvert;
  if (onv_line) {
    gx = 2 * HX * (int)(nid / NY + 1);
    gy = (int)(nid % NY);
  } else {
    const unsigned h = nid - nvert;
    gy = 2 * HY * (int)(h / NX + 1);
    gx = (int)(h % NX);
  }
  const bool onv = gx % (2 * HX) == 0 && gx > 0 && gx / (2 * HX) <= (int)nvl;
  if (!onv_line && onv) return;  // done by the vertical pass
  const bool onh = gy % (2 * HY) == 0 && gy > 0 && gy / (2 * HY) <= (int)nhl;
  // tiles (and local node coordinates) left / right of the node, below / above
  int tx0, lx0, tx1 = 0, lx1 = 0;
  if (onv) {
    tx0 = gx / (2 * HX) - 1; lx0 = 2 * HX;
    tx1 = gx / (2 * HX);     lx1 = 0;
  } else {
    tx0 = min(gx / (2 * HX), tiles_x - 1); lx0 = gx - 2 * HX * tx0;
  }
  int ty0, ly0, ty1 = 0, ly1 = 0;
  if (onh) {
    ty0 = gy / (2 * HY) - 1; ly0 = 2 * HY;
    ty1 = gy / (2 * HY);     ly1 = 0;
  } else {
    ty0 = min(gy / (2 * HY), tiles_y - 1); ly0 = gy - 2 * HY * ty0;
  }
  const double* es = edge + (size_t)s * kPerim;
  auto part = [&](int ty, int tx, int lx, int ly) {
    return es[((size_t)ty * tiles_x + tx) * (4 * kPerim) + perim_index(lx, ly)];
  };
  const size_t idx = (size_t)(s >> 1) * g.ns + (size_t)(s & 1) * g.nn + (size_t)gy * NX + gx;
  const double e00 = part(ty0, tx0, lx0, ly0);
  const double e01 = onv ? part(ty0, tx1, lx1, ly0) : 0.0;
  const double e10 = onh ? part(ty1, tx0, lx0, ly1) : 0.0;
  const double e11 = (onv && onh) ? part(ty1, tx1, lx1, ly1) : 0.0;
  const double bv = MODE ? (double)b[idx] : 0.0;
  // tile order (0,0), (0,1), (1,0), (1,1); an absent tile adds +0, which
  // leaves every partial sum unchanged
  const double v = ((e00 + e01) + e10) + e11;
  y[idx] = MODE ? (T)(bv - v) : (T)v;
}

template <typename T, int LIN, bool CONV, bool CACHED>
hipError_t launch4(const Grid& g, const Model& m, double tau, const T* uk, const T* cache,
                   const T* x, const T* b, T* y, double* edge, int mode, hipStream_t s) {
  constexpr int OFF = halo_tiles<T, CACHED>() ? 1 : 0;
  const int tx = (g.nx + HX - OFF - 1) / (HX - OFF), ty = (g.ny + HY - OFF - 1) / (HY - OFF);
  dim3 grid(tx * ty), block(kThreads);
  if (m.ordered) {
    if (mode == 0)
      hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 0, CACHED, true>), grid, block, 0, s, g,
                         m, tau, uk, cache, x, b, y, edge, tx);
    else
      hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 1, CACHED, true>), grid, block, 0, s, g,
                         m, tau, uk, cache, x, b, y, edge, tx);
  } else {
    if (mode == 0)
      hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 0, CACHED, false>), grid, block, 0, s,
                         g, m, tau, uk, cache, x, b, y, edge, tx);
    else
      hipLaunchKernelGGL((cell_apply_kernel<T, LIN, CONV, 1, CACHED, false>), grid, block, 0, s,
                         g, m, tau, uk, cache, x, b, y, edge, tx);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || OFF) return e;
  const int nvl = tx - 1, nhl = ty - 1;
  const int64_t nshared = (int64_t)nvl * (2 * g.ny + 1) + (int64_t)nhl * (2 * g.nx + 1);
  if (nshared == 0) return hipSuccess;
  const dim3 eg((unsigned)((4 * nshared + 255) / 256));
  if (mode == 0)
    hipLaunchKernelGGL((edge_sum_kernel<T, 0>), eg, dim3(256), 0, s, g, (const double*)edge, b, y,
                       tx, ty);
  else
    hipLaunchKernelGGL((edge_sum_kernel<T, 1>), eg, dim3(256), 0, s, g, (const double*)edge, b, y,
                       tx, ty);
  return hipGetLastError();
}

template <typename T, int LIN>
hipError_t launch2(const Grid& g, const Model& m, double tau, const T* uk, const T* cache,
                   const T* x, const T* b, T* y, double* edge, int mode, hipStream_t s) {
  if (cache)
    return m.convection
               ? launch4<T, LIN, true, true>(g, m, tau, uk, cache, x, b, y, edge, mode, s)
               : launch4<T, LIN, false, true>(g, m, tau, uk, cache, x, b, y, edge, mode, s);
  return m.convection
             ? launch4<T, LIN, true, false>(g, m, tau, uk, cache, x, b, y, edge, mode, s)
             : launch4<T, LIN, false, false>(g, m, tau, uk, cache, x, b, y, edge, mode, s);
}

}  // namespace

template <typename T>
hipError_t launch_cell_apply(const Grid& g, const Model& m, double tau, const T* uk, const T* cache,
                             const T* x, const T* b, T* y, double* edge, int mode,
                             hipStream_t s) {
  switch (m.lin) {
    case PNS_PICARD: return launch2<T, PNS_PICARD>(g, m, tau, uk, cache, x, b, y, edge, mode, s);
    case PNS_EXACT_NEWTON:
      return launch2<T, PNS_EXACT_NEWTON>(g, m, tau, uk, cache, x, b, y, edge, mode, s);
    default:
      return launch2<T, PNS_MODIFIED_NEWTON>(g, m, tau, uk, cache, x, b, y, edge, mode, s);
  }
}

int64_t cell_apply_edge_doubles(const Grid& g) {
  const int64_t tx = (g.nx + HX - 1) / HX, ty = (g.ny + HY - 1) / HY;
  return tx * ty * 4 * kPerim;
}

template <typename T>
hipError_t launch_tangent_cache(const Grid& g, const Model& m, double tau, const double* uk,
                                T* cache, hipStream_t s) {
  const int64_t n = g.nc * 18;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (m.lin) {
    case PNS_PICARD:
      hipLaunchKernelGGL((tangent_cache_kernel<T, PNS_PICARD>), grid, block, 0, s, g, m, tau, uk,
                         cache);
      break;
    case PNS_EXACT_NEWTON:
      hipLaunchKernelGGL((tangent_cache_kernel<T, PNS_EXACT_NEWTON>), grid, block, 0, s, g, m, tau,
                         uk, cache);
      break;
    default:
      hipLaunchKernelGGL((tangent_cache_kernel<T, PNS_MODIFIED_NEWTON>), grid, block, 0, s, g, m,
                         tau, uk, cache);
  }
  return hipGetLastError();
}

template hipError_t launch_cell_apply<double>(const Grid&, const Model&, double, const double*,
                                              const double*, const double*, const double*, double*,
                                              double*, int, hipStream_t);
template hipError_t launch_cell_apply<float>(const Grid&, const Model&, double, const float*,
                                             const float*, const float*, const float*, float*,
                                             double*, int, hipStream_t);
template hipError_t launch_tangent_cache<double>(const Grid&, const Model&, double, const double*,
                                                 double*, hipStream_t);
template hipError_t launch_tangent_cache<float>(const Grid&, const Model&, double, const double*,
                                                float*, hipStream_t);

}  // namespace pns
