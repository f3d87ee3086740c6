// Coarse levels of the space-time multigrid on hexahedra (Sec. 6.3), the
// 3D counterparts of the quadrilateral setup and V-cycle kernels:
// * galerkin3d_kernel: coarse space-time element matrices
//   E_C = sum_children P_f^T E_f P_f (A_{l+1} = P^T A_l P restricted cell by
//   cell); the local prolongation is block diagonal (one 27 x 27 Q2
//   interpolation per Radau node and velocity component, one 4 x 4 P1disc
//   restriction per Radau node), so one workgroup forms one block of E_C
//   (row group x column group) over the 8 children;
// * patch3m_kernel: exact patches R_K A_l R_K^T (sums of the element matrices
//   of the cells around the patch: stored Galerkin matrices on coarse levels,
//   or on the finest level K_t (x) M + tau M_t (x) diag(J_1, J_2) formed from
//   the spatial matrices of both Radau nodes), inverted by blocked
//   Gauss-Jordan with partial pivoting in FP64 on the matrix cores; the
//   170 x 170 matrix (231 KB) is larger than the LDS of a CU but fits in the
//   registers of a 512-thread workgroup as 16 x 16 accumulator tiles; the
//   inverse is written in the context precision;
// * ebe3_kernel: the level operator element by element, y_K = E_K x_K into the
//   per-cell slots, summed per unknown by the gather of the 3D action;
// * patch_sweep3r_kernel: additive Vanka step with the real coarse inverses,
//   one colour (cell parity) per launch;
// * restrict3_kernel / prolong_add3_kernel: P^T and P of the nested Q2 / P1disc
//   interpolation, one thread per output unknown;
// * coarse_assemble3_kernel: dense coarsest operator, one colour per launch
//   (cells of one colour share no unknown), so the sums are race-free and in a
//   fixed order.
#include <type_traits>

#include "hex3.h"

namespace pns {
namespace {

// ----------------------------------------------------------- Galerkin

// level-0 space-time element entry: K_t[mu][nu] M (same velocity component) +
// delta_mu,nu tau w_mu Es_mu (spatial matrices at the state of Radau node mu)
struct FineSrc3 {
  Grid3 g;
  double tau;
  const double* Es_a;
  const double* Es_b;
  __device__ double operator()(int64_t cell, int r, int c) const {
    const int mu = r / kNs3, i = r % kNs3, nu = c / kNs3, j = c % kNs3;
    double v = 0.0;
    if (i < kNv3 && j < kNv3 && i / kNb3 == j / kNb3) {
      const double kt = mu == 0 ? (nu == 0 ? kKt[0][0] : kKt[0][1])
                                : (nu == 0 ? kKt[1][0] : kKt[1][1]);
      v = kt * cell_mass3(g, i % kNb3, j % kNb3);
    }
    if (mu == nu) v += tau * kWt[mu] * (mu == 0 ? Es_a : Es_b)[cell * kEs3 + i * kNs3 + j];
    return v;
  }
};

struct StoredSrc3 {
  const double* E;
  __device__ double operator()(int64_t cell, int r, int c) const {
    return E[cell * kE3 + r * kNst3 + c];
  }
};

// local prolongation of child o = (ox, oy, oz): fine unknown a of a group from
// coarse unknown A of the same group (velocity: Q2 interpolation at the fine
// node's position (2 o + a_k) / 4 in the coarse cell; pressure: the coarse
// linear function restricted to the child)
__device__ __forceinline__ double rentry3(int vel, int a, int A, const int o[3]) {
  if (vel) {
    const int ak[3] = {a % 3, (a / 3) % 3, a / 9}, Ak[3] = {A % 3, (A / 3) % 3, A / 9};
    double w = 1.0;
    for (int k = 0; k < 3; ++k) w *= q2v(Ak[k], 0.25 * (2 * o[k] + ak[k]));
    return w;
  }
  if (a == 0) return A == 0 ? 1.0 : 0.5 * (o[A - 1] - 0.5);
  return a == A ? 0.5 : 0.0;
}

template <typename Src>
__global__ __launch_bounds__(256) void galerkin3d_kernel(Grid3 gc, Grid3 gf, Src src,
                                                         double* __restrict__ Ec) {
  __shared__ double Eb[kNb3][kNb3 + 1], Rr[kNb3][kNb3 + 1], Rc[kNb3][kNb3 + 1],
      Tm[kNb3][kNb3 + 1];
  const int64_t C = blockIdx.x;
  const int cx = (int)(C % gc.nx), cy = (int)((C / gc.nx) % gc.ny),
            cz = (int)(C / ((int64_t)gc.nx * gc.ny));
  // groups: mu * 4 + k, k < 3 velocity component k (27 unknowns), k = 3 pressure (4)
  const int grow = blockIdx.y >> 3, gcol = blockIdx.y & 7;
  const int kr = grow & 3, kc = gcol & 3;
  const int nr = kr < 3 ? kNb3 : 4, ncl = kc < 3 ? kNb3 : 4;
  const int offr = (grow >> 2) * kNs3 + (kr < 3 ? kr * kNb3 : kNv3);
  const int offc = (gcol >> 2) * kNs3 + (kc < 3 ? kc * kNb3 : kNv3);
  const int t = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int ch = 0; ch < 8; ++ch) {
    const int o[3] = {ch & 1, (ch >> 1) & 1, ch >> 2};
    const int64_t f = cell_index3(gf, 2 * cx + o[0], 2 * cy + o[1], 2 * cz + o[2]);
    for (int e = t; e < nr * ncl; e += 256) Eb[e / ncl][e % ncl] = src(f, offr + e / ncl, offc + e % ncl);
    for (int e = t; e < nr * nr; e += 256) Rr[e / nr][e % nr] = rentry3(kr < 3, e / nr, e % nr, o);
    for (int e = t; e < ncl * ncl; e += 256)
      Rc[e / ncl][e % ncl] = rentry3(kc < 3, e / ncl, e % ncl, o);
    __syncthreads();
    for (int e = t; e < nr * ncl; e += 256) {  // Tm = Eb Rc
      const int a = e / ncl, B = e % ncl;
      double s = 0.0;
      for (int b = 0; b < ncl; ++b) s += Eb[a][b] * Rc[b][B];
      Tm[a][B] = s;
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {  // acc += Rr^T Tm
      const int e = t + 256 * q;
      if (e < nr * ncl) {
        const int A = e / ncl, B = e % ncl;
        double s = 0.0;
        for (int a = 0; a < nr; ++a) s += Rr[a][A] * Tm[a][B];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < 3; ++q) {
    const int e = t + 256 * q;
    if (e < nr * ncl) Ec[C * kE3 + (offr + e / ncl) * kNst3 + offc + e % ncl] = acc[q];
  }
}

template <typename T>
__global__ void transpose_convert3_kernel(int64_t ncells, const double* __restrict__ E,
                                          T* __restrict__ Et) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncells * kE3) return;
  const int64_t c = i / kE3;
  const int e = (int)(i % kE3);
  const int col = e / kNst3, row = e % kNst3;  // output index = col * 170 + row
  Et[i] = (T)E[c * kE3 + row * kNst3 + col];
}

// ------------------------------------------------------------- patches

constexpr int kPT = 512;

// Entry (i, j) of the exact patch R_K A R_K^T of cell (cx, cy, cz): the sum of
// the element matrices of the cells that hold both unknowns (the cell's own
// pressure lives in that cell only).
template <typename Src>
__device__ double patch3_entry(const Grid3& g, const Src& Esrc, int cx, int cy, int cz, int i,
                               int j) {
  const int64_t K = cell_index3(g, cx, cy, cz);
  const int mr = i / kNs3, sr = i % kNs3, mc = j / kNs3, sc = j % kNs3;
  if (sr >= kNv3 || sc >= kNv3) return Esrc(K, i, j);
  const int ea = sr % kNb3, eb = sc % kNb3;
  const int ax = ea % 3, ay = (ea / 3) % 3, az = ea / 9;
  const int bx = eb % 3, by = (eb / 3) % 3, bz = eb / 9;
  // neighbours that share both nodes: a step -1 (+1) along a direction when
  // both nodes lie on the low (high) face of the cell in that direction
  const int lox = (ax == 0 && bx == 0 && cx > 0) ? -1 : 0;
  const int hix = (ax == 2 && bx == 2 && cx < g.nx - 1) ? 1 : 0;
  const int loy = (ay == 0 && by == 0 && cy > 0) ? -1 : 0;
  const int hiy = (ay == 2 && by == 2 && cy < g.ny - 1) ? 1 : 0;
  const int loz = (az == 0 && bz == 0 && cz > 0) ? -1 : 0;
  const int hiz = (az == 2 && bz == 2 && cz < g.nz - 1) ? 1 : 0;
  const int rbase = mr * kNs3 + (sr / kNb3) * kNb3, cbase = mc * kNs3 + (sc / kNb3) * kNb3;
  double v = 0.0;
  for (int oz = loz; oz <= hiz; ++oz)
    for (int oy = loy; oy <= hiy; ++oy)
      for (int ox = lox; ox <= hix; ++ox) {
        const int na = (ax - 2 * ox) + 3 * (ay - 2 * oy) + 9 * (az - 2 * oz);
        const int nb = (bx - 2 * ox) + 3 * (by - 2 * oy) + 9 * (bz - 2 * oz);
        v += Esrc(cell_index3(g, cx + ox, cy + oy, cz + oz), rbase + na, cbase + nb);
      }
  return v;
}

// Blocked Gauss-Jordan inversion of the 170 x 170 patches on the FP64 matrix
// cores.  The patch, padded to 176 x 176 with an identity block (whose inverse
// is the identity again), is held in the registers of a 512-thread workgroup
// as 121 tiles of 16 x 16 in the accumulator layout of v_mfma_f64_16x16x4f64
// (lane l holds rows l/16 + 4r, r = 0..3, of column l%16 of a tile); wave w
// holds tiles t = 8 s + w.  Per block column K of 16 columns:
// * the panel (all rows, the 16 columns of K) goes through LDS into the
//   registers of the workgroup, one panel row per lane (22 per wave), and the
//   workgroup performs its 16 exchange steps (pivot = largest |entry| among
//   the rows not yet pivoted, reduced within each wave and then across the
//   waves; the pivot row is scaled and broadcast through LDS, the column
//   eliminated from every other row, the pivot column replaced by its
//   elementary-transform column; two barriers per step), so the panel ends
//   as the columns E[:, r_m] of the product E of the 16 transforms, r_m the
//   pivot rows;
// * every other column is multiplied by E: W[:, J] += (E[:, R] - I[:, R])
//   W[R, J], a rank-16 update whose left factor is the panel with 1
//   subtracted at (r_m, m) and whose right factor the 16 pivot rows gathered
//   before the update: 4 MFMA per 16 x 16 tile.
// Rows are never interchanged (the pivot rows are recorded): the final array
// holds the inverse with permuted rows and columns, A^{-1}[i][j] =
// W[r_i][c] with r_c = j, which the write-out undoes.  Same arithmetic as
// Gauss-Jordan with partial pivoting, in another summation order.
constexpr int kMB = 16;                       // block = MFMA tile
constexpr int kMN = 176;                      // padded order
constexpr int kMT = kMN / kMB;                // 11 tile rows / columns
constexpr int kMWaves = 8;                    // 2 waves per SIMD: room for 16 tiles each
constexpr int kMThreads = 64 * kMWaves;
constexpr int kMSlots = (kMT * kMT + kMWaves - 1) / kMWaves;  // 16 tiles per wave
constexpr int kPS = kMB + 1;                  // panel row stride (odd: spreads the banks)
constexpr int kMR = (kMN + kMWaves - 1) / kMWaves;  // panel rows per wave (22)
constexpr int kOS = kMN + 1;                  // output staging row stride
constexpr int kAB = 4;                        // block columns assembled per round
constexpr int kAS = kAB * kMB + 1;            // assembly staging row stride
constexpr int kPool = (kMN * kAS > kMN * kPS + kMB * kOS) ? kMN * kAS : kMN * kPS + kMB * kOS;
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename T, typename Src>
__global__ __launch_bounds__(kMThreads) void patch3m_kernel(Grid3 g, Src Esrc, T* __restrict__ inv,
                                                       int* status, int px, int py, int pz,
                                                       int ncx, int ncy) {
  // one LDS pool: the assembly staging first, then the panel and the pivot
  // rows (right factor; output staging at the end)
  __shared__ double pool[kPool];
  double* const P = pool;
  double* const Bm = pool + kMN * kPS;
  double* const S = pool;
  __shared__ int rowpiv[kMN];          // pivot row of each column
  __shared__ int rinv[kMN];            // column of each pivot row (-1: not yet pivoted)
  __shared__ double prow[kMB];         // scaled pivot row of the current exchange step
  __shared__ double cand_v[2][kMWaves];  // per-wave pivot candidates (two steps in turn)
  __shared__ int cand_i[2][kMWaves];
  __shared__ int s_sing;
  const int64_t pid = blockIdx.x;
  const int cx = px + 2 * (int)(pid % ncx);
  const int cy = py + 2 * (int)((pid / ncx) % ncy);
  const int cz = pz + 2 * (int)(pid / ((int64_t)ncx * ncy));
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int lr = l >> 4, lc = l & 15;  // row quarter and column of the lane in a tile
  if (t < kMN) rinv[t] = -1;
  if (t == 0) s_sing = 0;
  // assembly, kAB block columns at a time through LDS (rolled loops: the
  // tile registers are only ever indexed by compile-time slot numbers)
  mfma_d4 C[kMSlots];
  for (int J0 = 0; J0 < kMT; J0 += kAB) {
    const int ncol = kMB * min(kAB, kMT - J0);
#pragma unroll 2
    for (int e = t; e < kMN * ncol; e += kMThreads) {
      const int row = e / ncol, cl = e % ncol, col = kMB * J0 + cl;
      double v;
      if (row < kNst3 && col < kNst3)
        v = patch3_entry(g, Esrc, cx, cy, cz, row, col);
      else
        v = row == col ? 1.0 : 0.0;
      S[row * kAS + cl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
      const int tile = s * kMWaves + w;
      const int J = tile % kMT;
      if (tile < kMT * kMT && J >= J0 && J < J0 + kAB) {
        const int I = tile / kMT;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          C[s][r] = S[(kMB * I + lr + 4 * r) * kAS + kMB * (J - J0) + lc];
      }
    }
    __syncthreads();
  }
  for (int K = 0; K < kMT; ++K) {
    // the panel to LDS
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
      const int tile = s * kMWaves + w;
      if (tile < kMT * kMT && tile % kMT == K) {
        const int I = tile / kMT;
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(kMB * I + lr + 4 * r) * kPS + lc] = C[s][r];
      }
    }
    __syncthreads();
    // 16 exchange steps on the panel, its rows held one per lane (lanes
    // 0 .. kMR-1 of each wave), the pivot found by a wave reduction and one
    // across the waves
    {
      const int prow_i = w * kMR + l;  // panel row of this lane
      const bool has = l < kMR && prow_i < kMN;
      double rv[kMB];
#pragma unroll
      for (int j = 0; j < kMB; ++j) rv[j] = has ? P[prow_i * kPS + j] : 0.0;
      bool used = has ? rinv[prow_i] >= 0 : true;
#pragma unroll 1
      for (int m = 0; m < kMB; ++m) {
        double vm = 0.0;  // rv[m] (a select chain keeps rv in registers)
#pragma unroll
        for (int j = 0; j < kMB; ++j) vm = j == m ? rv[j] : vm;
        double bv = used ? -1.0 : fabs(vm);
        int bi = used ? kMN : prow_i;
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(bv, off);
          const int oi = __shfl_xor(bi, off);
          if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
          }
        }
        if (l == 0) {
          cand_v[m & 1][w] = bv;
          cand_i[m & 1][w] = bi;
        }
        __syncthreads();
        bv = cand_v[m & 1][0];
        bi = cand_i[m & 1][0];
        for (int q = 1; q < kMWaves; ++q) {
          const double ov = cand_v[m & 1][q];
          const int oi = cand_i[m & 1][q];
          if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
          }
        }
        const int rp = bi;  // uniform over the workgroup
        if (has && prow_i == rp) {
          double pv = vm;
          if (!(bv > 0.0)) {
            pv = 1.0;
            s_sing = 1;
          }
          const double dinv = 1.0 / pv;
#pragma unroll
          for (int j = 0; j < kMB; ++j) prow[j] = (j == m ? 1.0 : rv[j]) * dinv;
          rinv[rp] = kMB * K + m;
          rowpiv[kMB * K + m] = rp;
        }
        __syncthreads();
        if (has) {
          const bool piv = prow_i == rp;
          const double f = piv ? -1.0 : vm;
#pragma unroll
          for (int j = 0; j < kMB; ++j) {
            const double keep = (piv || j == m) ? 0.0 : rv[j];
            rv[j] = keep - f * prow[j];
          }
          used = used || piv;
        }
      }
      if (has) {
#pragma unroll
        for (int j = 0; j < kMB; ++j) P[prow_i * kPS + j] = rv[j];
      }
    }
    __syncthreads();
    // the panel back into its tiles; the pivot rows of the other columns to Bm
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
      const int tile = s * kMWaves + w;
      if (tile >= kMT * kMT) continue;
      const int I = tile / kMT, J = tile % kMT;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kMB * I + lr + 4 * r;
        if (J == K) {
          C[s][r] = P[row * kPS + lc];
        } else {
          const int m = rinv[row] - kMB * K;
          if (m >= 0 && m < kMB) Bm[m * kOS + kMB * J + lc] = C[s][r];
        }
      }
    }
    __syncthreads();
    // left factor: the panel minus the selection of its pivot rows
    if (t < kMB) P[rowpiv[kMB * K + t] * kPS + t] -= 1.0;
    __syncthreads();
    // rank-16 update of every other block column
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
      const int tile = s * kMWaves + w;
      if (tile >= kMT * kMT) continue;
      const int I = tile / kMT, J = tile % kMT;
      if (J == K) continue;
      double a[4], b[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a[c] = P[(kMB * I + lc) * kPS + 4 * c + lr];
        b[c] = Bm[(4 * c + lr) * kOS + kMB * J + lc];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) C[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b[c], C[s], 0, 0, 0);
      // the operands of one tile at a time
      asm volatile("" ::: "memory");
    }
    __syncthreads();
  }
  if (t == 0 && s_sing) atomicOr(status, 1);
  // A^{-1}[i][j] = W[a][b] with i = rinv[a], j = rowpiv[b]; column-major, one
  // block column of W at a time staged so that each output column is written
  // contiguously
  T* out = inv + patch_slot3(g, cx, cy, cz) * kE3;
  double* O = Bm;
  for (int Jb = 0; Jb < kMT; ++Jb) {
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
      const int tile = s * kMWaves + w;
      if (tile >= kMT * kMT || tile % kMT != Jb) continue;
      const int I = tile / kMT;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kMB * I + lr + 4 * r;
        const int i = rinv[row];
        if (i < kNst3) O[lc * kOS + i] = C[s][r];
      }
    }
    __syncthreads();
    for (int e = t; e < kMB * kNst3; e += kMThreads) {
      const int m = e / kNst3, i = e % kNst3;
      const int b = kMB * Jb + m;
      if (b < kNst3) out[(int64_t)rowpiv[b] * kNst3 + i] = (T)O[m * kOS + i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------- element-by-element action

constexpr int kColPart = (kNst3 + 2) / 3;  // 57 columns per thread (3 threads per row)

template <typename T>
__global__ __launch_bounds__(kPT) void ebe3_kernel(Grid3 g, const T* __restrict__ Et,
                                                   const T* __restrict__ x, T* __restrict__ S) {
  __shared__ T xs[kNst3];
  __shared__ T part[3][kNst3];
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % g.nx), cy = (int)((cell / g.nx) % g.ny),
            cz = (int)(cell / ((int64_t)g.nx * g.ny));
  const int t = threadIdx.x;
  if (t < kNst3) xs[t] = x[gidx_st3(g, cx, cy, cz, t)];
  __syncthreads();
  if (t < 3 * kNst3) {
    const int i = t % kNst3, p = t / kNst3;
    const int j0 = p * kColPart, j1 = min(kNst3, j0 + kColPart);
    const T* C = Et + cell * kE3;
    T s = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) s += C[j * kNst3 + i] * xs[j];
    part[p][i] = s;
  }
  __syncthreads();
  if (t < kNst3) S[cell * kNst3 + slot_pos3(t)] = part[0][t] + part[1][t] + part[2][t];
}

// ------------------------------------------------------------------ sweep

template <typename T>
__global__ __launch_bounds__(kPT) void patch_sweep3r_kernel(Grid3 g, const T* __restrict__ inv,
                                                            const T* __restrict__ res,
                                                            T* __restrict__ d, T omega, int px,
                                                            int py, int pz, int ncx, int ncy,
                                                            int64_t slot0) {
  __shared__ T z[kNst3];
  __shared__ T part[3][kNst3];
  const int64_t pid = blockIdx.x;
  const int cx = px + 2 * (int)(pid % ncx);
  const int cy = py + 2 * (int)((pid / ncx) % ncy);
  const int cz = pz + 2 * (int)(pid / ((int64_t)ncx * ncy));
  const int t = threadIdx.x;
  int64_t gi = 0;
  if (t < kNst3) {
    gi = gidx_st3(g, cx, cy, cz, t);
    z[t] = res[gi];
  }
  __syncthreads();
  if (t < 3 * kNst3) {
    const int i = t % kNst3, p = t / kNst3;
    const int j0 = p * kColPart, j1 = min(kNst3, j0 + kColPart);
    const T* C = inv + (slot0 + pid) * kE3;
    T s = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) s += C[j * kNst3 + i] * z[j];
    part[p][i] = s;
  }
  __syncthreads();
  if (t < kNst3) d[gi] += omega * (part[0][t] + part[1][t] + part[2][t]);
}

// -------------------------------------------------------------- transfers

// value of the coarse 1D Q2 nodal basis function I at fine node i (spacing h/4)
__device__ __forceinline__ double w1d3(int I, int i) {
  if ((i & 1) == 0) return (i >> 1) == I ? 1.0 : 0.0;
  const int C = i >> 2;
  const int a = I - 2 * C;
  if (a < 0 || a > 2) return 0.0;
  return q2v(a, 0.25 * (i - 4 * C));
}

template <typename T>
__global__ void restrict3_kernel(Grid3 gf, Grid3 gc, const T* __restrict__ rf, T* __restrict__ rc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= gc.nst) return;
  const int mu = (int)(r / gc.ns);
  const int64_t s = r % gc.ns;
  const T* f = rf + (int64_t)mu * gf.ns;
  double acc = 0.0;
  if (s < gc.nv) {
    const int comp = (int)(s / gc.nn);
    const int64_t node = s % gc.nn;
    const int64_t NXc = 2 * gc.nx + 1, NYc = 2 * gc.ny + 1;
    const int64_t NXf = 2 * gf.nx + 1, NYf = 2 * gf.ny + 1;
    const int IX = (int)(node % NXc), IY = (int)((node / NXc) % NYc), IZ = (int)(node / (NXc * NYc));
    const T* fc = f + (int64_t)comp * gf.nn;
    for (int iz = 2 * IZ - 3; iz <= 2 * IZ + 3; ++iz) {
      if (iz < 0 || iz > 2 * gf.nz) continue;
      const double wz = w1d3(IZ, iz);
      if (wz == 0.0) continue;
      for (int iy = 2 * IY - 3; iy <= 2 * IY + 3; ++iy) {
        if (iy < 0 || iy > 2 * gf.ny) continue;
        const double wy = w1d3(IY, iy);
        if (wy == 0.0) continue;
        for (int ix = 2 * IX - 3; ix <= 2 * IX + 3; ++ix) {
          if (ix < 0 || ix > 2 * gf.nx) continue;
          const double wx = w1d3(IX, ix);
          if (wx == 0.0) continue;
          acc += wx * wy * wz * (double)fc[ix + NXf * (iy + NYf * (int64_t)iz)];
        }
      }
    }
  } else {
    const int64_t cell = (s - gc.nv) / 4;
    const int j = (int)((s - gc.nv) % 4);
    const int cx = (int)(cell % gc.nx), cy = (int)((cell / gc.nx) % gc.ny),
              cz = (int)(cell / ((int64_t)gc.nx * gc.ny));
    for (int ch = 0; ch < 8; ++ch) {
      const int o[3] = {ch & 1, (ch >> 1) & 1, ch >> 2};
      const int64_t fcell = cell_index3(gf, 2 * cx + o[0], 2 * cy + o[1], 2 * cz + o[2]);
      const T* fp = f + gf.nv + 4 * fcell;
      if (j == 0)
        acc += (double)fp[0];
      else
        acc += 0.5 * (o[j - 1] - 0.5) * (double)fp[0] + 0.5 * (double)fp[j];
    }
  }
  rc[r] = (T)acc;
}

template <typename T>
__global__ void prolong_add3_kernel(Grid3 gf, Grid3 gc, const T* __restrict__ dc,
                                    T* __restrict__ df) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= gf.nst) return;
  const int mu = (int)(r / gf.ns);
  const int64_t s = r % gf.ns;
  const T* c = dc + (int64_t)mu * gc.ns;
  double acc = 0.0;
  if (s < gf.nv) {
    const int comp = (int)(s / gf.nn);
    const int64_t node = s % gf.nn;
    const int64_t NXc = 2 * gc.nx + 1, NYc = 2 * gc.ny + 1;
    const int64_t NXf = 2 * gf.nx + 1, NYf = 2 * gf.ny + 1;
    const int ii[3] = {(int)(node % NXf), (int)((node / NXf) % NYf), (int)(node / (NXf * NYf))};
    int I[3][3], nI[3];
    double w[3][3];
    for (int k = 0; k < 3; ++k) {
      const int v = ii[k];
      if ((v & 1) == 0) {
        I[k][0] = v >> 1;
        w[k][0] = 1.0;
        nI[k] = 1;
      } else {
        const int C = v >> 2;
        for (int a = 0; a < 3; ++a) {
          I[k][a] = 2 * C + a;
          w[k][a] = q2v(a, 0.25 * (v - 4 * C));
        }
        nI[k] = 3;
      }
    }
    const T* cc = c + (int64_t)comp * gc.nn;
    for (int cz = 0; cz < nI[2]; ++cz)
      for (int cy = 0; cy < nI[1]; ++cy)
        for (int cx = 0; cx < nI[0]; ++cx)
          acc += w[0][cx] * w[1][cy] * w[2][cz] *
                 (double)cc[I[0][cx] + NXc * (I[1][cy] + NYc * (int64_t)I[2][cz])];
  } else {
    const int64_t fcell = (s - gf.nv) / 4;
    const int j = (int)((s - gf.nv) % 4);
    const int fx = (int)(fcell % gf.nx), fy = (int)((fcell / gf.nx) % gf.ny),
              fz = (int)(fcell / ((int64_t)gf.nx * gf.ny));
    const int o[3] = {fx & 1, fy & 1, fz & 1};
    const T* cp = c + gc.nv + 4 * cell_index3(gc, fx >> 1, fy >> 1, fz >> 1);
    if (j == 0)
      acc = (double)cp[0] + 0.5 * (o[0] - 0.5) * (double)cp[1] + 0.5 * (o[1] - 0.5) * (double)cp[2] +
            0.5 * (o[2] - 0.5) * (double)cp[3];
    else
      acc = 0.5 * (double)cp[j];
  }
  df[r] = (T)((double)df[r] + acc);
}

// ------------------------------------------------------------ coarsest level

// rows of the cells of one colour: thread per (cell, local row)
__global__ void coarse_assemble3_kernel(Grid3 g, const double* __restrict__ E, double* __restrict__ A,
                                        int px, int py, int pz, int ncx, int ncy, int64_t count) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pid = id / kNst3;
  const int r = (int)(id % kNst3);
  if (pid >= count) return;
  const int cx = px + 2 * (int)(pid % ncx);
  const int cy = py + 2 * (int)((pid / ncx) % ncy);
  const int cz = pz + 2 * (int)(pid / ((int64_t)ncx * ncy));
  const int64_t cell = cell_index3(g, cx, cy, cz);
  const int64_t n = g.nst;
  const int64_t gr = gidx_st3(g, cx, cy, cz, r);
  for (int c = 0; c < kNst3; ++c)
    A[gr * n + gidx_st3(g, cx, cy, cz, c)] += E[cell * kE3 + r * kNst3 + c];
}

inline unsigned nblk3(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_galerkin3d_from_fine(const Grid3& gc, const Grid3& gf, double tau,
                                       const double* Es0, const double* Es1, double* Ec,
                                       hipStream_t s) {
  FineSrc3 src{gf, tau, Es0, Es1};
  hipLaunchKernelGGL(galerkin3d_kernel<FineSrc3>, dim3((unsigned)gc.nc, 64), dim3(256), 0, s, gc,
                     gf, src, Ec);
  return hipGetLastError();
}

hipError_t launch_galerkin3d(const Grid3& gc, const Grid3& gf, const double* Ef, double* Ec,
                             hipStream_t s) {
  StoredSrc3 src{Ef};
  hipLaunchKernelGGL(galerkin3d_kernel<StoredSrc3>, dim3((unsigned)gc.nc, 64), dim3(256), 0, s, gc,
                     gf, src, Ec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose_convert3(int64_t ncells, const double* E, T* Et, hipStream_t s) {
  hipLaunchKernelGGL(transpose_convert3_kernel<T>, dim3(nblk3(ncells * kE3, 256)), dim3(256), 0, s,
                     ncells, E, Et);
  return hipGetLastError();
}

namespace {
template <typename T, typename Src>
hipError_t patches3r_by_colour(const Grid3& g, Src src, T* inv, int* status, hipStream_t s) {
  for (int c = 0; c < 8; ++c) {
    const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
    const int64_t np = colour_count3(g, c);
    if (np == 0) continue;
    hipLaunchKernelGGL((patch3m_kernel<T, Src>), dim3((unsigned)np), dim3(kMThreads), 0, s, g, src, inv,
                       status, px, py, pz, (g.nx - px + 1) / 2, (g.ny - py + 1) / 2);
  }
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_level_patches3d(const Grid3& g, const double* E, T* inv, int* status,
                                  hipStream_t s) {
  return patches3r_by_colour<T>(g, StoredSrc3{E}, inv, status, s);
}

template <typename T>
hipError_t launch_exact_fine_patches3d(const Grid3& g, double tau, const double* Es0,
                                       const double* Es1, T* inv, int* status, hipStream_t s) {
  return patches3r_by_colour<T>(g, FineSrc3{g, tau, Es0, Es1}, inv, status, s);
}

template <typename T>
hipError_t launch_ebe_apply3d(const Grid3& g, const T* Et, const T* x, const T* b, T* y, T* S,
                              hipStream_t s) {
  hipLaunchKernelGGL(ebe3_kernel<T>, dim3((unsigned)g.nc), dim3(kPT), 0, s, g, Et, x, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gather3<T>(g, S, b, y, s);
}

template <typename T>
hipError_t launch_patch_sweep3r(const Grid3& g, const T* inv, const T* res, T* d, double omega,
                                hipStream_t s) {
  int64_t slot0 = 0;
  for (int c = 0; c < 8; ++c) {
    const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
    const int64_t np = colour_count3(g, c);
    if (np > 0)
      hipLaunchKernelGGL(patch_sweep3r_kernel<T>, dim3((unsigned)np), dim3(kPT), 0, s, g, inv, res,
                         d, (T)omega, px, py, pz, (g.nx - px + 1) / 2, (g.ny - py + 1) / 2, slot0);
    slot0 += np;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict3(const Grid3& gf, const Grid3& gc, const T* rf, T* rc, hipStream_t s) {
  hipLaunchKernelGGL(restrict3_kernel<T>, dim3(nblk3(gc.nst, 256)), dim3(256), 0, s, gf, gc, rf, rc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add3(const Grid3& gf, const Grid3& gc, const T* dc, T* df,
                               hipStream_t s) {
  hipLaunchKernelGGL(prolong_add3_kernel<T>, dim3(nblk3(gf.nst, 256)), dim3(256), 0, s, gf, gc, dc,
                     df);
  return hipGetLastError();
}

hipError_t launch_coarse_assemble3(const Grid3& g, const double* E, double* A, hipStream_t s) {
  for (int c = 0; c < 8; ++c) {
    const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
    const int64_t np = colour_count3(g, c);
    if (np == 0) continue;
    hipLaunchKernelGGL(coarse_assemble3_kernel, dim3(nblk3(np * kNst3, 256)), dim3(256), 0, s, g, E,
                       A, px, py, pz, (g.nx - px + 1) / 2, (g.ny - py + 1) / 2, np);
  }
  return hipGetLastError();
}

#define PNS_MG3D_INST(T)                                                                         \
  template hipError_t launch_transpose_convert3<T>(int64_t, const double*, T*, hipStream_t);    \
  template hipError_t launch_level_patches3d<T>(const Grid3&, const double*, T*, int*,          \
                                                hipStream_t);                                   \
  template hipError_t launch_exact_fine_patches3d<T>(const Grid3&, double, const double*,       \
                                                     const double*, T*, int*, hipStream_t);     \
  template hipError_t launch_ebe_apply3d<T>(const Grid3&, const T*, const T*, const T*, T*, T*, \
                                            hipStream_t);                                       \
  template hipError_t launch_patch_sweep3r<T>(const Grid3&, const T*, const T*, T*, double,     \
                                              hipStream_t);                                     \
  template hipError_t launch_restrict3<T>(const Grid3&, const Grid3&, const T*, T*, hipStream_t); \
  template hipError_t launch_prolong_add3<T>(const Grid3&, const Grid3&, const T*, T*,          \
                                             hipStream_t);
PNS_MG3D_INST(double)
PNS_MG3D_INST(float)
#undef PNS_MG3D_INST

}  // namespace pns
