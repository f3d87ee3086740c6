// Per-iteration smoother and transfer kernels (Sec. 6.3):
// * coarse-level operator action with Galerkin element matrices: the
//   transposed (column-major) element matrices are stored like the patch
//   inverses, so the sweep kernels below stream them (omega = +-1);
// * additive Vanka update d += omega sum_K R_K^T A_K^{-1} R_K res,
//   eq. (stmg-vanka-update): the stored patch inverses streamed column by
//   column (level 0: complex 21x21 time-diagonal form, three patches per wave;
//   real 42x42: one patch per wave, or three with two rows per lane); each
//   form comes in variants of workgroup size and loads in flight, among which
//   the smoother setup picks the fastest on the device;
// * two ways to sum the per-patch results: four colour launches adding into
//   the vector (patches of one parity class share no unknown), or one launch
//   over every patch writing its 42 results to the patch's slot, then a node
//   gather summing the slots of the cells around each unknown in a fixed order
//   (two launches instead of four, used on the coarse levels, where the colour
//   launches are short);
// * restriction P^T and prolongation P of the nested Q2 / P1disc spaces;
// * dense coarsest solve with the stored inverse.
#include <type_traits>

#include "pns_internal.h"

namespace pns {
namespace {

__device__ __forceinline__ int64_t gidx(const Grid& g, int cx, int cy, int l) {
  const int mu = l / kNs, i = l % kNs;
  const int NX = 2 * g.nx + 1;
  if (i < 18) {
    const int comp = i / 9, a = i % 9;
    return (int64_t)mu * g.ns + (int64_t)comp * g.nn + (int64_t)(2 * cy + a / 3) * NX +
           (2 * cx + a % 3);
  }
  return (int64_t)mu * g.ns + g.nv + 3 * ((int64_t)cy * g.nx + cx) + (i - 18);
}

// Cell of the patch stored at position q (0 <= q < nc) of the colour-major
// order of patch_slot: the inverse of that cell.
__device__ __forceinline__ void slot_cell(const Grid& g, int64_t q, int& cx, int& cy) {
  const int64_t ncx0 = (g.nx + 1) / 2, ncx1 = g.nx / 2, ncy0 = (g.ny + 1) / 2;
  int px = 0, py = 0;
  int64_t w = ncx0;
  if (q >= ncx0 * ncy0) {
    q -= ncx0 * ncy0;
    if (q < ncx1 * ncy0) {
      px = 1;
      w = ncx1;
    } else {
      q -= ncx1 * ncy0;
      if (q < ncx0 * (g.ny / 2)) {
        py = 1;
      } else {
        q -= ncx0 * (g.ny / 2);
        px = py = 1;
        w = ncx1;
      }
    }
  }
  cx = px + 2 * (int)(q % w);
  cy = py + 2 * (int)(q / w);
}

// Patch of a launch: in a colour launch the pid-th cell of the colour class
// (px, py); in a slot launch (SLOT) the cell whose inverse sits at position
// pid, every patch of the level in one launch.
template <bool SLOT>
__device__ __forceinline__ bool launch_cell(const Grid& g, int64_t pid, int px, int py, int ncx,
                                            int ncy, int& cx, int& cy) {
  if (SLOT) {
    if (pid >= g.nc) return false;
    slot_cell(g, pid, cx, cy);
    return true;
  }
  if (pid >= (int64_t)ncx * ncy) return false;
  cx = px + 2 * (int)(pid % ncx);
  cy = py + 2 * (int)(pid / ncx);
  return true;
}

// Real 42x42 patches, one wave per patch, lane r < 42 forms row r; WAVES
// patches per workgroup, UNROLL column loads in flight.  Colour launch: d[gi]
// += omega * row; slot launch: out[42 pid + r] = omega * row.
template <typename T, int WAVES, int UNROLL, bool SLOT>
__global__ __launch_bounds__(64 * WAVES) void patch_sweep_kernel(Grid g, const T* __restrict__ inv,
                                                                 const T* __restrict__ res,
                                                                 T* __restrict__ d, T omega,
                                                                 int px, int py, int ncx,
                                                                 int ncy) {
  __shared__ T rhs[WAVES][kNst];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t pid = (int64_t)blockIdx.x * WAVES + w;
  int cx = 0, cy = 0;
  const bool active = launch_cell<SLOT>(g, pid, px, py, ncx, ncy, cx, cy);
  int64_t gi = 0;
  if (active && lane < kNst) {
    gi = gidx(g, cx, cy, lane);
    rhs[w][lane] = res[gi];
  }
  __syncthreads();
  if (!active || lane >= kNst) return;
  const T* A = inv + patch_slot(g, cx, cy) * (kNst * kNst);
  T acc = 0;
#pragma unroll UNROLL
  for (int j = 0; j < kNst; ++j) acc += A[j * kNst + lane] * rhs[w][j];
  if (SLOT)
    d[pid * kNst + lane] = omega * acc;
  else
    d[gi] += omega * acc;
}

// Real 42x42 patches, three patches per wave, lane 21 p + i forms rows 2i and
// 2i + 1 of patch p from paired loads (63 of 64 lanes busy); WAVES waves per
// workgroup, UNROLL column loads in flight; colour or slot launch as above.
template <typename T, int WAVES, int UNROLL, bool SLOT>
__global__ __launch_bounds__(64 * WAVES) void patch_sweep2_kernel(Grid g, const T* __restrict__ inv,
                                                                  const T* __restrict__ res,
                                                                  T* __restrict__ d, T omega,
                                                                  int px, int py, int ncx,
                                                                  int ncy) {
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  __shared__ T rhs[WAVES][3][kNst];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = lane / 21, i = lane % 21;
  const int64_t pid = ((int64_t)blockIdx.x * WAVES + w) * 3 + p;
  int cx = 0, cy = 0;
  const bool active = lane < 63 && launch_cell<SLOT>(g, pid, px, py, ncx, ncy, cx, cy);
  int64_t g0 = 0, g1 = 0;
  if (active) {
    g0 = gidx(g, cx, cy, 2 * i);
    g1 = gidx(g, cx, cy, 2 * i + 1);
    rhs[w][p][2 * i] = res[g0];
    rhs[w][p][2 * i + 1] = res[g1];
  }
  __syncthreads();
  if (!active) return;
  // column j starts at an even offset, so the pair (2i, 2i+1) is aligned
  const T2* A = reinterpret_cast<const T2*>(inv + patch_slot(g, cx, cy) * (kNst * kNst));
  T a0 = 0, a1 = 0;
#pragma unroll UNROLL
  for (int j = 0; j < kNst; ++j) {
    const T2 c = A[j * (kNst / 2) + i];
    const T r = rhs[w][p][j];
    a0 += c.x * r;
    a1 += c.y * r;
  }
  if (SLOT) {
    d[pid * kNst + 2 * i] = omega * a0;
    d[pid * kNst + 2 * i + 1] = omega * a1;
  } else {
    d[g0] += omega * a0;
    d[g1] += omega * a1;
  }
}

// level-0 patches in time-diagonal form (complex 21x21 inverse): three
// patches per wave, lane 21 p + i handles spatial unknown i of patch p
template <typename T, int WAVES, int UNROLL>
__global__ __launch_bounds__(64 * WAVES) void patch_sweep_c_kernel(Grid g, const T* __restrict__ inv,
                                                                   const T* __restrict__ res,
                                                                   T* __restrict__ d, T omega,
                                                                   int px, int py, int ncx,
                                                                   int ncy) {
  __shared__ T zs[WAVES][3][2][kNs];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = lane / kNs, i = lane % kNs;
  const int64_t pid = ((int64_t)blockIdx.x * WAVES + w) * 3 + p;
  const bool active = lane < 3 * kNs && pid < (int64_t)ncx * ncy;
  int cx = 0, cy = 0;
  int64_t g0 = 0, g1 = 0;
  if (active) {
    cx = px + 2 * (int)(pid % ncx);
    cy = py + 2 * (int)(pid / ncx);
    g0 = gidx(g, cx, cy, i);
    g1 = gidx(g, cx, cy, kNs + i);
    const T r0 = res[g0], r1 = res[g1];
    zs[w][p][0][i] = (T)kZr0 * r0;
    zs[w][p][1][i] = (T)kZi0 * r0 + (T)kZi1 * r1;
  }
  __syncthreads();
  if (!active) return;
  const T* C = inv + patch_slot(g, cx, cy) * (2 * kNs * kNs);
  T yr = 0, yi = 0;
#pragma unroll UNROLL
  for (int j = 0; j < kNs; ++j) {
    const T cr = C[2 * (j * kNs + i)], ci = C[2 * (j * kNs + i) + 1];
    const T zr = zs[w][p][0][j], zi = zs[w][p][1][j];
    yr += cr * zr - ci * zi;
    yi += cr * zi + ci * zr;
  }
  d[g0] += omega * (T)2 * yr;
  d[g1] += omega * (T)2 * (yr - (T)kBackIm * yi);
}

template <typename T>
__global__ void copy_kernel(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// y = base + sum of the slot values of every cell whose patch holds the
// unknown (base = 0 when null; y may be base): a velocity node on a cell
// corner is in up to four patches, on an edge in up to two, inside a cell in
// one; a pressure coefficient in its cell's.  Cells are visited row by row, so
// the order of the sum is fixed.
template <typename T>
__global__ __launch_bounds__(256) void slot_gather_kernel(Grid g, const T* __restrict__ slot,
                                                          const T* base, T* y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.nst) return;
  const int mu = (int)(r / g.ns);
  const int64_t s = r % g.ns;
  double acc = base ? (double)base[r] : 0.0;
  if (s < g.nv) {
    const int comp = (int)(s / g.nn);
    const int64_t node = s % g.nn;
    const int NX = 2 * g.nx + 1;
    const int ix = (int)(node % NX), iy = (int)(node / NX);
    // cells touching the node along each axis and the node's local index there
    int cxs[2], axs[2], cys[2], ays[2], ncx = 0, ncy = 0;
    if (ix & 1) {
      cxs[0] = ix >> 1; axs[0] = 1; ncx = 1;
    } else {
      if (ix > 0) { cxs[ncx] = (ix >> 1) - 1; axs[ncx] = 2; ++ncx; }
      if (ix < 2 * g.nx) { cxs[ncx] = ix >> 1; axs[ncx] = 0; ++ncx; }
    }
    if (iy & 1) {
      cys[0] = iy >> 1; ays[0] = 1; ncy = 1;
    } else {
      if (iy > 0) { cys[ncy] = (iy >> 1) - 1; ays[ncy] = 2; ++ncy; }
      if (iy < 2 * g.ny) { cys[ncy] = iy >> 1; ays[ncy] = 0; ++ncy; }
    }
    const int loc = mu * kNs + comp * 9;
    for (int b = 0; b < ncy; ++b)
      for (int a = 0; a < ncx; ++a)
        acc += (double)slot[patch_slot(g, cxs[a], cys[b]) * kNst + loc + 3 * ays[b] + axs[a]];
  } else {
    const int64_t cell = (s - g.nv) / 3;
    const int j = (int)((s - g.nv) % 3);
    const int cx = (int)(cell % g.nx), cy = (int)(cell / g.nx);
    acc += (double)slot[patch_slot(g, cx, cy) * kNst + mu * kNs + 18 + j];
  }
  y[r] = (T)acc;
}

__device__ __forceinline__ double w1d(int I, int i) {
  // value of the coarse 1D Q2 nodal basis function I at fine node i
  if ((i & 1) == 0) return (i >> 1) == I ? 1.0 : 0.0;
  const int C = i >> 2;
  const int a = I - 2 * C;
  if (a < 0 || a > 2) return 0.0;
  return q2v(a, 0.25 * (i - 4 * C));
}

template <typename T>
__global__ void restrict_kernel(Grid gf, Grid gc, const T* __restrict__ rf, T* __restrict__ rc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= gc.nst) return;
  const int mu = (int)(r / gc.ns);
  const int64_t s = r % gc.ns;
  const T* f = rf + (int64_t)mu * gf.ns;
  double acc = 0.0;
  if (s < gc.nv) {
    const int comp = (int)(s / gc.nn);
    const int64_t node = s % gc.nn;
    const int NXc = 2 * gc.nx + 1, NXf = 2 * gf.nx + 1;
    const int IX = (int)(node % NXc), IY = (int)(node / NXc);
    for (int iy = 2 * IY - 3; iy <= 2 * IY + 3; ++iy) {
      if (iy < 0 || iy > 2 * gf.ny) continue;
      const double wy = w1d(IY, iy);
      if (wy == 0.0) continue;
      for (int ix = 2 * IX - 3; ix <= 2 * IX + 3; ++ix) {
        if (ix < 0 || ix > 2 * gf.nx) continue;
        const double wx = w1d(IX, ix);
        if (wx == 0.0) continue;
        acc += wx * wy * (double)f[(int64_t)comp * gf.nn + (int64_t)iy * NXf + ix];
      }
    }
  } else {
    const int64_t cell = (s - gc.nv) / 3;
    const int j = (int)((s - gc.nv) % 3);
    const int cx = (int)(cell % gc.nx), cy = (int)(cell / gc.nx);
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        const int64_t fc = (int64_t)(2 * cy + oy) * gf.nx + (2 * cx + ox);
        const T* fp = f + gf.nv + 3 * fc;
        if (j == 0)
          acc += (double)fp[0];
        else if (j == 1)
          acc += 0.5 * (ox - 0.5) * (double)fp[0] + 0.5 * (double)fp[1];
        else
          acc += 0.5 * (oy - 0.5) * (double)fp[0] + 0.5 * (double)fp[2];
      }
  }
  rc[r] = (T)acc;
}

template <typename T>
__global__ void prolong_add_kernel(Grid gf, Grid gc, const T* __restrict__ dc, T* __restrict__ df) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= gf.nst) return;
  const int mu = (int)(r / gf.ns);
  const int64_t s = r % gf.ns;
  const T* c = dc + (int64_t)mu * gc.ns;
  double acc = 0.0;
  if (s < gf.nv) {
    const int comp = (int)(s / gf.nn);
    const int64_t node = s % gf.nn;
    const int NXc = 2 * gc.nx + 1, NXf = 2 * gf.nx + 1;
    const int ix = (int)(node % NXf), iy = (int)(node / NXf);
    int Ix[3], Iy[3], nxI = 0, nyI = 0;
    double wx[3], wy[3];
    if ((ix & 1) == 0) {
      Ix[0] = ix >> 1; wx[0] = 1.0; nxI = 1;
    } else {
      const int C = ix >> 2;
      for (int a = 0; a < 3; ++a) { Ix[a] = 2 * C + a; wx[a] = q2v(a, 0.25 * (ix - 4 * C)); }
      nxI = 3;
    }
    if ((iy & 1) == 0) {
      Iy[0] = iy >> 1; wy[0] = 1.0; nyI = 1;
    } else {
      const int C = iy >> 2;
      for (int a = 0; a < 3; ++a) { Iy[a] = 2 * C + a; wy[a] = q2v(a, 0.25 * (iy - 4 * C)); }
      nyI = 3;
    }
    for (int b = 0; b < nyI; ++b)
      for (int a = 0; a < nxI; ++a)
        acc += wx[a] * wy[b] * (double)c[(int64_t)comp * gc.nn + (int64_t)Iy[b] * NXc + Ix[a]];
  } else {
    const int64_t fc = (s - gf.nv) / 3;
    const int j = (int)((s - gf.nv) % 3);
    const int fx = (int)(fc % gf.nx), fy = (int)(fc / gf.nx);
    const int ox = fx & 1, oy = fy & 1;
    const T* cp = c + gc.nv + 3 * ((int64_t)(fy >> 1) * gc.nx + (fx >> 1));
    if (j == 0)
      acc = (double)cp[0] + 0.5 * (ox - 0.5) * (double)cp[1] + 0.5 * (oy - 0.5) * (double)cp[2];
    else
      acc = 0.5 * (double)cp[j];
  }
  df[r] = (T)((double)df[r] + acc);
}

// d = Ainv r~, r~ = r with the pinned entries zeroed, the inverse stored in the
// precision T of the vectors; one wave per kGemvRows consecutive rows, so each
// load of r serves kGemvRows rows (r is re-read from cache once per row group,
// not once per row); pair loads of the rows and of r (n is even, so every row
// starts pair-aligned), four steps in flight, sums in FP64
constexpr int kGemvRows = 8;

template <typename T>
__global__ __launch_bounds__(256) void dense_gemv_kernel(int64_t n, const T* __restrict__ Ainv,
                                                         const T* __restrict__ r, T* __restrict__ d,
                                                         int64_t pin0, int64_t pin1) {
  // the pinned entries of r count as zero: their products are taken out once
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kGemvRows;
  const int lane = threadIdx.x & 63;
  if (row0 >= n) return;
  // rows past the end repeat the last row (their results are not stored)
  const T2* A[kGemvRows];
#pragma unroll
  for (int k = 0; k < kGemvRows; ++k)
    A[k] = reinterpret_cast<const T2*>(Ainv + (row0 + k < n ? row0 + k : n - 1) * n);
  const T2* r2 = reinterpret_cast<const T2*>(r);
  double acc[kGemvRows][2];
#pragma unroll
  for (int k = 0; k < kGemvRows; ++k) acc[k][0] = acc[k][1] = 0.0;
  const int64_t npair = n >> 1;
  int64_t q = lane;
  for (; q + 192 < npair; q += 256) {
    T2 b[4], a[4][kGemvRows];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      b[u] = r2[q + 64 * u];
#pragma unroll
      for (int k = 0; k < kGemvRows; ++k) a[u][k] = A[k][q + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < kGemvRows; ++k) {
        acc[k][0] += (double)a[u][k].x * (double)b[u].x;
        acc[k][1] += (double)a[u][k].y * (double)b[u].y;
      }
  }
  for (; q < npair; q += 64) {
    const T2 b = r2[q];
#pragma unroll
    for (int k = 0; k < kGemvRows; ++k) {
      const T2 a = A[k][q];
      acc[k][0] += (double)a.x * (double)b.x;
      acc[k][1] += (double)a.y * (double)b.y;
    }
  }
#pragma unroll
  for (int k = 0; k < kGemvRows; ++k) {
    double s = acc[k][0] + acc[k][1];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && row0 + k < n) {
      const T* Ar = Ainv + (row0 + k) * n;
      if (pin0 >= 0) s -= (double)Ar[pin0] * (double)r[pin0];
      if (pin1 >= 0) s -= (double)Ar[pin1] * (double)r[pin1];
      d[row0 + k] = (T)s;
    }
  }
}

template <typename T>
__global__ void fill_kernel(int64_t n, T v, T* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

template <typename T>
hipError_t launch_copy(int64_t n, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

namespace {

// The four colour launches of one additive step with one kernel variant;
// PPB patches per workgroup.
template <typename T, typename K>
hipError_t sweep_colours(K kern, int threads, int ppb, const Grid& g, const T* inv, const T* res,
                         T* d, double omega, hipStream_t s) {
  for (int c = 0; c < 4; ++c) {
    const int px = c & 1, py = c >> 1;
    const int ncx = (g.nx - px + 1) / 2, ncy = (g.ny - py + 1) / 2;
    const int64_t np = (int64_t)ncx * ncy;
    if (np == 0) continue;
    hipLaunchKernelGGL(kern, dim3(nblk(np, ppb)), dim3(threads), 0, s, g, inv, res, d, (T)omega,
                       px, py, ncx, ncy);
  }
  return hipGetLastError();
}

// One slot launch over every patch of the level (PPB patches per workgroup),
// writing omega A_K^{-1} R_K res to the patch slots, then the node gather y =
// base + sum of the slots.
template <typename T, typename K>
hipError_t sweep_slots(K kern, int threads, int ppb, const Grid& g, const T* inv, const T* res,
                       const T* base, T* y, double omega, T* slot, hipStream_t s) {
  if (g.nc > 0)
    hipLaunchKernelGGL(kern, dim3(nblk(g.nc, ppb)), dim3(threads), 0, s, g, inv, res, slot,
                       (T)omega, 0, 0, 0, 0);
  hipLaunchKernelGGL(slot_gather_kernel<T>, dim3(nblk(g.nst, 256)), dim3(256), 0, s, g,
                     (const T*)slot, base, y);
  return hipGetLastError();
}

// Launchers of the variants: four colour launches adding into d (slot null),
// or the slot launch and gather with d = base + sum (slot non-null; base is d
// for a sweep, b or null for the coarse-level action).
template <typename T, int W, int U>
hipError_t sweep_r1(const Grid& g, const T* inv, const T* res, const T* base, T* d, double omega,
                    T* slot, hipStream_t s) {
  if (slot)
    return sweep_slots<T>(patch_sweep_kernel<T, W, U, true>, 64 * W, W, g, inv, res, base, d,
                          omega, slot, s);
  return sweep_colours<T>(patch_sweep_kernel<T, W, U, false>, 64 * W, W, g, inv, res, d, omega, s);
}
template <typename T, int W, int U>
hipError_t sweep_r2(const Grid& g, const T* inv, const T* res, const T* base, T* d, double omega,
                    T* slot, hipStream_t s) {
  if (slot)
    return sweep_slots<T>(patch_sweep2_kernel<T, W, U, true>, 64 * W, 3 * W, g, inv, res, base,
                          d, omega, slot, s);
  return sweep_colours<T>(patch_sweep2_kernel<T, W, U, false>, 64 * W, 3 * W, g, inv, res, d,
                          omega, s);
}
template <typename T, int W, int U>
hipError_t sweep_c(const Grid& g, const T* inv, const T* res, const T* base, T* d, double omega,
                   T* slot, hipStream_t s) {
  // the complex form lives on level 0 only, which keeps the colour launches
  if (slot) return hipErrorInvalidValue;
  return sweep_colours<T>(patch_sweep_c_kernel<T, W, U>, 64 * W, 3 * W, g, inv, res, d, omega, s);
}

template <typename T>
using SweepFn = hipError_t (*)(const Grid&, const T*, const T*, const T*, T*, double, T*,
                               hipStream_t);

// variant tables: {launcher, waves per workgroup, column loads in flight, rows per lane}
template <typename T>
struct SweepVariant {
  SweepFn<T> fn;
  int waves, unroll, rows;
};

template <typename T>
const SweepVariant<T>* real_variants() {
  static const SweepVariant<T> v[] = {
      {sweep_r1<T, 4, 6>, 4, 6, 1},   {sweep_r1<T, 1, 6>, 1, 6, 1},   {sweep_r1<T, 2, 6>, 2, 6, 1},
      {sweep_r1<T, 1, 42>, 1, 42, 1}, {sweep_r1<T, 2, 42>, 2, 42, 1}, {sweep_r1<T, 4, 42>, 4, 42, 1},
      {sweep_r2<T, 1, 7>, 1, 7, 2},   {sweep_r2<T, 2, 7>, 2, 7, 2},   {sweep_r2<T, 4, 7>, 4, 7, 2},
      {sweep_r2<T, 1, 42>, 1, 42, 2}, {sweep_r2<T, 2, 42>, 2, 42, 2}, {sweep_r2<T, 4, 42>, 4, 42, 2}};
  return v;
}
template <typename T>
const SweepVariant<T>* complex_variants() {
  static const SweepVariant<T> v[] = {
      {sweep_c<T, 4, 7>, 4, 7, 1},  {sweep_c<T, 1, 7>, 1, 7, 1},  {sweep_c<T, 2, 7>, 2, 7, 1},
      {sweep_c<T, 1, 21>, 1, 21, 1}, {sweep_c<T, 2, 21>, 2, 21, 1}, {sweep_c<T, 4, 21>, 4, 21, 1}};
  return v;
}

}  // namespace

int sweep_variant_count(bool complex_form) { return complex_form ? 6 : 12; }

void sweep_variant_shape(bool complex_form, int v, int out[3]) {
  const SweepVariant<double>& e = complex_form ? complex_variants<double>()[v]
                                               : real_variants<double>()[v];
  out[0] = e.waves;
  out[1] = e.unroll;
  out[2] = e.rows;
}

template <typename T>
hipError_t launch_patch_sweep(const Grid& g, const T* inv, const T* res, T* d, double omega,
                              int variant, T* slot, hipStream_t s, bool d_zero) {
  // slot form with d = 0 on entry: the gather writes d = sum of the slots
  return real_variants<T>()[variant].fn(g, inv, res, (slot && d_zero) ? nullptr : d, d, omega,
                                        slot, s);
}

template <typename T>
hipError_t launch_patch_sweep_c(const Grid& g, const T* inv, const T* res, T* d, double omega,
                                int variant, hipStream_t s) {
  return complex_variants<T>()[variant].fn(g, inv, res, d, d, omega, nullptr, s);
}

// Coarse-level action from the transposed element matrices, stored per cell
// at its patch slot: y = 0 (mode 0) or b (mode 1), plus sign E_c x_c summed
// over the cells, which is the additive patch step with the element matrices
// in place of the inverses (omega = sign) in the level's sweep variant: with
// the per-cell slots and the node gather (slot non-null), else y set first and
// the four colour passes adding into it (cells of one colour share no unknown)
template <typename T>
hipError_t launch_ebe_apply(const Grid& g, const T* E, const T* x, const T* b, T* y, int mode,
                            int variant, T* slot, hipStream_t s) {
  const double sign = mode == 0 ? 1.0 : -1.0;
  if (slot) return real_variants<T>()[variant].fn(g, E, x, mode == 0 ? nullptr : b, y, sign, slot, s);
  if (mode == 0)
    hipLaunchKernelGGL(fill_kernel<T>, dim3(nblk(g.nst, 256)), dim3(256), 0, s, g.nst, (T)0, y);
  else
    hipLaunchKernelGGL(copy_kernel<T>, dim3(nblk(g.nst, 256)), dim3(256), 0, s, g.nst, b, y);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return real_variants<T>()[variant].fn(g, E, x, y, y, sign, nullptr, s);
}

template <typename T>
hipError_t launch_restrict(const Grid& gf, const Grid& gc, const T* rf, T* rc, hipStream_t s) {
  hipLaunchKernelGGL(restrict_kernel<T>, dim3(nblk(gc.nst, 256)), dim3(256), 0, s, gf, gc, rf, rc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Grid& gf, const Grid& gc, const T* dc, T* df, hipStream_t s) {
  hipLaunchKernelGGL(prolong_add_kernel<T>, dim3(nblk(gf.nst, 256)), dim3(256), 0, s, gf, gc, dc,
                     df);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_gemv(int64_t n, const T* Ainv, const T* r, T* d, const int64_t* pin,
                             int npin, hipStream_t s) {
  // space-time sizes are 2 ns: rows are pair-aligned; A and r are read in pairs
  if ((n & 1) || ((uintptr_t)r % (2 * sizeof(T))) != 0 || ((uintptr_t)Ainv % (2 * sizeof(T))) != 0)
    return hipErrorInvalidValue;
  const int64_t p0 = npin > 0 ? pin[0] : -1, p1 = npin > 1 ? pin[1] : -1;
  hipLaunchKernelGGL(dense_gemv_kernel<T>, dim3(nblk(n, 4 * kGemvRows)), dim3(256), 0, s, n, Ainv,
                     r, d, p0, p1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(int64_t n, T v, T* y, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(nblk(n, 256)), dim3(256), 0, s, n, v, y);
  return hipGetLastError();
}

#define PNS_INST(T)                                                                              \
  template hipError_t launch_ebe_apply<T>(const Grid&, const T*, const T*, const T*, T*, int,   \
                                          int, T*, hipStream_t);                                 \
  template hipError_t launch_patch_sweep<T>(const Grid&, const T*, const T*, T*, double, int,   \
                                            T*, hipStream_t, bool);                              \
  template hipError_t launch_restrict<T>(const Grid&, const Grid&, const T*, T*, hipStream_t);  \
  template hipError_t launch_prolong_add<T>(const Grid&, const Grid&, const T*, T*,             \
                                            hipStream_t);                                        \
  template hipError_t launch_dense_gemv<T>(int64_t, const T*, const T*, T*, const int64_t*,     \
                                           int, hipStream_t);                                    \
  template hipError_t launch_fill<T>(int64_t, T, T*, hipStream_t);                               \
  template hipError_t launch_patch_sweep_c<T>(const Grid&, const T*, const T*, T*, double, int, \
                                              hipStream_t);                                      \
  template hipError_t launch_copy<T>(int64_t, const T*, T*, hipStream_t);
PNS_INST(double)
PNS_INST(float)
#undef PNS_INST

}  // namespace pns
