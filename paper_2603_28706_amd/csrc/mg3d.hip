// Coarse levels of the space-time multigrid on hexahedra (Sec. 6.3), the
// 3D counterparts of the quadrilateral setup and V-cycle kernels:
// * galerkin3d_kernel: coarse space-time element matrices
//   E_C = sum_children P_f^T E_f P_f (A_{l+1} = P^T A_l P restricted cell by
//   cell); the local prolongation is block diagonal (one 27 x 27 Q2
//   interpolation per Radau node and velocity component, one 4 x 4 P1disc
//   restriction per Radau node), so one workgroup forms one block of E_C
//   (row group x column group) over the 8 children;
// * patch3r_kernel: exact patches R_K A_l R_K^T (sums of the element matrices
//   of the cells around the patch: stored Galerkin matrices on coarse levels,
//   or on the finest level K_t (x) M + tau M_t (x) diag(J_1, J_2) formed from
//   the spatial matrices of both Radau nodes), inverted by Gauss-Jordan with
//   partial row pivoting in FP64; the 170 x 170 matrix (231 KB) is larger than
//   the LDS of a CU but fits in the registers of a 1024-thread workgroup, which
//   holds it there (29 entries per thread) and exchanges only the pivot row and
//   column through LDS; the inverse is written in the context precision;
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
    if (i < kNv3 && j < kNv3 && i / kNb3 == j / kNb3)
      v = kKt[mu][nu] * cell_mass3(g, i % kNb3, j % kNb3);
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
// register-resident Gauss-Jordan: 6 threads per row, each holding 29 entries
// (columns part, part + 6, ...) of one row of the 170 x 170 FP64 matrix
constexpr int kRP = 6;
constexpr int kRS = (kNst3 + kRP - 1) / kRP;  // 29
constexpr int kRT = kNst3 * kRP;               // 1020 working threads

// One workgroup of 1024 threads per patch (one colour per launch).  The matrix
// lives in registers (58 VGPRs per thread); each pivot step exchanges only
// column k, rows k and p and the new pivot row through LDS, so a step costs
// five barriers and O(170) LDS traffic.
template <typename T, typename Src>
__global__ __launch_bounds__(1024) void patch3r_kernel(Grid3 g, Src Esrc, T* __restrict__ inv,
                                                       int* status, int px, int py, int pz,
                                                       int ncx, int ncy) {
  __shared__ double colv[kNst3], rowk[kNst3], rowp[kNst3], rowb[kNst3], fk[kNst3];
  __shared__ int piv[kNst3], dst[kNst3], srcc[kNst3];
  __shared__ double s_pv;
  __shared__ int s_p, s_sing;
  const int64_t pid = blockIdx.x;
  const int cx = px + 2 * (int)(pid % ncx);
  const int cy = py + 2 * (int)((pid / ncx) % ncy);
  const int cz = pz + 2 * (int)(pid / ((int64_t)ncx * ncy));
  const int64_t K = cell_index3(g, cx, cy, cz);
  const int cc[3] = {cx, cy, cz}, nc[3] = {g.nx, g.ny, g.nz};
  const int t = threadIdx.x;
  const bool active = t < kRT;
  const int i = t % kNst3, part = t / kNst3;  // row i, columns part + 6 s
  if (t == 0) s_sing = 0;
  double a[kRS];
#pragma unroll
  for (int s = 0; s < kRS; ++s) a[s] = 0.0;
  // assembly: entry (i, j) sums the cells that hold both unknowns (a rolled
  // loop; each value is moved into its register by a select chain)
  const int mr = i / kNs3, sr = i % kNs3;
#pragma unroll 1
  for (int s = 0; s < kRS; ++s) {
    const int j = part + kRP * s;
    double v = 0.0;
    if (active && j < kNst3) {
      const int mc = j / kNs3, sc = j % kNs3;
      if (sr >= kNv3 || sc >= kNv3) {
        v = Esrc(K, i, j);  // the cell's own pressure lives in this cell only
      } else {
        const int ea = sr % kNb3, eb = sc % kNb3;
        const int pa[3] = {ea % 3, (ea / 3) % 3, ea / 9}, pb[3] = {eb % 3, (eb / 3) % 3, eb / 9};
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
          lo[k] = (pa[k] == 0 && pb[k] == 0 && cc[k] > 0) ? -1 : 0;
          hi[k] = (pa[k] == 2 && pb[k] == 2 && cc[k] < nc[k] - 1) ? 1 : 0;
        }
        const int rbase = mr * kNs3 + (sr / kNb3) * kNb3, cbase = mc * kNs3 + (sc / kNb3) * kNb3;
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
          for (int oy = lo[1]; oy <= hi[1]; ++oy)
            for (int ox = lo[0]; ox <= hi[0]; ++ox) {
              const int na = (pa[0] - 2 * ox) + 3 * (pa[1] - 2 * oy) + 9 * (pa[2] - 2 * oz);
              const int nb = (pb[0] - 2 * ox) + 3 * (pb[1] - 2 * oy) + 9 * (pb[2] - 2 * oz);
              v += Esrc(cell_index3(g, cx + ox, cy + oy, cz + oz), rbase + na, cbase + nb);
            }
      }
    }
#pragma unroll
    for (int q = 0; q < kRS; ++q)
      if (q == s) a[q] = v;
  }
  for (int k = 0; k < kNst3; ++k) {
    const int ks = k / kRP, kp = k % kRP;
    // column k to LDS
    if (active && part == kp) {
      double v = 0.0;
#pragma unroll
      for (int s = 0; s < kRS; ++s)
        if (s == ks) v = a[s];
      colv[i] = v;
    }
    __syncthreads();
    // pivot: largest |a_ik| over i >= k (ties to the smaller row)
    if (t < 64) {
      double bv = -1.0;
      int bi = k;
      for (int r = k + t; r < kNst3; r += 64) {
        const double v = fabs(colv[r]);
        if (v > bv) {
          bv = v;
          bi = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (t == 0) {
        s_p = bi;
        piv[k] = bi;
        if (!(bv > 0.0)) {
          s_sing = 1;
          s_pv = 1.0;
        } else {
          s_pv = colv[bi];
        }
      }
    }
    __syncthreads();
    const int p = s_p;
    const double dinv = 1.0 / s_pv;
    // rows k and p as they are
    if (active && (i == k || i == p)) {
#pragma unroll
      for (int s = 0; s < kRS; ++s) {
        const int j = part + kRP * s;
        if (j < kNst3) {
          if (i == k) rowk[j] = a[s];
          if (i == p) rowp[j] = a[s];
        }
      }
    }
    __syncthreads();
    // new row k (old row p scaled, its pivot entry becomes 1 / pivot) and the
    // elimination factors (column k after the interchange, zero on row k)
    if (t < kNst3) {
      rowb[t] = (t == k ? 1.0 : rowp[t]) * dinv;
    } else if (t >= 256 && t < 256 + kNst3) {
      const int r = t - 256;
      fk[r] = r == k ? 0.0 : (r == p ? rowk[k] : colv[r]);
    }
    __syncthreads();
    if (active) {
      if (i == k) {
#pragma unroll
        for (int s = 0; s < kRS; ++s) {
          const int j = part + kRP * s;
          if (j < kNst3) a[s] = rowb[j];
        }
      } else if (i == p) {  // old row k moves to row p (6 threads)
        const double f = fk[i];
#pragma unroll
        for (int s = 0; s < kRS; ++s) {
          const int j = part + kRP * s;
          if (j < kNst3) {
            double v = rowk[j];
            if (j == k) v = 0.0;
            a[s] = v - f * rowb[j];
          }
        }
      } else {  // every other row: only the new pivot row is read from LDS
        const double f = fk[i];
#pragma unroll
        for (int s = 0; s < kRS; ++s) {
          const int j = part + kRP * s;
          if (j < kNst3) {
            double v = a[s];
            if (j == k) v = 0.0;
            a[s] = v - f * rowb[j];
          }
        }
      }
    }
  }
  // the row interchanges become column interchanges of the inverse, applied
  // in reverse order: column dst[j] of the inverse is column j of the result
  if (t == 0) {
    for (int j = 0; j < kNst3; ++j) srcc[j] = j;
    for (int k = kNst3 - 1; k >= 0; --k) {
      const int tmp = srcc[k];
      srcc[k] = srcc[piv[k]];
      srcc[piv[k]] = tmp;
    }
    for (int c = 0; c < kNst3; ++c) dst[srcc[c]] = c;
    if (s_sing) atomicOr(status, 1);
  }
  __syncthreads();
  T* out = inv + patch_slot3(g, cx, cy, cz) * kE3;
  if (active) {
#pragma unroll
    for (int s = 0; s < kRS; ++s) {
      const int j = part + kRP * s;
      if (j < kNst3) out[dst[j] * kNst3 + i] = (T)a[s];
    }
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
    hipLaunchKernelGGL((patch3r_kernel<T, Src>), dim3((unsigned)np), dim3(1024), 0, s, g, src, inv,
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
