// Continuous-interior-penalty stabilisation on the interior faces of a
// quadrilateral mesh (Sec. 3.2, eq. scip-def):
//   s_CIP(uw; x, v) = sum_F gamma h_F^2 int_F |uw . n_F| [grad x n_F] . [grad v n_F] ds,
// [g] = g|_L - g|_R, h_F the cell size normal to F, 3 Gauss points per face.
// Across a vertical face at node column X the jump of the normal derivative
// of a continuous Q2 field is, on each node row of the face's cells, the
// 5-point difference (1, -4, 6, -4, 1) / h_x of the node columns X-2 .. X+2
// (d_x of the left cell's basis at its right end, (1, -4, 3) / h, minus that
// of the right cell at its left end, (-3, 4, -1) / h), interpolated along the
// face with the Q2 basis in y; likewise for horizontal faces.  Two kernels,
// no atomics, fixed summation order:
// * cip_face_kernel: one thread per (face, Radau node) forms, at the 3 face
//   points, G = tau w_mu gamma h_F^2 |uw . n_F| W_q |F| [d_n x] (2 components);
// * cip_node_kernel: one thread per velocity unknown gathers the G of the
//   faces whose 5 x 3 node stencil holds its node, times its own jump
//   coefficient, and adds (action) or subtracts (defect, residual) the sum.
// The multigrid operators carry the same term in factored form (per face a
// 3 x 3 matrix S over its node rows): level-0 S from the lagged velocity,
// coarse S by the Galerkin restriction along the faces, the level action by
// the same face / node kernel pair, and the dense coarsest operator row by
// row.
#include "pns_internal.h"

namespace pns {
namespace {

__device__ __forceinline__ double d4(int o) { return cip_d4(o); }

__device__ __forceinline__ double gp(int q) { return q == 0 ? kGP[0] : (q == 1 ? kGP[1] : kGP[2]); }
__device__ __forceinline__ double gw(int q) { return q == 0 ? kGW[0] : (q == 1 ? kGW[1] : kGW[2]); }

// faces: vertical ones (node column 2 cx, cx = 1 .. nx-1, cell row cy) first,
// f = cy (nx-1) + cx - 1; then horizontal ones (node row 2 cy, cy = 1 .. ny-1,
// cell column cx), f = nV + (cy-1) nx + cx.  G[((f * 2 + mu) * 3 + q) * 2 + c].
template <typename T>
__global__ __launch_bounds__(256) void cip_face_kernel(Grid g, Model m, double tau,
                                                       const T* __restrict__ uw,
                                                       int64_t uw_stride,
                                                       const T* __restrict__ x,
                                                       double* __restrict__ G) {
  const int64_t nV = (int64_t)(g.nx - 1) * g.ny, nH = (int64_t)g.nx * (g.ny - 1);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * (nV + nH)) return;
  const int mu = (int)(id & 1);
  const int64_t f = id >> 1;
  const bool vert = f < nV;
  int cx, cy;
  if (vert) {
    cy = (int)(f / (g.nx - 1));
    cx = (int)(f % (g.nx - 1)) + 1;
  } else {
    cy = (int)((f - nV) / g.nx) + 1;
    cx = (int)((f - nV) % g.nx);
  }
  const int NX = 2 * g.nx + 1;
  const double h = vert ? g.hx : g.hy;      // normal cell size
  const double len = vert ? g.hy : g.hx;    // face length
  const double ih = vert ? g.ihx : g.ihy;
  const T* um = uw + (int64_t)mu * uw_stride + (vert ? 0 : g.nn);  // normal component
  const T* x0 = x + (int64_t)mu * g.ns;
  const T* x1 = x0 + g.nn;
  const double scale = tau * (mu ? kWt[1] : kWt[0]) * m.gamma_cip * h * h * len;
  double out[6];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double un = 0.0, j0 = 0.0, j1 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {   // along the face
      const double phi = q2v(a, gp(q));
      const int64_t base = vert ? (int64_t)(2 * cy + a) * NX + 2 * cx
                                : (int64_t)(2 * cy) * NX + 2 * cx + a;
      un += phi * (double)um[base];
#pragma unroll
      for (int o = -2; o <= 2; ++o) {  // across the face
        const int64_t node = vert ? base + o : base + (int64_t)o * NX;
        const double c = phi * d4(o) * ih;
        j0 += c * (double)x0[node];
        j1 += c * (double)x1[node];
      }
    }
    const double wq = scale * fabs(un) * gw(q);
    out[2 * q] = wq * j0;
    out[2 * q + 1] = wq * j1;
  }
  double* Gf = G + (f * 2 + mu) * 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) Gf[k] = out[k];
}

// NODAL: G holds per face row a the value sum_b S[a][b] j_b (multigrid
// levels) instead of the weighted jumps at the 3 face points
template <typename T, bool NODAL>
__global__ __launch_bounds__(256) void cip_node_kernel(Grid g, const double* __restrict__ G,
                                                       T* __restrict__ y, double sign) {
  const int64_t nV = (int64_t)(g.nx - 1) * g.ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 4 * g.nn) return;
  const int mu = (int)(id / (2 * g.nn));
  const int c = (int)((id / g.nn) & 1);
  const int64_t node = id % g.nn;
  const int NX = 2 * g.nx + 1;
  const int gx = (int)(node % NX), gy = (int)(node / NX);
  double acc = 0.0;
  // vertical faces: node columns X = 2 cx within 2 of gx, cell rows holding gy
  for (int X = ((gx - 2) + 1) / 2 * 2; X <= gx + 2; X += 2) {
    const int cx = X / 2;
    if (X < gx - 2 || cx < 1 || cx > g.nx - 1) continue;
    const double cf = d4(gx - X) * g.ihx;
    for (int cy = gy / 2 - 1; cy <= gy / 2; ++cy) {
      if (cy < 0 || cy >= g.ny) continue;
      const int a = gy - 2 * cy;
      if (a > 2) continue;
      const int64_t f = (int64_t)cy * (g.nx - 1) + cx - 1;
      const double* Gf = G + (f * 2 + mu) * 6;
      if (NODAL) {
        acc += Gf[2 * a + c] * cf;
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += Gf[2 * q + c] * cf * q2v(a, gp(q));
      }
    }
  }
  // horizontal faces: node rows Y = 2 cy within 2 of gy, cell columns holding gx
  for (int Y = ((gy - 2) + 1) / 2 * 2; Y <= gy + 2; Y += 2) {
    const int cy = Y / 2;
    if (Y < gy - 2 || cy < 1 || cy > g.ny - 1) continue;
    const double cf = d4(gy - Y) * g.ihy;
    for (int cx = gx / 2 - 1; cx <= gx / 2; ++cx) {
      if (cx < 0 || cx >= g.nx) continue;
      const int a = gx - 2 * cx;
      if (a > 2) continue;
      const int64_t f = nV + (int64_t)(cy - 1) * g.nx + cx;
      const double* Gf = G + (f * 2 + mu) * 6;
      if (NODAL) {
        acc += Gf[2 * a + c] * cf;
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += Gf[2 * q + c] * cf * q2v(a, gp(q));
      }
    }
  }
  const int64_t idx = (int64_t)mu * g.ns + (int64_t)c * g.nn + node;
  y[idx] = (T)((double)y[idx] + sign * acc);
}


// face f of the numbering above: vertical or not, its node column (row) X and
// the cell row (column) it spans
struct FaceAt {
  bool vert;
  int cx, cy;
};

__device__ __forceinline__ FaceAt face_at(const Grid& g, int64_t f) {
  const int64_t nV = (int64_t)(g.nx - 1) * g.ny;
  FaceAt F;
  F.vert = f < nV;
  if (F.vert) {
    F.cy = (int)(f / (g.nx - 1));
    F.cx = (int)(f % (g.nx - 1)) + 1;
  } else {
    F.cy = (int)((f - nV) / g.nx) + 1;
    F.cx = (int)((f - nV) % g.nx);
  }
  return F;
}

// S_mu[a][b] = scale_mu gamma h^2 |F| sum_q w_q |uw_mu . n_F| phi_a phi_b, one
// thread per (face, Radau node)
__global__ __launch_bounds__(256) void cip_face_matrix_kernel(Grid g, Model m,
                                                              const double* __restrict__ uw,
                                                              int64_t uw_stride, int nm,
                                                              double scale0, double scale1,
                                                              double* __restrict__ S) {
  const int64_t nf = (int64_t)(g.nx - 1) * g.ny + (int64_t)g.nx * (g.ny - 1);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nm * nf) return;
  const int mu = (int)(id % nm);
  const int64_t f = id / nm;
  const FaceAt F = face_at(g, f);
  const int NX = 2 * g.nx + 1;
  const double h = F.vert ? g.hx : g.hy, len = F.vert ? g.hy : g.hx;
  const double* um = uw + (int64_t)mu * uw_stride + (F.vert ? 0 : g.nn);  // normal component
  const double scale = (mu ? scale1 : scale0) * m.gamma_cip * h * h * len;
  double out[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) out[k] = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double phi[3], un = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      phi[a] = q2v(a, gp(q));
      const int64_t node = F.vert ? (int64_t)(2 * F.cy + a) * NX + 2 * F.cx
                                  : (int64_t)(2 * F.cy) * NX + 2 * F.cx + a;
      un += phi[a] * um[node];
    }
    const double wq = scale * gw(q) * fabs(un);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) out[3 * a + b] += wq * phi[a] * phi[b];
  }
  double* Sf = S + (f * nm + mu) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) Sf[k] = out[k];
}

// coarse S = sum over the two fine faces on the coarse face of Py^T S_f Py,
// Py[i][a] = phi_a((2 child + i) / 4); one thread per (coarse face, Radau node)
__global__ __launch_bounds__(256) void cip_restrict_kernel(Grid gc, Grid gf,
                                                           const double* __restrict__ Sf,
                                                           double* __restrict__ Sc) {
  const int64_t nf = (int64_t)(gc.nx - 1) * gc.ny + (int64_t)gc.nx * (gc.ny - 1);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * nf) return;
  const int mu = (int)(id & 1);
  const int64_t f = id >> 1;
  const FaceAt F = face_at(gc, f);
  const int64_t nVf = (int64_t)(gf.nx - 1) * gf.ny;
  double out[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) out[k] = 0.0;
  for (int ch = 0; ch < 2; ++ch) {
    const int64_t ff = F.vert ? (int64_t)(2 * F.cy + ch) * (gf.nx - 1) + 2 * F.cx - 1
                              : nVf + (int64_t)(2 * F.cy - 1) * gf.nx + 2 * F.cx + ch;
    const double* s = Sf + (ff * 2 + mu) * 9;
    double P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) P[i][a] = q2v(a, 0.25 * (2 * ch + i));
    double T[3][3];  // S_f Py
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        T[i][b] = s[3 * i] * P[0][b] + s[3 * i + 1] * P[1][b] + s[3 * i + 2] * P[2][b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        out[3 * a + b] += P[0][a] * T[0][b] + P[1][a] * T[1][b] + P[2][a] * T[2][b];
  }
  double* o = Sc + (f * 2 + mu) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) o[k] = out[k];
}

// G[((f * 2 + mu) * 3 + a) * 2 + c] = sum_b S[a][b] j_b(x_mu,c), one thread per
// (face, Radau node)
template <typename T>
__global__ __launch_bounds__(256) void cip_level_face_kernel(Grid g, const double* __restrict__ S,
                                                             const T* __restrict__ x,
                                                             double* __restrict__ G) {
  const int64_t nf = (int64_t)(g.nx - 1) * g.ny + (int64_t)g.nx * (g.ny - 1);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * nf) return;
  const int mu = (int)(id & 1);
  const int64_t f = id >> 1;
  const FaceAt F = face_at(g, f);
  const int NX = 2 * g.nx + 1;
  const double ih = F.vert ? g.ihx : g.ihy;
  const T* x0 = x + (int64_t)mu * g.ns;
  const T* x1 = x0 + g.nn;
  double j0[3], j1[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int64_t base = F.vert ? (int64_t)(2 * F.cy + b) * NX + 2 * F.cx
                                : (int64_t)(2 * F.cy) * NX + 2 * F.cx + b;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      const int64_t node = F.vert ? base + o : base + (int64_t)o * NX;
      s0 += d4(o) * (double)x0[node];
      s1 += d4(o) * (double)x1[node];
    }
    j0[b] = ih * s0;
    j1[b] = ih * s1;
  }
  const double* s = S + (f * 2 + mu) * 9;
  double* Gf = G + (f * 2 + mu) * 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Gf[2 * a] = s[3 * a] * j0[0] + s[3 * a + 1] * j0[1] + s[3 * a + 2] * j0[2];
    Gf[2 * a + 1] = s[3 * a] * j1[0] + s[3 * a + 1] * j1[1] + s[3 * a + 2] * j1[2];
  }
}

// rows of the dense operator: one thread per velocity row (Radau node,
// component, node) adds ih^2 d4(o_row) d4(o_col) S[a_row][b_col] for every face
// whose stencil holds the row's node, over the 15 nodes of that stencil
__global__ __launch_bounds__(256) void cip_dense_kernel(Grid g, const double* __restrict__ S,
                                                        double* __restrict__ A) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 4 * g.nn) return;
  const int mu = (int)(id / (2 * g.nn));
  const int c = (int)((id / g.nn) & 1);
  const int64_t node = id % g.nn;
  const int NX = 2 * g.nx + 1;
  const int gx = (int)(node % NX), gy = (int)(node / NX);
  const int64_t nV = (int64_t)(g.nx - 1) * g.ny;
  const int64_t n = g.nst;
  const int64_t off = (int64_t)mu * g.ns + (int64_t)c * g.nn;
  double* row = A + (off + node) * n + off;
  for (int X = ((gx - 2) + 1) / 2 * 2; X <= gx + 2; X += 2) {
    const int cx = X / 2;
    if (X < gx - 2 || cx < 1 || cx > g.nx - 1) continue;
    const double cf = d4(gx - X) * g.ihx * g.ihx;
    for (int cy = gy / 2 - 1; cy <= gy / 2; ++cy) {
      if (cy < 0 || cy >= g.ny) continue;
      const int a = gy - 2 * cy;
      if (a > 2) continue;
      const double* s = S + (((int64_t)cy * (g.nx - 1) + cx - 1) * 2 + mu) * 9 + 3 * a;
      for (int b = 0; b < 3; ++b)
        for (int o = -2; o <= 2; ++o)
          row[(int64_t)(2 * cy + b) * NX + X + o] += cf * d4(o) * s[b];
    }
  }
  for (int Y = ((gy - 2) + 1) / 2 * 2; Y <= gy + 2; Y += 2) {
    const int cy = Y / 2;
    if (Y < gy - 2 || cy < 1 || cy > g.ny - 1) continue;
    const double cf = d4(gy - Y) * g.ihy * g.ihy;
    for (int cx = gx / 2 - 1; cx <= gx / 2; ++cx) {
      if (cx < 0 || cx >= g.nx) continue;
      const int a = gx - 2 * cx;
      if (a > 2) continue;
      const double* s = S + ((nV + (int64_t)(cy - 1) * g.nx + cx) * 2 + mu) * 9 + 3 * a;
      for (int b = 0; b < 3; ++b)
        for (int o = -2; o <= 2; ++o)
          row[(int64_t)(Y + o) * NX + 2 * cx + b] += cf * d4(o) * s[b];
    }
  }
}

}  // namespace

int64_t cip_face_doubles(const Grid& g) {
  return 12 * ((int64_t)(g.nx - 1) * g.ny + (int64_t)g.nx * (g.ny - 1));
}

template <typename T>
hipError_t launch_cip(const Grid& g, const Model& m, double tau, const T* uw, int64_t uw_stride,
                      const T* x, T* y, double sign, double* G, hipStream_t s) {
  const int64_t nf = (int64_t)(g.nx - 1) * g.ny + (int64_t)g.nx * (g.ny - 1);
  if (nf > 0) {
    hipLaunchKernelGGL((cip_face_kernel<T>), dim3((unsigned)((2 * nf + 255) / 256)), dim3(256), 0,
                       s, g, m, tau, uw, uw_stride, x, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((cip_node_kernel<T, false>), dim3((unsigned)((4 * g.nn + 255) / 256)),
                     dim3(256), 0, s, g, (const double*)G, y, sign);
  return hipGetLastError();
}

int64_t cip_face_count(const Grid& g) {
  return (int64_t)(g.nx - 1) * g.ny + (int64_t)g.nx * (g.ny - 1);
}

hipError_t launch_cip_face_matrices(const Grid& g, const Model& m, const double* uw,
                                    int64_t uw_stride, int nm, double scale0, double scale1,
                                    double* S, hipStream_t s) {
  const int64_t n = nm * cip_face_count(g);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cip_face_matrix_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                     m, uw, uw_stride, nm, scale0, scale1, S);
  return hipGetLastError();
}

hipError_t launch_cip_restrict(const Grid& gc, const Grid& gf, const double* Sf, double* Sc,
                               hipStream_t s) {
  const int64_t n = 2 * cip_face_count(gc);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cip_restrict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gc,
                     gf, Sf, Sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cip_level(const Grid& g, const double* S, const T* x, T* y, double sign,
                            double* G, hipStream_t s) {
  const int64_t nf = cip_face_count(g);
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL((cip_level_face_kernel<T>), dim3((unsigned)((2 * nf + 255) / 256)), dim3(256),
                     0, s, g, S, x, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((cip_node_kernel<T, true>), dim3((unsigned)((4 * g.nn + 255) / 256)),
                     dim3(256), 0, s, g, (const double*)G, y, sign);
  return hipGetLastError();
}

hipError_t launch_cip_dense(const Grid& g, const double* S, double* A, hipStream_t s) {
  if (cip_face_count(g) == 0) return hipSuccess;
  hipLaunchKernelGGL(cip_dense_kernel, dim3((unsigned)((4 * g.nn + 255) / 256)), dim3(256), 0, s, g,
                     S, A);
  return hipGetLastError();
}

template hipError_t launch_cip<double>(const Grid&, const Model&, double, const double*, int64_t,
                                       const double*, double*, double, double*, hipStream_t);
template hipError_t launch_cip<float>(const Grid&, const Model&, double, const float*, int64_t,
                                      const float*, float*, double, double*, hipStream_t);

template hipError_t launch_cip_level<double>(const Grid&, const double*, const double*, double*,
                                             double, double*, hipStream_t);
template hipError_t launch_cip_level<float>(const Grid&, const double*, const float*, float*,
                                            double, double*, hipStream_t);

}  // namespace pns
