// Vector kernels of the slab solve (Sec. 6.1): the block mass of the time step
// (the inner product in which residuals are measured), deterministic multi-dot
// products and combinations of Krylov vectors, precision conversions.  All
// reductions use a fixed partition and a fixed summation tree, so results do
// not depend on scheduling.
#include "pns_internal.h"

namespace pns {
namespace {

constexpr int kBlock = 256;
constexpr int kDotBlocks = 1024;  // partial sums per vector
constexpr int kGroup = 8;         // vectors handled per pass over the shared operand

// entry (i, k) of the 1D Q2 mass matrix on nodes 0..N-1 (spacing h/2, cells of
// length h): per cell h/30 [[4, 2, -1], [2, 16, 2], [-1, 2, 4]]
__device__ __forceinline__ double mass1d(int i, int k, int N, double h) {
  const int d = k - i;
  if (k < 0 || k >= N || d < -2 || d > 2) return 0.0;
  if (i & 1) return d == 0 ? 16.0 * h / 30.0 : (d == 1 || d == -1 ? 2.0 * h / 30.0 : 0.0);
  if (d == 0) return (i == 0 || i == N - 1 ? 4.0 : 8.0) * h / 30.0;
  return (d == 1 || d == -1) ? 2.0 * h / 30.0 : -h / 30.0;
}

// y = M x with M = tau M_t (x) blockdiag(M_x per velocity component, M_p):
// Q2 mass = 1D mass (x) 1D mass (uniform tensor grid), P1disc mass per cell
// |K| diag(1, 1/12, 1/12)
__global__ __launch_bounds__(kBlock) void mass_kernel(Grid g, double tau, const double* __restrict__ x,
                                                      double* __restrict__ y) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nst) return;
  const int mu = (int)(id / g.ns);
  const int64_t r = id - (int64_t)mu * g.ns;
  const double tw = tau * (mu ? kWt[1] : kWt[0]);
  if (r >= g.nv) {
    const int j = (int)((r - g.nv) % 3);
    y[id] = tw * g.hx * g.hy * (j == 0 ? 1.0 : 1.0 / 12.0) * x[id];
    return;
  }
  const int NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  const int64_t node = r % g.nn;
  const int gx = (int)(node % NX), gy = (int)(node / NX);
  const double* xb = x + (id - node);
  double s = 0.0;
#pragma unroll
  for (int dy = -2; dy <= 2; ++dy) {
    const double my = mass1d(gy, gy + dy, NY, g.hy);
    if (my == 0.0) continue;
    double t = 0.0;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      const double mx = mass1d(gx, gx + dx, NX, g.hx);
      if (mx != 0.0) t += mx * xb[(int64_t)(gy + dy) * NX + gx + dx];
    }
    s += my * t;
  }
  y[id] = tw * s;
}

// Hexahedra: y_mu = c_mu (M_x x_v,mu ; pscale M_p x_p,mu), Q2 mass = tensor
// product of three 1D masses, P1disc mass per cell |K| diag(1, 1/12, 1/12, 1/12).
// c_mu = tau w_mu, pscale = 1 gives the block mass of the time step; c = m_t,
// pscale = 0 the left-trace coupling of the residual.
__global__ __launch_bounds__(kBlock) void mass3_kernel(Grid3 g, double c0, double c1, double pscale,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nst) return;
  const int mu = (int)(id / g.ns);
  const int64_t r = id - (int64_t)mu * g.ns;
  const double cw = mu ? c1 : c0;
  if (r >= g.nv) {
    const int j = (int)((r - g.nv) % 4);
    y[id] = cw * pscale * g.hx * g.hy * g.hz * (j == 0 ? 1.0 : 1.0 / 12.0) * x[id];
    return;
  }
  const int NX = 2 * g.nx + 1, NY = 2 * g.ny + 1, NZ = 2 * g.nz + 1;
  const int64_t node = r % g.nn;
  const int gx = (int)(node % NX), gy = (int)((node / NX) % NY), gz = (int)(node / ((int64_t)NX * NY));
  const double* xb = x + (id - node);
  double s = 0.0;
  for (int dz = -2; dz <= 2; ++dz) {
    const double mz = mass1d(gz, gz + dz, NZ, g.hz);
    if (mz == 0.0) continue;
    double sy = 0.0;
    for (int dy = -2; dy <= 2; ++dy) {
      const double my = mass1d(gy, gy + dy, NY, g.hy);
      if (my == 0.0) continue;
      double t = 0.0;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        const double mx = mass1d(gx, gx + dx, NX, g.hx);
        if (mx != 0.0) t += mx * xb[((int64_t)(gz + dz) * NY + gy + dy) * NX + gx + dx];
      }
      sy += my * t;
    }
    s += mz * sy;
  }
  y[id] = cw * s;
}

// partial[i * kDotBlocks + b] = sum over block b's chunk of V_i . u, i < k
__global__ __launch_bounds__(kBlock) void multi_dot_kernel(int64_t n, int k, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ u,
                                                           double* __restrict__ partial) {
  __shared__ double red[kGroup][kBlock / 64];
  const int64_t chunk = (n + kDotBlocks - 1) / kDotBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  for (int i0 = 0; i0 < k; i0 += kGroup) {
    double s[kGroup];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) s[j] = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBlock) {
      const double ut = u[t];
#pragma unroll
      for (int j = 0; j < kGroup; ++j)
        if (i0 + j < k) s[j] += V[(int64_t)(i0 + j) * ldv + t] * ut;
    }
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
      double v = s[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < kGroup && i0 + (int)threadIdx.x < k) {
      const int j = threadIdx.x;
      partial[(int64_t)(i0 + j) * kDotBlocks + blockIdx.x] =
          (red[j][0] + red[j][1]) + (red[j][2] + red[j][3]);
    }
    __syncthreads();
  }
}

// out[i] = sum_b partial[i * kDotBlocks + b], one block per i, fixed tree
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(const double* __restrict__ partial,
                                                                 double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  const double* p = partial + (int64_t)blockIdx.x * kDotBlocks;
  double v = 0.0;
  for (int b = threadIdx.x; b < kDotBlocks; b += kBlock) v += p[b];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w = alpha w + sgn sum_{i<k} c[i] V_i   (c on the device)
__global__ __launch_bounds__(kBlock) void lincomb_kernel(int64_t n, int k, const double* __restrict__ V,
                                                         int64_t ldv, const double* __restrict__ c,
                                                         double sgn, double alpha,
                                                         double* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += c[i] * V[(int64_t)i * ldv + t];
  w[t] = (alpha == 0.0 ? 0.0 : alpha * w[t]) + sgn * s;
}

// z = a x + b y
__global__ __launch_bounds__(kBlock) void axpby_kernel(int64_t n, double a, const double* __restrict__ x,
                                                       double b, const double* __restrict__ y,
                                                       double* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) z[t] = a * x[t] + (b == 0.0 ? 0.0 : b * y[t]);
}

__global__ __launch_bounds__(kBlock) void widen_kernel(int64_t n, const float* __restrict__ x,
                                                       double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] = (double)x[t];
}

__global__ __launch_bounds__(kBlock) void narrow_kernel(int64_t n, const double* __restrict__ x,
                                                        float* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] = (float)x[t];
}

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

int dot_partials() { return kDotBlocks; }

hipError_t launch_mass(const Grid& g, double tau, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(mass_kernel, grid_for(g.nst), dim3(kBlock), 0, s, g, tau, x, y);
  return hipGetLastError();
}

hipError_t launch_mass3(const Grid3& g, double c0, double c1, double pscale, const double* x,
                        double* y, hipStream_t s) {
  hipLaunchKernelGGL(mass3_kernel, grid_for(g.nst), dim3(kBlock), 0, s, g, c0, c1, pscale, x, y);
  return hipGetLastError();
}

hipError_t launch_multi_dot(int64_t n, int k, const double* V, int64_t ldv, const double* u,
                            double* partial, double* out, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, s, n, k, V, ldv, u,
                     partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(k), dim3(kBlock), 0, s, partial, out);
  return hipGetLastError();
}

hipError_t launch_combine(int64_t n, int k, const double* V, int64_t ldv, const double* c,
                          double sgn, double alpha, double* w, hipStream_t s) {
  hipLaunchKernelGGL(lincomb_kernel, grid_for(n), dim3(kBlock), 0, s, n, k, V, ldv, c, sgn, alpha,
                     w);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, grid_for(n), dim3(kBlock), 0, s, n, a, x, b, y, z);
  return hipGetLastError();
}

hipError_t launch_widen(int64_t n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(widen_kernel, grid_for(n), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t launch_narrow(int64_t n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(narrow_kernel, grid_for(n), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError();
}

}  // namespace pns
