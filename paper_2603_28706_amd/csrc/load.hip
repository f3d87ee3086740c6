// Volume-force right-hand side of the slab (the f-term of eq. disc-residual
// under the Radau rule of eq. slab-underint):
//   F_v,mu[node, comp] = tau w_mu sum_{cells K at the node} sum_q W_q |K| f_mu(x_q)_comp phi_node(x_q),
//   F_p = 0,
// from f given at the 3^d Gauss points of every cell.  One thread per
// (Radau node, component, mesh node) gathers over the <= 2^d cells around its
// node in a fixed order (deterministic, no atomics).
#include "pns_internal.h"

namespace pns {
namespace {

// f_qp[((mu * cells + cell) * 3^d + q) * d + comp], q = qx + 3 qy (+ 9 qz)
__global__ void load2_kernel(Grid g, double tau, const double* __restrict__ f,
                             double* __restrict__ F) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = 2 * g.nn;  // (comp, node) per Radau node
  if (id >= 2 * per) return;
  const int mu = (int)(id / per);
  const int comp = (int)((id % per) / g.nn);
  const int64_t node = id % g.nn;
  const int NX = 2 * g.nx + 1;
  const int gx = (int)(node % NX), gy = (int)(node / NX);
  const double area = g.hx * g.hy;
  double acc = 0.0;
  for (int cy = (gy >> 1) - 1; cy <= (gy >> 1); ++cy) {
    if (cy < 0 || cy >= g.ny) continue;
    const int ay = gy - 2 * cy;
    if (ay > 2) continue;
    for (int cx = (gx >> 1) - 1; cx <= (gx >> 1); ++cx) {
      if (cx < 0 || cx >= g.nx) continue;
      const int ax = gx - 2 * cx;
      if (ax > 2) continue;
      const int64_t cell = (int64_t)cy * g.nx + cx;
      const double* fc = f + ((int64_t)mu * g.nc + cell) * 9 * 2;
      for (int qy = 0; qy < 3; ++qy)
        for (int qx = 0; qx < 3; ++qx) {
          const double w = kGW[qx] * kGW[qy] * q2v(ax, kGP[qx]) * q2v(ay, kGP[qy]);
          acc += w * fc[(qy * 3 + qx) * 2 + comp];
        }
    }
  }
  F[(int64_t)mu * g.ns + (int64_t)comp * g.nn + node] = tau * kWt[mu] * area * acc;
}

__global__ void load3_kernel(Grid3 g, double tau, const double* __restrict__ f,
                             double* __restrict__ F) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = 3 * g.nn;
  if (id >= 2 * per) return;
  const int mu = (int)(id / per);
  const int comp = (int)((id % per) / g.nn);
  const int64_t node = id % g.nn;
  const int64_t NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
  const int gx = (int)(node % NX), gy = (int)((node / NX) % NY), gz = (int)(node / (NX * NY));
  const double vol = g.hx * g.hy * g.hz;
  double acc = 0.0;
  for (int cz = (gz >> 1) - 1; cz <= (gz >> 1); ++cz) {
    if (cz < 0 || cz >= g.nz) continue;
    const int az = gz - 2 * cz;
    if (az > 2) continue;
    for (int cy = (gy >> 1) - 1; cy <= (gy >> 1); ++cy) {
      if (cy < 0 || cy >= g.ny) continue;
      const int ay = gy - 2 * cy;
      if (ay > 2) continue;
      for (int cx = (gx >> 1) - 1; cx <= (gx >> 1); ++cx) {
        if (cx < 0 || cx >= g.nx) continue;
        const int ax = gx - 2 * cx;
        if (ax > 2) continue;
        const int64_t cell = ((int64_t)cz * g.ny + cy) * g.nx + cx;
        const double* fc = f + ((int64_t)mu * g.nc + cell) * 27 * 3;
        for (int qz = 0; qz < 3; ++qz)
          for (int qy = 0; qy < 3; ++qy)
            for (int qx = 0; qx < 3; ++qx) {
              const double w = kGW[qx] * kGW[qy] * kGW[qz] * q2v(ax, kGP[qx]) *
                                q2v(ay, kGP[qy]) * q2v(az, kGP[qz]);
              acc += w * fc[((qz * 3 + qy) * 3 + qx) * 3 + comp];
            }
      }
    }
  }
  F[(int64_t)mu * g.ns + (int64_t)comp * g.nn + node] = tau * kWt[mu] * vol * acc;
}

__global__ void add_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

}  // namespace

hipError_t launch_add(int64_t n, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t launch_load2(const Grid& g, double tau, const double* f_qp, double* F,
                        hipStream_t s) {
  hipError_t e = launch_fill<double>(g.nst, 0.0, F, s);
  if (e != hipSuccess) return e;
  const int64_t n = 4 * g.nn;
  hipLaunchKernelGGL(load2_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, tau,
                     f_qp, F);
  return hipGetLastError();
}

hipError_t launch_load3(const Grid3& g, double tau, const double* f_qp, double* F,
                        hipStream_t s) {
  hipError_t e = launch_fill<double>(g.nst, 0.0, F, s);
  if (e != hipSuccess) return e;
  const int64_t n = 6 * g.nn;
  hipLaunchKernelGGL(load3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, tau,
                     f_qp, F);
  return hipGetLastError();
}

}  // namespace pns
