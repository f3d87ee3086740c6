// Internal declarations of the MI355X smoothing-step library: context layout,
// device-side constants of the Q2 / P1disc x dG(1) element, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pnsmg.h"

namespace pns {

// ---------------------------------------------------------------- element
// Reference cell [0,1]^2; Q2 Lagrange basis on the nodes {0, 1/2, 1} per
// direction; 3-point Gauss-Legendre rule per direction on cells and faces.
constexpr double kGaussR = 0.38729833462074168852;  // sqrt(3/5) / 2
constexpr double kGP[3] = {0.5 - kGaussR, 0.5, 0.5 + kGaussR};
constexpr double kGW[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

__host__ __device__ constexpr double q2v(int a, double s) {
  return a == 0 ? 2.0 * (s - 0.5) * (s - 1.0) : (a == 1 ? -4.0 * s * (s - 1.0) : 2.0 * s * (s - 0.5));
}
__host__ __device__ constexpr double q2d(int a, double s) {
  return a == 0 ? 4.0 * s - 3.0 : (a == 1 ? -8.0 * s + 4.0 : 4.0 * s - 1.0);
}

// local spatial unknowns of a cell: velocity comp c at node a -> c*9 + a,
// pressure coefficient j -> 18 + j; space-time local index = mu*21 + spatial.
constexpr int kNb = 9;
constexpr int kNs = 21;
constexpr int kNst = 42;

// dG(1) on right Radau nodes {1/3, 1}: reference K_t (row = test), weights.
constexpr double kKt[2][2] = {{9.0 / 8.0, 3.0 / 8.0}, {-9.0 / 8.0, 5.0 / 8.0}};
constexpr double kWt[2] = {0.75, 0.25};
// Lagrange basis of the Radau nodes at the slab midpoint t = 1/2.
constexpr double kXiMid[2] = {0.75, 0.25};

// Time-diagonal form of patches K_t (x) M + tau M_t (x) J (level-0 surrogate
// patches): M_t^{-1} K_t = V diag(lam, conj(lam)) V^{-1} with lam = 2 + i sqrt2,
// V = [[1, 1], [1 + 2 sqrt2 i, 1 - 2 sqrt2 i]].  For a real right-hand side
// (r0, r1) the solution is d0 = 2 Re y, d1 = 2 (Re y - 2 sqrt2 Im y) with
// (lam M + tau J) y = z, z = (2/3 + i/(3 sqrt2)) r0 - (i/sqrt2) r1.
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kLamRe = 2.0, kLamIm = kSqrt2;
constexpr double kZr0 = 2.0 / 3.0, kZi0 = 1.0 / (3.0 * kSqrt2), kZi1 = -1.0 / kSqrt2;
constexpr double kBackIm = 2.0 * kSqrt2;

// ---------------------------------------------------------------- model
struct Model {
  double p, delta2, nu, nu_inf, expo;  // expo = (p-2)/2
  double sigma_max, etaD, gamma1, gamma2, qsign;
  double gamma_cip;  // CIP weight (0: off)
  int lin, convection;
  // Dirichlet data of the level-0 mesh as a table over its boundary face points
  // (launch_lift_table), or nullptr for homogeneous data (eq. def-b-gam)
  const double* lift;
  // 2D action and residual: sum the cell contributions of a tile in a fixed
  // order (bitwise reproducible) instead of with LDS atomics
  int ordered;
};

// LDS accumulation: atomic, or a plain add where the caller orders the adds
template <bool ATOMIC>
__device__ __forceinline__ void lds_add(double* p, double v) {
  if (ATOMIC)
    atomicAdd(p, v);
  else
    *p += v;
}

struct Grid {
  int nx, ny;
  double hx, hy, ihx, ihy;
  int64_t nn, nc, nv, ns, nst;  // nodes, cells, velocity, spatial, space-time
};

// Frozen Nitsche coefficients of eq. def-b-gam at G = D ghat_D: eta(G) and the
// coefficient k of the exact stress derivative DS(G)B = eta(G) B + k (G:B) G,
// k = (p-2) nu (delta^2 + |G|^2)^((p-4)/2); for G = 0, eta_D and 0.
__host__ __device__ inline void frozen_coef(const Model& m, double g00, double g01, double g11,
                                            double& eta, double& k) {
  const double D2 = m.delta2 + g00 * g00 + 2.0 * g01 * g01 + g11 * g11;
  const double mu = m.nu * pow(D2, m.expo);
  eta = m.nu_inf + mu;
  k = (m.p - 2.0) * mu / D2;
}

// Dirichlet data at the boundary face points of the 2D level-0 mesh: per
// point (side 0: x = lo, 1: x = hi, 2: y = lo, 3: y = hi; cell j along the
// side; Gauss point q) and time slot s (0, 1: the Radau nodes, 2: the slab
// midpoint t_rep), kLiftVals values: the lifting's value (g0, g1), its
// symmetric gradient G (G00, G01, G11) and the frozen coefficients eta(G),
// k(G) of frozen_coef.
constexpr int kLiftVals = 7;
__host__ __device__ inline int64_t lift_index(const Grid& g, int side, int j, int q, int s) {
  const int L = g.nx > g.ny ? g.nx : g.ny;
  return ((((int64_t)side * L + j) * 3 + q) * 3 + s) * kLiftVals;
}
inline int64_t lift_table_doubles(const Grid& g) {
  return lift_index(g, 4, 0, 0, 0);
}

inline Grid make_grid(int nx, int ny, double lx, double ly) {
  Grid g;
  g.nx = nx;
  g.ny = ny;
  g.hx = lx / nx;
  g.hy = ly / ny;
  g.ihx = nx / lx;
  g.ihy = ny / ly;
  g.nn = (int64_t)(2 * nx + 1) * (2 * ny + 1);
  g.nc = (int64_t)nx * ny;
  g.nv = 2 * g.nn;
  g.ns = g.nv + 3 * g.nc;
  g.nst = 2 * g.ns;
  return g;
}

// Storage position of the patch inverse of cell (cx, cy): colour-major (colour
// = parity class of (cx, cy), in the order (0,0), (1,0), (0,1), (1,1)), within a
// colour the cells of that class row by row, so that each of the four colour
// passes of a sweep streams one contiguous block of inverses.
__host__ __device__ inline int64_t patch_slot(const Grid& g, int cx, int cy) {
  const int px = cx & 1, py = cy & 1, c = px + 2 * py;
  const int64_t ncx0 = (g.nx + 1) / 2, ncx1 = g.nx / 2, ncy0 = (g.ny + 1) / 2;
  int64_t off = 0;
  if (c >= 1) off += ncx0 * ncy0;
  if (c >= 2) off += ncx1 * ncy0;
  if (c >= 3) off += ncx0 * (g.ny / 2);
  return off + (int64_t)(cy >> 1) * (px ? ncx1 : ncx0) + (cx >> 1);
}

// 3D box of hexahedra (x fastest); nodes (2nx+1)(2ny+1)(2nz+1), P1disc pressure
// with 4 coefficients per cell
struct Grid3 {
  int nx, ny, nz;
  double hx, hy, hz, ihx, ihy, ihz;
  int64_t nn, nc, nv, ns, nst;
};

inline Grid3 make_grid3(int nx, int ny, int nz, double lx, double ly, double lz) {
  Grid3 g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.hx = lx / nx;
  g.hy = ly / ny;
  g.hz = lz / nz;
  g.ihx = nx / lx;
  g.ihy = ny / ly;
  g.ihz = nz / lz;
  g.nn = (int64_t)(2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1);
  g.nc = (int64_t)nx * ny * nz;
  g.nv = 3 * g.nn;
  g.ns = g.nv + 4 * g.nc;
  g.nst = 2 * g.ns;
  return g;
}

// ---------------------------------------------------------------- launchers
// apply.hip: matrix-free level-0 operator; mode 0: y = J x, mode 1: y = b - J x;
// cache == nullptr: tangent recomputed from u_k at every point, else the
// per-point coefficients written by launch_tangent_cache are read
template <typename T>
hipError_t launch_cell_apply(const Grid& g, const Model& m, double tau, const T* uk, const T* cache,
                             const T* x, const T* b, T* y, double* edge, int mode,
                             hipStream_t s);
// doubles of the edge buffer of launch_cell_apply (per tile without halo:
// 4 fields x 96 perimeter nodes of partial sums)
int64_t cell_apply_edge_doubles(const Grid& g);
template <typename T>
hipError_t launch_tangent_cache(const Grid& g, const Model& m, double tau, const double* uk,
                                T* cache, hipStream_t s);

// apply3d.hip: the same operator on hexahedra; mode 0: y = J x, mode 1: y = b - J x;
// E: per-cell results, nc * 170 values of scratch
template <typename T>
hipError_t launch_cell_apply3d(const Grid3& g, const Model& m, double tau, const T* uk,
                               const T* x, const T* b, T* y, T* E, int mode, hipStream_t s);

// the same action with x and u_k stored in BF16 (uint16_t bit patterns),
// computed in FP32 (tangent scalars FP64), y and b in FP32
hipError_t launch_cell_apply3d_bf16(const Grid3& g, const Model& m, double tau, const uint16_t* uk,
                                    const uint16_t* x, const float* b, float* y, float* E,
                                    int mode, hipStream_t s);
// FP64 -> BF16 (round to nearest even through FP32)
hipError_t launch_to_bf16(int64_t n, const double* in, uint16_t* out, hipStream_t s);

// y[node, cell rows] = sum of the per-cell slots (170 per cell, layout of the
// 3D action) of the cells sharing each unknown, fixed order; b != nullptr:
// y = b - sum
template <typename T>
hipError_t launch_gather3(const Grid3& g, const T* E, const T* b, T* y, hipStream_t s);

// smooth3d.hip: finest-level Vanka smoother on hexahedra (surrogate patches in
// time-diagonal form).  Es: nc * 85 * 85 FP64 spatial cell matrices at the
// state u; inv: nc complex 85 x 85 inverses (2 * 85 * 85 values per patch,
// colour-major patch order); status bit 0 set on a zero pivot.
hipError_t launch_element_matrices3d(const Grid3& g, const Model& m, const double* u, int lslot,
                                     double* Es, hipStream_t s);
template <typename T>
hipError_t launch_patches3d(const Grid3& g, double tau, const double* Es, T* inv, int* status,
                            hipStream_t s);
// one additive Vanka step d += omega sum_K R_K^T A_K^{-1} R_K res (8 colour launches)
template <typename T>
hipError_t launch_patch_sweep3(const Grid3& g, const T* inv, const T* res, T* d, double omega,
                               hipStream_t s);

// mg3d.hip: coarse levels on hexahedra.  Space-time cell matrices are 170 x 170
// (local unknown mu * 85 + spatial), row-major in FP64; Et: transposed per cell
// in the context precision;
// inv: nc real 170 x 170 inverses, column-major, colour-major patch order.
hipError_t launch_galerkin3d_from_fine(const Grid3& gc, const Grid3& gf, double tau,
                                       const double* Es0, const double* Es1, double* Ec,
                                       hipStream_t s);
hipError_t launch_galerkin3d(const Grid3& gc, const Grid3& gf, const double* Ef, double* Ec,
                             hipStream_t s);
template <typename T>
hipError_t launch_transpose_convert3(int64_t ncells, const double* E, T* Et, hipStream_t s);
template <typename T>
hipError_t launch_level_patches3d(const Grid3& g, const double* E, T* inv, int* status,
                                  hipStream_t s);
// exact finest-level patches from the spatial cell matrices of both Radau nodes
template <typename T>
hipError_t launch_exact_fine_patches3d(const Grid3& g, double tau, const double* Es0,
                                       const double* Es1, T* inv, int* status, hipStream_t s);
// y = A x (b == nullptr) or y = b - A x with the element matrices; S: nc * 170 slots
template <typename T>
hipError_t launch_ebe_apply3d(const Grid3& g, const T* Et, const T* x, const T* b, T* y, T* S,
                              hipStream_t s);
template <typename T>
hipError_t launch_patch_sweep3r(const Grid3& g, const T* inv, const T* res, T* d, double omega,
                                hipStream_t s);
template <typename T>
hipError_t launch_restrict3(const Grid3& gf, const Grid3& gc, const T* rf, T* rc, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add3(const Grid3& gf, const Grid3& gc, const T* dc, T* df,
                               hipStream_t s);
// A (n x n, zeroed by the caller) += the cell matrices E, colour by colour
hipError_t launch_coarse_assemble3(const Grid3& g, const double* E, double* A, hipStream_t s);

// setup.hip
// spatial cell matrices at velocity u; with Dirichlet data (m.lift) the
// Nitsche coefficients of time slot lslot of its table (0, 1: Radau nodes, 2:
// the slab midpoint)
hipError_t launch_element_matrices(const Grid& g, const Model& m, const double* u, int lslot,
                                   double* Es, hipStream_t s);
hipError_t launch_state_combine(int64_t n, const double* u0, const double* u1, double a0,
                                double a1, double* out, hipStream_t s);
template <typename T>
hipError_t launch_convert(int64_t n, const double* in, T* out, hipStream_t s);
// level-0 surrogate patches in time-diagonal form: complex 21x21 inverses
// (interleaved re, im; column-major), from the spatial matrices Es at t_rep
// and the CIP face matrices Sr at t_rep (nm = 1, unscaled; NULL: no CIP)
template <typename T>
hipError_t launch_fine_patches(const Grid& g, double tau, const double* Es, const double* Sr,
                               const uint16_t* masks, T* inv, int* status, hipStream_t s);
// level-0 exact patches (real 42x42 inverses) from the spatial matrices at the
// two Radau nodes and the CIP face matrices S (nm = 2, scaled by tau w_mu; NULL:
// no CIP)
template <typename T>
hipError_t launch_exact_fine_patches(const Grid& g, double tau, const double* Es0,
                                     const double* Es1, const double* S, const uint16_t* masks,
                                     T* inv, int* status, hipStream_t s);
// E (row-major per cell, cell order) -> Et: transposed (column-major per
// cell) in the context precision, stored at patch_slot(g, cx, cy), the order of
// the patch inverses, so that the element-by-element action can stream them
// with the sweep kernels
template <typename T>
hipError_t launch_transpose_convert(const Grid& g, const double* E, T* Et, hipStream_t s);
template <typename T>
hipError_t launch_level_patches(const Grid& g, const double* E, const double* S, T* inv,
                                int* status, hipStream_t s);
hipError_t launch_galerkin_from_fine(const Grid& gc, double tau, const double* Es0,
                                     const double* Es1, double* Ec, hipStream_t s);
hipError_t launch_galerkin(const Grid& gc, const double* Ef, double* Ec, hipStream_t s);
hipError_t launch_coarse_assemble(const Grid& g, const double* E, double* Adense,
                                  hipStream_t s);
// panel width of the blocked coarse Gauss-Jordan inversion
constexpr int kGjNb = 128;
// doubles of work coarse_invert needs: two n x kGjNb panel copies, the
// kGjNb x n row block, per-block pivot candidates of the panel steps (value
// and row, twice)
inline int64_t coarse_invert_work_doubles(int64_t n) {
  return 3 * (int64_t)kGjNb * n + 4 * ((n + 63) / 64) + 8;
}
hipError_t coarse_invert(int64_t n, double* A, double* work, int* piv, int* status,
                         hipStream_t s);

// smooth.hip
// coarse-level action with the transposed element matrices in patch-slot
// order (mode 0: y = A x, mode 1: y = b - A x), through the real-patch sweep
// kernel of variant `variant`; with `slot` (nc x 42 values of scratch) one
// launch over all cells and a node gather, else four colour launches
template <typename T>
hipError_t launch_ebe_apply(const Grid& g, const T* E, const T* x, const T* b, T* y, int mode,
                            int variant, T* slot, hipStream_t s);
// additive Vanka step with sweep variant `variant` (real 42x42 or complex 21x21
// patches); variants differ in workgroup size, loads in flight and rows per
// lane, not in what they compute; real patches with `slot` (nc x 42 values of
// scratch) sum through the per-patch slots and the node gather, which with
// d_zero (d known to be zero on entry) writes d without reading it
template <typename T>
hipError_t launch_patch_sweep(const Grid& g, const T* inv, const T* res, T* d, double omega,
                              int variant, T* slot, hipStream_t s, bool d_zero = false);
template <typename T>
hipError_t launch_patch_sweep_c(const Grid& g, const T* inv, const T* res, T* d, double omega,
                                int variant, hipStream_t s);
int sweep_variant_count(bool complex_form);
// {waves per workgroup, column loads in flight, rows per lane}
void sweep_variant_shape(bool complex_form, int variant, int out[3]);
template <typename T>
hipError_t launch_copy(int64_t n, const T* x, T* y, hipStream_t s);
template <typename T>
hipError_t launch_restrict(const Grid& gf, const Grid& gc, const T* rf, T* rc, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(const Grid& gf, const Grid& gc, const T* dc, T* df,
                              hipStream_t s);
template <typename T>
hipError_t launch_dense_gemv(int64_t n, const T* Ainv, const T* r, T* d,
                             const int64_t* pin, int npin, hipStream_t s);
template <typename T>
hipError_t launch_fill(int64_t n, T v, T* y, hipStream_t s);

// residual.hip: FP64 slab residual R_n(U) (v_prev may be NULL)
hipError_t launch_residual(const Grid& g, const Model& m, double tau, const double* U,
                           const double* vprev, double* R, hipStream_t s);

// load.hip: volume-force right-hand side from f at the Gauss points of every
// cell (f_qp[((mu * cells + cell) * 3^d + q) * d + comp]), FP64; y += x
hipError_t launch_load2(const Grid& g, double tau, const double* f_qp, double* F, hipStream_t s);
hipError_t launch_load3(const Grid3& g, double tau, const double* f_qp, double* F, hipStream_t s);
hipError_t launch_add(int64_t n, const double* x, double* y, hipStream_t s);

// lift.hip: the boundary table of the Dirichlet data (see lift_index) from a
// lifting given as a Q2 velocity field per Radau node (stride g.nv)
hipError_t launch_lift_table(const Grid& g, const Model& m, const double* ghat, double* table,
                             hipStream_t s);
// hexahedra: the boundary table (lift3_index in hex3.h) and the data term
// -tau w_mu B_gamma(g_D, .) into the action's per-cell result slots E (170
// per cell, every cell written)
hipError_t launch_lift3_table(const Grid3& g, const Model& m, const double* ghat, double* table,
                              hipStream_t s);
hipError_t launch_lift3_rhs(const Grid3& g, const Model& m, double tau, const double* table,
                            double* E, hipStream_t s);

// cip.hip: CIP stabilisation on the interior faces of a quadrilateral mesh,
// y += sign * tau w_mu s_CIP(uw_mu; x_mu, .) (sign = +1 action, -1 defect /
// residual); uw_mu = uw + mu * uw_stride (velocity of Radau node mu), G a
// scratch buffer of cip_face_doubles(g) doubles
int64_t cip_face_doubles(const Grid& g);
template <typename T>
hipError_t launch_cip(const Grid& g, const Model& m, double tau, const T* uw, int64_t uw_stride,
                      const T* x, T* y, double sign, double* G, hipStream_t s);

// CIP in the multigrid operators.  Across a face at node column X (or row Y)
// the jump of the normal derivative of a continuous Q2 field is, per node row
// a of the face's cells, j_a = ih sum_o d4(o) x(X + o, a), o = -2..2; the face
// term is then x^T F v with F = (ih d4)(ih d4)^T (x) S, S a symmetric 3 x 3
// matrix over the face's node rows (per Radau node and the same for both
// velocity components).  A Galerkin product P^T F P keeps this form on the
// coarse faces: the fine jump functional applied to a coarse Q2 field is the
// coarse one, faces inside a coarse cell drop out (the coarse field is smooth
// there), and S_coarse sums Py^T S Py over the two fine faces on a coarse
// face, Py the quadratic interpolation along it.  S storage: cip_s_doubles(g)
// per Radau node, S[(f * nm + mu) * 9 + 3 a + b] with nm = 2 (one per Radau
// node) or 1, faces numbered as for launch_cip.
int64_t cip_face_count(const Grid& g);
// level 0: S_mu = scale_mu gamma h_F^2 |F| sum_q w_q |uw_mu . n_F| phi_a phi_b
// at the face points, uw_mu = uw + mu * uw_stride, mu < nm
hipError_t launch_cip_face_matrices(const Grid& g, const Model& m, const double* uw,
                                    int64_t uw_stride, int nm, double scale0, double scale1,
                                    double* S, hipStream_t s);
// coarse-level S (nm = 2) from those of the next finer level
hipError_t launch_cip_restrict(const Grid& gc, const Grid& gf, const double* Sf, double* Sc,
                               hipStream_t s);
// y += sign * F x on a level with stored S (nm = 2); G scratch as for launch_cip
template <typename T>
hipError_t launch_cip_level(const Grid& g, const double* S, const T* x, T* y, double sign,
                            double* G, hipStream_t s);
// adds the face terms to the rows of the dense space-time operator A (n = g.nst)
hipError_t launch_cip_dense(const Grid& g, const double* S, double* A, hipStream_t s);

__host__ __device__ inline double cip_d4(int o) {  // o = node column - face column, -2..2
  return o == 0 ? 6.0 : ((o == 1 || o == -1) ? -4.0 : 1.0);
}

// Entry of the face part between velocity unknowns of one component and one
// Radau node at nodes (xa, ya) and (xb, yb): the sum over the faces whose
// 5 x 3 node stencil holds both.
__device__ inline double cip_pair(const Grid& g, const double* __restrict__ S, int nm, int mu,
                                  int xa, int ya, int xb, int yb) {
  const int64_t nV = (int64_t)(g.nx - 1) * g.ny;
  double v = 0.0;
  const int xlo = (xa > xb ? xa : xb) - 2, xhi = (xa < xb ? xa : xb) + 2;
  const int ylo = (ya > yb ? ya : yb) - 2, yhi = (ya < yb ? ya : yb) + 2;
  // vertical faces: node column X = 2 cx, cx = 1 .. nx-1; cell row cy holding both rows
  for (int X = xlo + (xlo & 1); X <= xhi; X += 2) {
    const int cx = X / 2;
    if (cx < 1 || cx > g.nx - 1) continue;
    const double dd = cip_d4(xa - X) * cip_d4(xb - X) * g.ihx * g.ihx;
    for (int cy = (ya < yb ? ya : yb) / 2 - 1; cy <= (ya < yb ? ya : yb) / 2; ++cy) {
      if (cy < 0 || cy >= g.ny) continue;
      const int a = ya - 2 * cy, b = yb - 2 * cy;
      if (a < 0 || a > 2 || b < 0 || b > 2) continue;
      const int64_t f = (int64_t)cy * (g.nx - 1) + cx - 1;
      v += dd * S[(f * nm + mu) * 9 + 3 * a + b];
    }
  }
  // horizontal faces: node row Y = 2 cy, cy = 1 .. ny-1; cell column cx holding both columns
  for (int Y = ylo + (ylo & 1); Y <= yhi; Y += 2) {
    const int cy = Y / 2;
    if (cy < 1 || cy > g.ny - 1) continue;
    const double dd = cip_d4(ya - Y) * cip_d4(yb - Y) * g.ihy * g.ihy;
    for (int cx = (xa < xb ? xa : xb) / 2 - 1; cx <= (xa < xb ? xa : xb) / 2; ++cx) {
      if (cx < 0 || cx >= g.nx) continue;
      const int a = xa - 2 * cx, b = xb - 2 * cx;
      if (a < 0 || a > 2 || b < 0 || b > 2) continue;
      const int64_t f = nV + (int64_t)(cy - 1) * g.nx + cx;
      v += dd * S[(f * nm + mu) * 9 + 3 * a + b];
    }
  }
  return v;
}

// krylov.hip: vector kernels of the slab solve (FP64)
int dot_partials();  // partial sums per vector of launch_multi_dot
hipError_t launch_mass(const Grid& g, double tau, const double* x, double* y, hipStream_t s);
// hexahedra: y_mu = c_mu (M_x x_v,mu ; pscale M_p x_p,mu), FP64, x != y
hipError_t launch_mass3(const Grid3& g, double c0, double c1, double pscale, const double* x,
                        double* y, hipStream_t s);
// out[i] = V_i . u for i < k (V_i = V + i ldv); partial: k * dot_partials() doubles
hipError_t launch_multi_dot(int64_t n, int k, const double* V, int64_t ldv, const double* u,
                            double* partial, double* out, hipStream_t s);
// w = alpha w + sgn sum_{i<k} c[i] V_i, c on the device
hipError_t launch_combine(int64_t n, int k, const double* V, int64_t ldv, const double* c,
                          double sgn, double alpha, double* w, hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t s);
hipError_t launch_widen(int64_t n, const float* x, double* y, hipStream_t s);
hipError_t launch_narrow(int64_t n, const double* x, float* y, hipStream_t s);

}  // namespace pns
