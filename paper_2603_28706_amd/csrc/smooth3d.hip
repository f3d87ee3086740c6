// Vanka smoother on hexahedra (Q2 / P1disc x dG(1)) at the finest level,
// Sec. 6.3: cell patches (27 nodes x 3 components + 4 pressure coefficients per
// Radau node), patch matrix R_K A R_K^T of the surrogate slab operator whose
// state-dependent coefficients are frozen at the slab midpoint (eq.
// surrogate-diag), additive update d <- d + omega sum_K R_K^T A_K^{-1} R_K (r - A d)
// (eq. stmg-vanka-update).
//
// The surrogate patch matrix is K_t (x) M_K + tau M_t (x) J_K with the same
// spatial blocks at both Radau nodes, so it is inverted in time-diagonal form:
// M_t^{-1} K_t has the eigenvalues lam, conj(lam) (lam = 2 + i sqrt2) and for a
// real right-hand side a single complex 85 x 85 system (lam M_K + tau J_K) y = z
// gives both Radau blocks of the correction.
//
// * element_matrix3d_kernel: the 85 x 85 spatial Jacobian of every cell at the
//   midpoint state (volume terms and, on boundary cells, the Nitsche and flux
//   terms of the boundary faces), FP64, one workgroup per cell; one thread per
//   (test node, trial node) pair forms the 3 x 3 velocity block, one per
//   (node, pressure coefficient) the divergence couplings.
// * patch3_kernel: one workgroup per patch sums the element matrices of the up
//   to 27 cells around the patch on the unknowns of the patch (the cell's own
//   pressure enters through the cell alone), adds lam times the Q2 mass (the
//   tensor product of 1D masses), and inverts the complex matrix in LDS by
//   Gauss-Jordan with partial row pivoting, in place, in FP64; the inverse is
//   stored column-major, complex interleaved, in the context precision, patches
//   in colour-major order (colour = parity of the cell in x, y, z).
// * patch_sweep3_kernel: one workgroup per patch of one colour; cells of one
//   colour share no node, so their corrections are added without atomics.
#include <type_traits>

#include "hex3.h"

namespace pns {
namespace {

constexpr int kMaxPts = 27 + 6 * 9;  // volume points + face points of a cell

// ------------------------------------------------------------ cell matrices

struct Pt3 {
  double xi[3];   // reference coordinates
  double W;       // weight times measure
  double n[3];    // outward unit normal; zero at volume points
  double ihF;     // 1 / cell size normal to the face
  double u[3];    // state
  double A[3][3]; // symmetric gradient of the state
  double eta, kap;
  double GD[6];   // boundary points: G = D ghat_D (00, 01, 02, 11, 12, 22)
  double etaG, kG;
};


// lslot: time slot of the Dirichlet data table (m.lift) matching u (0, 1: the
// Radau nodes, 2: the slab midpoint); ignored without data
__global__ __launch_bounds__(256) void element_matrix3d_kernel(Grid3 g, Model m,
                                                               const double* __restrict__ u,
                                                               int lslot,
                                                               double* __restrict__ Es) {
  __shared__ double ul[kNv3];
  __shared__ Pt3 pts[kMaxPts];
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % g.nx), cy = (int)((cell / g.nx) % g.ny),
            cz = (int)(cell / ((int64_t)g.nx * g.ny));
  const int t = threadIdx.x;
  if (t < kNv3) ul[t] = u[(int64_t)(t / kNb3) * g.nn + node_index3(g, cx, cy, cz, t % kNb3)];
  // boundary sides of the cell: side 2k (low end of direction k), 2k + 1 (high)
  int sides[6], nsd = 0;
  const int ci[3] = {cx, cy, cz}, nc[3] = {g.nx, g.ny, g.nz};
  for (int k = 0; k < 3; ++k) {
    if (ci[k] == 0) sides[nsd++] = 2 * k;
    if (ci[k] == nc[k] - 1) sides[nsd++] = 2 * k + 1;
  }
  const int npts = 27 + 9 * nsd;
  const double h[3] = {g.hx, g.hy, g.hz};
  __syncthreads();
  if (t < npts) {
    Pt3 P;
    if (t < 27) {
      const int q[3] = {t % 3, (t / 3) % 3, t / 9};
      for (int k = 0; k < 3; ++k) {
        P.xi[k] = kGP[q[k]];
        P.n[k] = 0.0;
      }
      P.W = kGW[q[0]] * kGW[q[1]] * kGW[q[2]] * g.hx * g.hy * g.hz;
      P.ihF = 0.0;
    } else {
      const int sd = sides[(t - 27) / 9], qa = (t - 27) % 9;
      const int k = sd >> 1, hi = sd & 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      P.xi[k] = hi ? 1.0 : 0.0;
      P.xi[k1] = kGP[qa % 3];
      P.xi[k2] = kGP[qa / 3];
      for (int d = 0; d < 3; ++d) P.n[d] = d == k ? (hi ? 1.0 : -1.0) : 0.0;
      P.W = kGW[qa % 3] * kGW[qa / 3] * h[k1] * h[k2];
      P.ihF = 1.0 / h[k];
    }
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int c = 0; c < 3; ++c) P.u[c] = 0.0;
    for (int a = 0; a < kNb3; ++a) {
      double ph, gr[3];
      basis3(g, a, P.xi, ph, gr);
      for (int c = 0; c < 3; ++c) {
        const double v = ul[c * kNb3 + a];
        P.u[c] += v * ph;
        for (int d = 0; d < 3; ++d) G[c][d] += v * gr[d];
      }
    }
    double a2 = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        P.A[i][j] = 0.5 * (G[i][j] + G[j][i]);
        a2 += P.A[i][j] * P.A[i][j];
      }
    const double D2 = m.delta2 + a2;
    const double mu = m.nu * pow(D2, m.expo);
    P.eta = m.nu_inf + mu;
    double kp = 0.0;
    if (m.lin != PNS_PICARD) {
      kp = (m.p - 2.0) * mu / D2;
      if (m.lin == PNS_MODIFIED_NEWTON) {
        const double sig = mu * sqrt(a2);
        kp *= sig > 0.0 ? fmin(1.0, m.sigma_max / sig) : 0.0;
      }
    }
    P.kap = kp;
    for (int e = 0; e < 6; ++e) P.GD[e] = 0.0;
    P.etaG = m.etaD;
    P.kG = 0.0;
    if (m.lift && t >= 27) {
      const int sd = sides[(t - 27) / 9], qa = (t - 27) % 9;
      const int k = sd >> 1, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      const double* lt = m.lift + lift3_index(g, sd, ci[k1], ci[k2], qa, lslot);
      for (int e = 0; e < 6; ++e) P.GD[e] = lt[3 + e];
      P.etaG = lt[9];
      P.kG = lt[10];
    }
    pts[t] = P;
  }
  __syncthreads();
  const bool newton = m.lin != PNS_PICARD;
  double* Ec = Es + cell * kEs3;
  constexpr int kVV = kNb3 * kNb3, kVP = kNb3 * 4;
  for (int task = t; task < kVV + kVP + 1; task += blockDim.x) {
    if (task < kVV) {
      // velocity block: test node a, trial node b, all component pairs
      const int a = task / kNb3, b = task % kNb3;
      double blk[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int q = 0; q < npts; ++q) {
        const Pt3& P = pts[q];
        double pa, ga[3], pb, gb[3];
        basis3(g, a, P.xi, pa, ga);
        basis3(g, b, P.xi, pb, gb);
        double Aga[3], Agb[3];
        for (int i = 0; i < 3; ++i) {
          Aga[i] = P.A[i][0] * ga[0] + P.A[i][1] * ga[1] + P.A[i][2] * ga[2];
          Agb[i] = P.A[i][0] * gb[0] + P.A[i][1] * gb[1] + P.A[i][2] * gb[2];
        }
        if (q < 27) {
          const double gab = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
          const double Ug = P.u[0] * ga[0] + P.u[1] * ga[1] + P.u[2] * ga[2];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              // T(D x) : D w with x = phi_b e_j, w = phi_a e_i
              double v = P.eta * 0.5 * ((i == j ? gab : 0.0) + ga[j] * gb[i]) +
                         P.kap * Aga[i] * Agb[j];
              if (m.convection) {
                // -(x (x) u_k [+ u_k (x) x]) : grad w
                v -= (i == j ? pb * Ug : 0.0);
                if (newton) v -= P.u[i] * pb * ga[j];
              }
              blk[i][j] += P.W * v;
            }
        } else {
          const double* n = P.n;
          const double un = P.u[0] * n[0] + P.u[1] * n[1] + P.u[2] * n[2];
          const double gan = ga[0] * n[0] + ga[1] * n[1] + ga[2] * n[2];
          const double gbn = gb[0] * n[0] + gb[1] * n[1] + gb[2] * n[2];
          double An[3];
          for (int i = 0; i < 3; ++i) An[i] = P.A[i][0] * n[0] + P.A[i][1] * n[1] + P.A[i][2] * n[2];
          double GL[3][3], Gga[3], Gn[3];
          sym3(P.GD, GL);
          for (int i = 0; i < 3; ++i) {
            Gga[i] = GL[i][0] * ga[0] + GL[i][1] * ga[1] + GL[i][2] * ga[2];
            Gn[i] = GL[i][0] * n[0] + GL[i][1] * n[1] + GL[i][2] * n[2];
          }
          const double pab = pa * pb;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              const double dij = i == j ? 1.0 : 0.0;
              double v = 0.0;
              if (m.convection) {
                v += dij * un * pab;                       // (u_k . n)(x . w)
                if (newton) v += pb * n[j] * P.u[i] * pa;  // (x . n)(u_k . w)
                v -= 0.5 * (fabs(un) - un) * dij * pab;    // inflow: -(u_k . n)^- (x . w)
              }
              // -(T(D x) n) . w
              v -= pa * (P.eta * 0.5 * (dij * gbn + gb[i] * n[j]) + P.kap * Agb[j] * An[i]);
              // -(DS(G)(D w) n) . x, DS(G)(D w) = eta(G) D w + k (G : D w) G
              v -= pb * (P.etaG * 0.5 * (dij * gan + ga[j] * n[i]) + P.kG * Gga[i] * Gn[j]);
              // penalties
              v += m.gamma1 * P.etaG * P.ihF * dij * pab + m.gamma2 * P.ihF * pb * n[j] * pa * n[i];
              blk[i][j] += P.W * v;
            }
        }
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ec[(i * kNb3 + a) * kNs3 + j * kNb3 + b] = blk[i][j];
    } else if (task < kVV + kVP) {
      // divergence couplings of node a with pressure coefficient jp
      const int a = (task - kVV) / 4, jp = (task - kVV) % 4;
      double vp[3] = {0, 0, 0}, pv[3] = {0, 0, 0};
      for (int q = 0; q < npts; ++q) {
        const Pt3& P = pts[q];
        double pa, ga[3];
        basis3(g, a, P.xi, pa, ga);
        const double qj = jp == 0 ? 1.0 : P.xi[jp - 1] - 0.5;
        for (int c = 0; c < 3; ++c) {
          if (q < 27) {
            vp[c] -= P.W * ga[c] * qj;  // -(div w, q)
            pv[c] -= P.W * ga[c] * qj;  // -(div x, psi)
          } else {
            vp[c] += P.W * qj * pa * P.n[c];            // q (w . n)
            pv[c] += P.W * m.qsign * pa * P.n[c] * qj;  // sign * (x . n) psi
          }
        }
      }
      for (int c = 0; c < 3; ++c) {
        Ec[(c * kNb3 + a) * kNs3 + kNv3 + jp] = vp[c];
        Ec[(kNv3 + jp) * kNs3 + c * kNb3 + a] = pv[c];
      }
    } else {
      for (int e = 0; e < 16; ++e) Ec[(kNv3 + e / 4) * kNs3 + kNv3 + e % 4] = 0.0;
    }
  }
}

// ----------------------------------------------------------------- patches

constexpr int kPatchThreads = 512;

template <typename T>
__global__ __launch_bounds__(kPatchThreads) void patch3_kernel(Grid3 g, double tau,
                                                               const double* __restrict__ Es,
                                                               T* __restrict__ inv,
                                                               int* status) {
  __shared__ double Ar[kNs3][kNs3], Ai[kNs3][kNs3];
  __shared__ double rkr[kNs3], rki[kNs3], fr[kNs3], fi[kNs3];
  __shared__ int piv[kNs3], src[kNs3];
  __shared__ double s_pr, s_pi, s_kr, s_ki;
  __shared__ int s_p, s_sing;
  const int64_t K = blockIdx.x;
  const int cx = (int)(K % g.nx), cy = (int)((K / g.nx) % g.ny),
            cz = (int)(K / ((int64_t)g.nx * g.ny));
  const int cc[3] = {cx, cy, cz}, nc[3] = {g.nx, g.ny, g.nz};
  const int t = threadIdx.x;
  if (t == 0) s_sing = 0;
  // assembly: entry (r, c) sums the cells that hold both unknowns
  for (int e = t; e < kEs3; e += kPatchThreads) {
    const int r = e / kNs3, c = e % kNs3;
    double jv = 0.0, mv = 0.0;
    if (r >= kNv3 || c >= kNv3) {
      jv = Es[K * kEs3 + e];  // the cell's own pressure lives in this cell only
    } else {
      const int a = r % kNb3, b = c % kNb3;
      const int pa[3] = {a % 3, (a / 3) % 3, a / 9}, pb[3] = {b % 3, (b / 3) % 3, b / 9};
      int lo[3], hi[3];
      for (int k = 0; k < 3; ++k) {
        // a neighbour at offset -1 holds local position 0, at +1 position 2
        lo[k] = (pa[k] == 0 && pb[k] == 0 && cc[k] > 0) ? -1 : 0;
        hi[k] = (pa[k] == 2 && pb[k] == 2 && cc[k] < nc[k] - 1) ? 1 : 0;
      }
      const bool same = r / kNb3 == c / kNb3;
      for (int oz = lo[2]; oz <= hi[2]; ++oz)
        for (int oy = lo[1]; oy <= hi[1]; ++oy)
          for (int ox = lo[0]; ox <= hi[0]; ++ox) {
            const int o[3] = {ox, oy, oz};
            int na = 0, nb = 0, st = 1;
            for (int k = 0; k < 3; ++k) {
              na += (pa[k] - 2 * o[k]) * st;
              nb += (pb[k] - 2 * o[k]) * st;
              st *= 3;
            }
            const int64_t nbc = cell_index3(g, cx + ox, cy + oy, cz + oz);
            jv += Es[nbc * kEs3 + ((r / kNb3) * kNb3 + na) * kNs3 + (c / kNb3) * kNb3 + nb];
            if (same) mv += cell_mass3(g, na, nb);
          }
    }
    Ar[r][c] = kLamRe * mv + tau * jv;
    Ai[r][c] = kLamIm * mv;
  }
  __syncthreads();
  for (int k = 0; k < kNs3; ++k) {
    if (t < 64) {
      // pivot: largest |A[i][k]|^2 over i >= k (ties to the smaller row)
      double bv = -1.0;
      int bi = k;
      for (int i = k + t; i < kNs3; i += 64) {
        const double v = Ar[i][k] * Ar[i][k] + Ai[i][k] * Ai[i][k];
        if (v > bv) {
          bv = v;
          bi = i;
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
          s_pr = 1.0;
          s_pi = 0.0;
        } else {
          s_pr = Ar[bi][k];
          s_pi = Ai[bi][k];
        }
        s_kr = Ar[k][k];
        s_ki = Ai[k][k];
      }
    }
    __syncthreads();
    const int p = s_p;
    const double den = s_pr * s_pr + s_pi * s_pi;
    const double dr = s_pr / den, di = -s_pi / den;  // 1 / pivot
    if (t < kNs3) {
      // swap rows k and p; scale the new row k (its pivot entry becomes 1 / pivot)
      const int j = t;
      const double kr = Ar[k][j], ki = Ai[k][j];
      double xr = Ar[p][j], xi = Ai[p][j];
      if (p != k) {
        Ar[p][j] = kr;
        Ai[p][j] = ki;
      }
      if (j == k) {
        xr = 1.0;
        xi = 0.0;
      }
      const double yr = xr * dr - xi * di, yi = xr * di + xi * dr;
      Ar[k][j] = yr;
      Ai[k][j] = yi;
      rkr[j] = yr;
      rki[j] = yi;
    } else if (t >= 128 && t < 128 + kNs3) {
      // elimination factors: column k after the row swap, zero on row k
      const int i = t - 128;
      double vr = 0.0, vi = 0.0;
      if (i == p && p != k) {
        vr = s_kr;
        vi = s_ki;
      } else if (i != k) {
        vr = Ar[i][k];
        vi = Ai[i][k];
      }
      fr[i] = vr;
      fi[i] = vi;
    }
    __syncthreads();
    for (int e = t; e < kEs3; e += kPatchThreads) {
      const int i = e / kNs3, j = e % kNs3;
      if (i == k) continue;
      const double ar = j == k ? 0.0 : Ar[i][j], ai = j == k ? 0.0 : Ai[i][j];
      const double f_r = fr[i], f_i = fi[i], br = rkr[j], bi = rki[j];
      Ar[i][j] = ar - (f_r * br - f_i * bi);
      Ai[i][j] = ai - (f_r * bi + f_i * br);
    }
    __syncthreads();
  }
  // the row interchanges become column interchanges of the inverse, applied
  // in reverse order
  if (t == 0) {
    for (int j = 0; j < kNs3; ++j) src[j] = j;
    for (int k = kNs3 - 1; k >= 0; --k) {
      const int tmp = src[k];
      src[k] = src[piv[k]];
      src[piv[k]] = tmp;
    }
    if (s_sing) atomicOr(status, 1);
  }
  __syncthreads();
  T* out = inv + patch_slot3(g, cx, cy, cz) * (2 * kEs3);
  for (int e = t; e < kEs3; e += kPatchThreads) {
    const int c = e / kNs3, r = e % kNs3;
    out[2 * e] = (T)Ar[r][src[c]];
    out[2 * e + 1] = (T)Ai[r][src[c]];
  }
}

// ------------------------------------------------------------------ sweep

constexpr int kSweepThreads = 256;
constexpr int kColChunk = (kNs3 + 2) / 3;  // columns per thread (3 threads per row)

template <typename T>
__global__ __launch_bounds__(kSweepThreads) void patch_sweep3_kernel(
    Grid3 g, const T* __restrict__ inv, const T* __restrict__ res, T* __restrict__ d, T omega,
    int px, int py, int pz, int ncx, int ncy, int64_t slot0) {
  using T2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
  __shared__ T zr[kNs3], zi[kNs3];
  __shared__ T yr3[3][kNs3], yi3[3][kNs3];
  const int64_t pid = blockIdx.x;
  const int cx = px + 2 * (int)(pid % ncx);
  const int cy = py + 2 * (int)((pid / ncx) % ncy);
  const int cz = pz + 2 * (int)(pid / ((int64_t)ncx * ncy));
  const int t = threadIdx.x;
  int64_t g0 = 0, g1 = 0;
  if (t < kNs3) {
    g0 = gidx3(g, cx, cy, cz, t, 0);
    g1 = gidx3(g, cx, cy, cz, t, 1);
    const T r0 = res[g0], r1 = res[g1];
    zr[t] = (T)kZr0 * r0;
    zi[t] = (T)kZi0 * r0 + (T)kZi1 * r1;
  }
  __syncthreads();
  if (t < 3 * kNs3) {
    const int i = t % kNs3, part = t / kNs3;
    const int j0 = part * kColChunk, j1 = min(kNs3, j0 + kColChunk);
    const T2* C = reinterpret_cast<const T2*>(inv + (slot0 + pid) * (2 * kEs3));
    T sr = 0, si = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
      const T2 cv = C[j * kNs3 + i];
      sr += cv.x * zr[j] - cv.y * zi[j];
      si += cv.x * zi[j] + cv.y * zr[j];
    }
    yr3[part][i] = sr;
    yi3[part][i] = si;
  }
  __syncthreads();
  if (t < kNs3) {
    const T yr = yr3[0][t] + yr3[1][t] + yr3[2][t];
    const T yi = yi3[0][t] + yi3[1][t] + yi3[2][t];
    d[g0] += omega * (T)2 * yr;
    d[g1] += omega * (T)2 * (yr - (T)kBackIm * yi);
  }
}

}  // namespace

hipError_t launch_element_matrices3d(const Grid3& g, const Model& m, const double* u, int lslot,
                                     double* Es, hipStream_t s) {
  hipLaunchKernelGGL(element_matrix3d_kernel, dim3((unsigned)g.nc), dim3(256), 0, s, g, m, u, lslot,
                     Es);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_patches3d(const Grid3& g, double tau, const double* Es, T* inv, int* status,
                            hipStream_t s) {
  hipLaunchKernelGGL(patch3_kernel<T>, dim3((unsigned)g.nc), dim3(kPatchThreads), 0, s, g, tau, Es,
                     inv, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_patch_sweep3(const Grid3& g, const T* inv, const T* res, T* d, double omega,
                               hipStream_t s) {
  int64_t slot0 = 0;
  for (int c = 0; c < 8; ++c) {
    const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
    const int64_t np = colour_count3(g, c);
    if (np > 0)
      hipLaunchKernelGGL(patch_sweep3_kernel<T>, dim3((unsigned)np), dim3(kSweepThreads), 0, s, g,
                         inv, res, d, (T)omega, px, py, pz, (g.nx - px + 1) / 2,
                         (g.ny - py + 1) / 2, slot0);
    slot0 += np;
  }
  return hipGetLastError();
}

template hipError_t launch_patches3d<double>(const Grid3&, double, const double*, double*, int*,
                                             hipStream_t);
template hipError_t launch_patches3d<float>(const Grid3&, double, const double*, float*, int*,
                                            hipStream_t);
template hipError_t launch_patch_sweep3<double>(const Grid3&, const double*, const double*, double*,
                                                double, hipStream_t);
template hipError_t launch_patch_sweep3<float>(const Grid3&, const float*, const float*, float*,
                                               double, hipStream_t);

}  // namespace pns
