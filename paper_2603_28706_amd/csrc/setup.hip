// Smoother setup on the GPU (Sec. 6.3):
// * spatial cell matrices of J_mu at a given velocity state (FP64), used for the
//   surrogate patches (state frozen at the slab midpoint, eq. surrogate-diag)
//   and for the exact level-0 element matrices entering the Galerkin product;
// * patch matrices R_K A R_K^T of cell patches, including the contributions of
//   the 8 neighbouring cells on shared nodes, inverted by Gauss-Jordan with
//   partial pivoting in FP64 (one wave per patch, LDS resident);
// * coarse element matrices E_C = sum_children P_f^T E_f P_f (Galerkin,
//   A_{l+1} = P^T A_l P restricted cell by cell);
// * the dense coarsest operator, pinned at the constant pressure coefficient
//   of cell 0 per Radau node, and its in-place Gauss-Jordan inverse.
#include "pns_internal.h"

namespace pns {
namespace {

__device__ __forceinline__ int64_t st_global_index(const Grid& g, int cx, int cy, int l) {
  // space-time local index l = mu*21 + i  ->  canonical global index
  const int mu = l / kNs, i = l % kNs;
  const int NX = 2 * g.nx + 1;
  if (i < 18) {
    const int comp = i / 9, a = i % 9;
    return (int64_t)mu * g.ns + (int64_t)comp * g.nn + (int64_t)(2 * cy + a / 3) * NX +
           (2 * cx + a % 3);
  }
  return (int64_t)mu * g.ns + g.nv + 3 * ((int64_t)cy * g.nx + cx) + (i - 18);
}

// scalar Q2 mass matrix of the reference cell, by the 3x3 Gauss rule (times
// h_x h_y: the cell's)
__device__ __forceinline__ double ref_mass(int a, int b) {
  double s = 0.0;
  for (int qy = 0; qy < 3; ++qy)
    for (int qx = 0; qx < 3; ++qx)
      s += kGW[qx] * kGW[qy] * q2v(a % 3, kGP[qx]) * q2v(a / 3, kGP[qy]) * q2v(b % 3, kGP[qx]) *
           q2v(b / 3, kGP[qy]);
  return s;
}
__device__ __forceinline__ double cell_mass(const Grid& g, int a, int b) {
  return ref_mass(a, b) * g.hx * g.hy;
}
// the 81 reference values into LDS once per workgroup (the patch kernels read
// them for every entry and neighbour)
__device__ __forceinline__ void fill_ref_mass(double* M) {
  for (int e = threadIdx.x; e < 81; e += blockDim.x) M[e] = ref_mass(e / 9, e % 9);
}

// ----------------------------------------------------------- cell matrices

struct Pt {
  double xi, et, W, n0, n1, hF;  // reference point, weight, normal (0 inside)
  double u0, u1, a00, a01, a11, eta, kap;
  // boundary points: frozen Nitsche coefficients at G = D ghat_D
  double G00, G01, G11, etaG, kG;
};

struct Fld {
  double v0, v1, g00, g01, g10, g11, q;
};

__device__ __forceinline__ Fld unit_fld(const Grid& g, int i, double xi, double et) {
  Fld f{0, 0, 0, 0, 0, 0, 0};
  if (i < 18) {
    const int comp = i / 9, a = i % 9, ax = a % 3, ay = a / 3;
    const double ph = q2v(ax, xi) * q2v(ay, et);
    const double px = q2d(ax, xi) / g.hx * q2v(ay, et);
    const double py = q2v(ax, xi) * q2d(ay, et) / g.hy;
    if (comp == 0) {
      f.v0 = ph; f.g00 = px; f.g01 = py;
    } else {
      f.v1 = ph; f.g10 = px; f.g11 = py;
    }
  } else {
    const int j = i - 18;
    f.q = j == 0 ? 1.0 : (j == 1 ? xi - 0.5 : et - 0.5);
  }
  return f;
}

__device__ double pair_integrand(const Model& m, const Pt& P, const Fld& x, const Fld& w) {
  // tangent applied to the trial symmetric gradient
  const double b00 = x.g00, b01 = 0.5 * (x.g01 + x.g10), b11 = x.g11;
  const double ab = P.a00 * b00 + 2.0 * P.a01 * b01 + P.a11 * b11;
  const double T00 = P.eta * b00 + P.kap * ab * P.a00;
  const double T01 = P.eta * b01 + P.kap * ab * P.a01;
  const double T11 = P.eta * b11 + P.kap * ab * P.a11;
  const double d00 = w.g00, d01 = 0.5 * (w.g01 + w.g10), d11 = w.g11;
  const bool newton = m.lin != PNS_PICARD;
  double s = 0.0;
  if (P.n0 == 0.0 && P.n1 == 0.0) {
    s = T00 * d00 + 2.0 * T01 * d01 + T11 * d11;
    if (m.convection) {
      const double X[2] = {x.v0, x.v1}, U[2] = {P.u0, P.u1};
      const double G[2][2] = {{w.g00, w.g01}, {w.g10, w.g11}};
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          double c = X[i] * U[j];
          if (newton) c += U[i] * X[j];
          s -= c * G[i][j];
        }
    }
    s -= (w.g00 + w.g11) * x.q;
    s -= (x.g00 + x.g11) * w.q;
  } else {
    const double n0 = P.n0, n1 = P.n1;
    const double un = P.u0 * n0 + P.u1 * n1, xn = x.v0 * n0 + x.v1 * n1, wn = w.v0 * n0 + w.v1 * n1;
    const double xw = x.v0 * w.v0 + x.v1 * w.v1;
    if (m.convection) {
      s += un * xw;
      if (newton) s += xn * (P.u0 * w.v0 + P.u1 * w.v1);
      s -= 0.5 * (fabs(un) - un) * xw;
    }
    s -= (T00 * n0 + T01 * n1) * w.v0 + (T01 * n0 + T11 * n1) * w.v1;
    // -(DS(G)(Dw) n).x, DS(G)(Dw) = eta(G) Dw + k (G:Dw) G
    const double gd = P.G00 * d00 + 2.0 * P.G01 * d01 + P.G11 * d11;
    const double e00 = P.etaG * d00 + P.kG * gd * P.G00;
    const double e01 = P.etaG * d01 + P.kG * gd * P.G01;
    const double e11 = P.etaG * d11 + P.kG * gd * P.G11;
    s -= (e00 * n0 + e01 * n1) * x.v0 + (e01 * n0 + e11 * n1) * x.v1;
    s += x.q * wn;
    s += m.qsign * xn * w.q;
    s += m.gamma1 * P.etaG / P.hF * xw + m.gamma2 / P.hF * xn * wn;
  }
  return P.W * s;
}

// lslot: time slot of the Dirichlet data table (m.lift) matching u (0, 1: the
// Radau nodes, 2: the slab midpoint); ignored without data
__global__ __launch_bounds__(256) void element_matrix_kernel(Grid g, Model m,
                                                             const double* __restrict__ u,
                                                             int lslot,
                                                             double* __restrict__ Es) {
  __shared__ double ul[18];
  __shared__ Pt pts[21];
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % g.nx), cy = (int)(cell / g.nx);
  const int t = threadIdx.x;
  const int NX = 2 * g.nx + 1;
  if (t < 18) {
    const int comp = t / 9, a = t % 9;
    ul[t] = u[(int64_t)comp * g.nn + (int64_t)(2 * cy + a / 3) * NX + 2 * cx + a % 3];
  }
  // point list: 9 volume points, then 3 per boundary face
  int nfaces = 0;
  int faces[4];
  if (cx == 0) faces[nfaces++] = 0;
  if (cx == g.nx - 1) faces[nfaces++] = 1;
  if (cy == 0) faces[nfaces++] = 2;
  if (cy == g.ny - 1) faces[nfaces++] = 3;
  const int npts = 9 + 3 * nfaces;
  __syncthreads();
  if (t < npts) {
    Pt P;
    if (t < 9) {
      const int qx = t % 3, qy = t / 3;
      P.xi = kGP[qx]; P.et = kGP[qy];
      P.W = kGW[qx] * kGW[qy] * g.hx * g.hy;
      P.n0 = P.n1 = 0.0; P.hF = 1.0;
    } else {
      const int f = faces[(t - 9) / 3], q = (t - 9) % 3;
      const bool xf = f < 2;
      P.xi = xf ? (f == 0 ? 0.0 : 1.0) : kGP[q];
      P.et = xf ? kGP[q] : (f == 2 ? 0.0 : 1.0);
      P.W = kGW[q] * (xf ? g.hy : g.hx);
      P.n0 = xf ? (f == 0 ? -1.0 : 1.0) : 0.0;
      P.n1 = xf ? 0.0 : (f == 2 ? -1.0 : 1.0);
      P.hF = xf ? g.hx : g.hy;
    }
    double u0 = 0, u1 = 0, g00 = 0, g01 = 0, g10 = 0, g11 = 0;
    for (int a = 0; a < 9; ++a) {
      const int ax = a % 3, ay = a / 3;
      const double ph = q2v(ax, P.xi) * q2v(ay, P.et);
      const double px = q2d(ax, P.xi) / g.hx * q2v(ay, P.et);
      const double py = q2v(ax, P.xi) * q2d(ay, P.et) / g.hy;
      u0 += ul[a] * ph; u1 += ul[9 + a] * ph;
      g00 += ul[a] * px; g01 += ul[a] * py;
      g10 += ul[9 + a] * px; g11 += ul[9 + a] * py;
    }
    P.u0 = u0; P.u1 = u1;
    P.a00 = g00; P.a01 = 0.5 * (g01 + g10); P.a11 = g11;
    const double a2 = P.a00 * P.a00 + 2.0 * P.a01 * P.a01 + P.a11 * P.a11;
    const double D2 = m.delta2 + a2;
    const double mu = m.nu * pow(D2, m.expo);
    P.eta = m.nu_inf + mu;
    double k = 0.0;
    if (m.lin != PNS_PICARD) {
      k = (m.p - 2.0) * mu / D2;
      if (m.lin == PNS_MODIFIED_NEWTON) {
        const double sig = mu * sqrt(a2);
        k *= sig > 0.0 ? fmin(1.0, m.sigma_max / sig) : 0.0;
      }
    }
    P.kap = k;
    P.G00 = P.G01 = P.G11 = 0.0;
    P.etaG = m.etaD;
    P.kG = 0.0;
    if (m.lift && t >= 9) {
      const int side = faces[(t - 9) / 3];
      const double* lt = m.lift + lift_index(g, side, side < 2 ? cy : cx, (t - 9) % 3, lslot);
      P.G00 = lt[2];
      P.G01 = lt[3];
      P.G11 = lt[4];
      P.etaG = lt[5];
      P.kG = lt[6];
    }
    pts[t] = P;
  }
  __syncthreads();
  for (int e = t; e < kNs * kNs; e += blockDim.x) {
    const int i = e / kNs, j = e % kNs;  // row = test i, column = trial j
    double s = 0.0;
    for (int q = 0; q < npts; ++q) {
      const Pt P = pts[q];
      const Fld w = unit_fld(g, i, P.xi, P.et);
      const Fld x = unit_fld(g, j, P.xi, P.et);
      s += pair_integrand(m, P, x, w);
    }
    Es[cell * (kNs * kNs) + e] = s;
  }
}

__global__ void combine_kernel(int64_t n, const double* a, const double* b, double ca, double cb,
                               double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ca * a[i] + cb * b[i];
}

template <typename T>
__global__ void convert_kernel(int64_t n, const double* in, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

// --------------------------------------------------------------- patches

// space-time element entry of the level-0 operator built from spatial cell
// matrices: K_t[mu][nu] M (same velocity component) + delta_mu,nu tau w_mu Es_mu
struct FineEntry {
  Grid g;
  double tau;
  const double* Es_a;  // spatial matrices used at Radau node 0
  const double* Es_b;  // ... at Radau node 1
  const double* mref = nullptr;  // reference mass in LDS (fill_ref_mass), or computed
  __device__ void set_mass(const double* m) { mref = m; }
  __device__ double operator()(int64_t cell, int r, int c) const {
    const int mu = r / kNs, i = r % kNs, nu = c / kNs, j = c % kNs;
    double v = 0.0;
    if (i < 18 && j < 18 && i / 9 == j / 9)
      v = kKt[mu][nu] * (mref ? mref[(i % 9) * 9 + j % 9] * g.hx * g.hy
                              : cell_mass(g, i % 9, j % 9));
    if (mu == nu) {
      const double* E = (mu == 0 ? Es_a : Es_b) + cell * (kNs * kNs);
      v += tau * kWt[mu] * E[i * kNs + j];
    }
    return v;
  }
};

struct StoredEntry {
  const double* E;  // 42 x 42 per cell
  __device__ void set_mass(const double*) {}
  __device__ double operator()(int64_t cell, int r, int c) const {
    return E[cell * (kNst * kNst) + r * kNst + c];
  }
};

// local index of patch-cell unknown l seen from the neighbour at offset (ox,oy);
// -1 if the neighbour does not carry it
__device__ __forceinline__ int map_to_neighbour(int l, int ox, int oy) {
  const int mu = l / kNs, i = l % kNs;
  if (i >= 18) return (ox == 0 && oy == 0) ? l : -1;
  const int comp = i / 9, a = i % 9;
  const int ax = a % 3 - 2 * ox, ay = a / 3 - 2 * oy;
  if (ax < 0 || ax > 2 || ay < 0 || ay > 2) return -1;
  return mu * kNs + comp * 9 + ax + 3 * ay;
}

__device__ __forceinline__ bool dropped(uint16_t mask, int l) {
  const int i = l % kNs;
  return i < 18 && !((mask >> (i % 9)) & 1u);
}

// CIP face part between patch unknowns l and m of cell (cx, cy): velocity
// unknowns of the same Radau node and component only (S: per Radau node, nm
// of them; nm = 1 for the time-diagonal form)
__device__ __forceinline__ double patch_cip(const Grid& g, const double* S, int nm, int cx, int cy,
                                            int l, int m) {
  const int mu = l / kNs, i = l % kNs, nu = m / kNs, j = m % kNs;
  if (!S || mu != nu || i >= 18 || j >= 18 || i / 9 != j / 9) return 0.0;
  const int a = i % 9, b = j % 9;
  return cip_pair(g, S, nm, nm == 1 ? 0 : mu, 2 * cx + a % 3, 2 * cy + a / 3, 2 * cx + b % 3,
                  2 * cy + b / 3);
}

// One wave (64 lanes) assembles and inverts one 42x42 patch matrix (cell
// terms from `entry`, CIP face terms from S when it is not null).
template <typename T, typename Entry>
__global__ __launch_bounds__(64) void patch_kernel(Grid g, Entry entry, const double* __restrict__ S,
                                                   const uint16_t* __restrict__ masks,
                                                   T* __restrict__ inv, int* status) {
  __shared__ double A[kNst][kNst + 1];
  __shared__ double Mref[81];
  __shared__ int s_piv[kNst];  // lane (row of the patch matrix) that is the pivot of step k
  const int64_t K = blockIdx.x;
  const int cx = (int)(K % g.nx), cy = (int)(K / g.nx);
  const int t = threadIdx.x;
  const uint16_t mask = masks ? masks[K] : (uint16_t)0x1ff;
  fill_ref_mass(Mref);
  __syncthreads();
  Entry ent = entry;
  ent.set_mass(Mref);
  for (int e = t; e < kNst * kNst; e += 64) {
    const int r = e / kNst, c = e % kNst;
    double v = 0.0;
    if (dropped(mask, r) || dropped(mask, c)) {
      v = (r == c) ? 1.0 : 0.0;
    } else {
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int nx_ = cx + ox, ny_ = cy + oy;
          if (nx_ < 0 || ny_ < 0 || nx_ >= g.nx || ny_ >= g.ny) continue;
          const int rr = map_to_neighbour(r, ox, oy), cc = map_to_neighbour(c, ox, oy);
          if (rr < 0 || cc < 0) continue;
          v += ent((int64_t)ny_ * g.nx + nx_, rr, cc);
        }
      v += patch_cip(g, S, 2, cx, cy, r, c);
    }
    A[r][c] = v;
  }
  __syncthreads();
  // Gauss-Jordan with partial pivoting, the rows in registers: lane t < 42
  // holds row t.  Pivot rows are marked, not exchanged (lane p_k is the pivot
  // of step k: largest |entry| of the current column among the rows not yet
  // used, ties to the smaller row), and every step shifts each row left by
  // one column and appends the new column of the inverse, so the current
  // column is always element 0.  At the end lane p_k holds row k of the
  // inverse, and register column j is its column p_j.
  const bool act = t < kNst;
  double row[kNst];
#pragma unroll
  for (int c = 0; c < kNst; ++c) row[c] = act ? A[t][c] : 0.0;
  bool used = !act;
  int mystep = 0;
  bool singular = false;
  for (int k = 0; k < kNst; ++k) {
    double a = used ? -1.0 : fabs(row[0]);
    int bi = used ? 64 : t;
    for (int off = 32; off > 0; off >>= 1) {
      const double oa = __shfl_xor(a, off);
      const int oi = __shfl_xor(bi, off);
      if (oa > a || (oa == a && oi < bi)) {
        a = oa;
        bi = oi;
      }
    }
    const int p = __builtin_amdgcn_readfirstlane(bi);
    if (!(a > 0.0)) singular = true;
    if (t == p) {
      used = true;
      mystep = k;
    }
    if (t == 0) s_piv[k] = p;
    const double pv = singular ? 1.0 : __shfl(row[0], p);
    const double dinv = 1.0 / pv;
    const double f = row[0];
    const bool isp = t == p;
#pragma unroll
    for (int j = 1; j < kNst; ++j) {
      const double pj = __shfl(row[j], p);
      row[j - 1] = isp ? row[j] * dinv : row[j] - f * (pj * dinv);
    }
    row[kNst - 1] = isp ? dinv : -f * dinv;
  }
  __syncthreads();
  if (singular && t == 0) atomicOr(status, 1);
  // store the inverse column-major, dropped rows/columns zeroed
  T* out = inv + patch_slot(g, cx, cy) * (kNst * kNst);
  if (act) {
#pragma unroll
    for (int j = 0; j < kNst; ++j) {
      const int col = s_piv[j];
      const bool z = dropped(mask, mystep) || dropped(mask, col);
      out[col * kNst + mystep] = z ? (T)0 : (T)row[j];
    }
  }
}

// Level-0 surrogate patch in time-diagonal form: C = lam M_K + tau J_K with
// M_K, J_K the spatial mass and surrogate matrix restricted to the patch
// (neighbour contributions included); one wave inverts C by complex
// Gauss-Jordan with partial pivoting.
template <typename T>
__global__ __launch_bounds__(64) void patch_complex_kernel(Grid g, double tau,
                                                           const double* __restrict__ Es,
                                                           const double* __restrict__ Sr,
                                                           const uint16_t* __restrict__ masks,
                                                           T* __restrict__ inv, int* status) {
  __shared__ double Ar[kNs][2 * kNs + 1], Ai[kNs][2 * kNs + 1];
  __shared__ double fr[kNs], fi[kNs];
  __shared__ double Mref[81];
  const int64_t K = blockIdx.x;
  const int cx = (int)(K % g.nx), cy = (int)(K / g.nx);
  const int t = threadIdx.x;
  const uint16_t mask = masks ? masks[K] : (uint16_t)0x1ff;
  fill_ref_mass(Mref);
  __syncthreads();
  for (int e = t; e < kNs * kNs; e += 64) {
    const int r = e / kNs, c = e % kNs;
    double cr = 0.0, ci = 0.0;
    if (dropped(mask, r) || dropped(mask, c)) {
      cr = (r == c) ? 1.0 : 0.0;
    } else {
      double jv = 0.0, mv = 0.0;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int nx_ = cx + ox, ny_ = cy + oy;
          if (nx_ < 0 || ny_ < 0 || nx_ >= g.nx || ny_ >= g.ny) continue;
          const int rr = map_to_neighbour(r, ox, oy), cc = map_to_neighbour(c, ox, oy);
          if (rr < 0 || cc < 0) continue;
          const int64_t nb = (int64_t)ny_ * g.nx + nx_;
          jv += Es[nb * (kNs * kNs) + rr * kNs + cc];
          if (rr < 18 && cc < 18 && rr / 9 == cc / 9)
            mv += Mref[(rr % 9) * 9 + cc % 9] * g.hx * g.hy;
        }
      jv += patch_cip(g, Sr, 1, cx, cy, r, c);
      cr = kLamRe * mv + tau * jv;
      ci = kLamIm * mv;
    }
    Ar[r][c] = cr;
    Ai[r][c] = ci;
    Ar[r][kNs + c] = (r == c) ? 1.0 : 0.0;
    Ai[r][kNs + c] = 0.0;
  }
  __syncthreads();
  // complex Gauss-Jordan with partial pivoting on [C | I]; lane t owns column t
  // of the augmented matrix, the pivot comes from a wave reduction
  bool singular = false;
  for (int k = 0; k < kNs; ++k) {
    double bv = -1.0;
    int bi = k;
    if (t >= k && t < kNs) {
      bv = Ar[t][k] * Ar[t][k] + Ai[t][k] * Ai[t][k];
      bi = t;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const int p = bi;
    if (!(bv > 0.0)) singular = true;
    __syncthreads();
    for (int c = t; c < 2 * kNs; c += 64) {
      const double tr = Ar[k][c], ti = Ai[k][c];
      Ar[k][c] = Ar[p][c];
      Ai[k][c] = Ai[p][c];
      Ar[p][c] = tr;
      Ai[p][c] = ti;
    }
    __syncthreads();
    double pr = Ar[k][k], pi = Ai[k][k];
    if (singular) { pr = 1.0; pi = 0.0; }
    const double den = pr * pr + pi * pi;
    const double qr = pr / den, qi = -pi / den;  // 1 / pivot
    __syncthreads();
    for (int c = t; c < 2 * kNs; c += 64) {
      const double ar = Ar[k][c], ai = Ai[k][c];
      Ar[k][c] = ar * qr - ai * qi;
      Ai[k][c] = ar * qi + ai * qr;
    }
    if (t < kNs) {
      fr[t] = (t == k) ? 0.0 : Ar[t][k];
      fi[t] = (t == k) ? 0.0 : Ai[t][k];
    }
    __syncthreads();
    for (int c = t; c < 2 * kNs; c += 64) {
      const double br = Ar[k][c], bi2 = Ai[k][c];
      for (int r = 0; r < kNs; ++r)
        if (r != k) {
          Ar[r][c] -= fr[r] * br - fi[r] * bi2;
          Ai[r][c] -= fr[r] * bi2 + fi[r] * br;
        }
    }
    __syncthreads();
  }
  if (singular && t == 0) atomicOr(status, 1);
  T* out = inv + patch_slot(g, cx, cy) * (2 * kNs * kNs);
  for (int e = t; e < kNs * kNs; e += 64) {
    const int c = e / kNs, r = e % kNs;
    const bool z = dropped(mask, r) || dropped(mask, c);
    out[2 * e] = z ? (T)0 : (T)Ar[r][kNs + c];
    out[2 * e + 1] = z ? (T)0 : (T)Ai[r][kNs + c];
  }
}

template <typename T>
__global__ void transpose_convert_kernel(Grid g, const double* __restrict__ E,
                                         T* __restrict__ Et) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nc * kNst * kNst) return;
  const int64_t c = i / (kNst * kNst);
  const int e = (int)(i % (kNst * kNst));
  const int col = e / kNst, row = e % kNst;  // output index = col*42 + row
  const int64_t slot = patch_slot(g, (int)(c % g.nx), (int)(c / g.nx));
  Et[slot * (kNst * kNst) + e] = (T)E[c * (kNst * kNst) + row * kNst + col];
}

// ---------------------------------------------------------------- Galerkin

// local prolongation of child (ox,oy) of a coarse cell: fine local unknown
// (row) from coarse local unknowns (column), identity in time
__device__ double prolong_entry(int rf, int cc, int ox, int oy) {
  const int muf = rf / kNs, i = rf % kNs, muc = cc / kNs, j = cc % kNs;
  if (muf != muc) return 0.0;
  if (i < 18 && j < 18) {
    if (i / 9 != j / 9) return 0.0;
    const int af = i % 9, ac = j % 9;
    const double sx = 0.5 * ox + 0.25 * (af % 3), sy = 0.5 * oy + 0.25 * (af / 3);
    return q2v(ac % 3, sx) * q2v(ac / 3, sy);
  }
  if (i >= 18 && j >= 18) {
    const int pf = i - 18, pc = j - 18;
    if (pf == 0) return pc == 0 ? 1.0 : (pc == 1 ? 0.5 * (ox - 0.5) : 0.5 * (oy - 0.5));
    return pf == pc ? 0.5 : 0.0;
  }
  return 0.0;
}

template <typename Entry>
__global__ __launch_bounds__(256) void galerkin_kernel(Grid gc, Grid gf, Entry fine_entry,
                                                       double* __restrict__ Ec) {
  __shared__ double Pf[kNst][kNst + 1];
  __shared__ double Ef[kNst][kNst + 1];
  __shared__ double Tm[kNst][kNst + 1];
  __shared__ double Mref[81];
  const int64_t C = blockIdx.x;
  const int cx = (int)(C % gc.nx), cy = (int)(C / gc.nx);
  const int t = threadIdx.x;
  fill_ref_mass(Mref);
  __syncthreads();
  Entry fe = fine_entry;
  fe.set_mass(Mref);
  constexpr int kPer = (kNst * kNst + 255) / 256;
  double accv[kPer];
  for (int q = 0; q < kPer; ++q) accv[q] = 0.0;
  for (int ch = 0; ch < 4; ++ch) {
    const int ox = ch & 1, oy = ch >> 1;
    const int64_t f = (int64_t)(2 * cy + oy) * gf.nx + (2 * cx + ox);
    for (int e = t; e < kNst * kNst; e += 256) {
      const int r = e / kNst, c = e % kNst;
      Pf[r][c] = prolong_entry(r, c, ox, oy);
      Ef[r][c] = fe(f, r, c);
    }
    __syncthreads();
    for (int e = t; e < kNst * kNst; e += 256) {  // Tm = Ef Pf
      const int r = e / kNst, c = e % kNst;
      double s = 0.0;
      for (int k = 0; k < kNst; ++k) s += Ef[r][k] * Pf[k][c];
      Tm[r][c] = s;
    }
    __syncthreads();
    for (int q = 0; q < kPer; ++q) {  // Ec += Pf^T Tm
      const int e = t + 256 * q;
      if (e < kNst * kNst) {
        const int r = e / kNst, c = e % kNst;
        double s = 0.0;
        for (int k = 0; k < kNst; ++k) s += Pf[k][r] * Tm[k][c];
        accv[q] += s;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < kPer; ++q) {
    const int e = t + 256 * q;
    if (e < kNst * kNst) Ec[C * (kNst * kNst) + e] = accv[q];
  }
}

// ------------------------------------------------------------ coarsest level

// dense row r of the assembled level operator (thread per row)
__global__ void coarse_assemble_kernel(Grid g, const double* __restrict__ E,
                                       double* __restrict__ A) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.nst) return;
  const int64_t n = g.nst;
  const int mu = (int)(r / g.ns);
  const int64_t s = r % g.ns;
  const int NX = 2 * g.nx + 1;
  int cxs[2], cys[2], ncx = 0, ncy = 0, lrow_fixed = -1;
  int gx = 0, gy = 0, comp = 0;
  if (s < g.nv) {
    comp = (int)(s / g.nn);
    const int64_t node = s % g.nn;
    gx = (int)(node % NX);
    gy = (int)(node / NX);
    if (gx % 2 == 0) {
      if (gx / 2 - 1 >= 0) cxs[ncx++] = gx / 2 - 1;
      if (gx / 2 < g.nx) cxs[ncx++] = gx / 2;
    } else {
      cxs[ncx++] = (gx - 1) / 2;
    }
    if (gy % 2 == 0) {
      if (gy / 2 - 1 >= 0) cys[ncy++] = gy / 2 - 1;
      if (gy / 2 < g.ny) cys[ncy++] = gy / 2;
    } else {
      cys[ncy++] = (gy - 1) / 2;
    }
  } else {
    const int64_t cell = (s - g.nv) / 3;
    cxs[ncx++] = (int)(cell % g.nx);
    cys[ncy++] = (int)(cell / g.nx);
    lrow_fixed = mu * kNs + 18 + (int)((s - g.nv) % 3);
  }
  for (int iy = 0; iy < ncy; ++iy)
    for (int ix = 0; ix < ncx; ++ix) {
      const int cx = cxs[ix], cy = cys[iy];
      const int lr = lrow_fixed >= 0
                         ? lrow_fixed
                         : mu * kNs + comp * 9 + (gx - 2 * cx) + 3 * (gy - 2 * cy);
      const double* Er = E + ((int64_t)cy * g.nx + cx) * (kNst * kNst) + (int64_t)lr * kNst;
      for (int lc = 0; lc < kNst; ++lc) A[r * n + st_global_index(g, cx, cy, lc)] += Er[lc];
    }
}

__global__ void pin_kernel(int64_t n, double* A, const int64_t* pin, int npin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < npin; ++k) {
    const int64_t p = pin[k];
    A[p * n + i] = (i == p) ? 1.0 : 0.0;
    A[i * n + p] = (i == p) ? 1.0 : 0.0;
  }
}

// Blocked Gauss-Jordan inversion, in place, partial row pivoting.
// Panels of kGjNb columns K: (1) the panel is copied to a contiguous
// column-major buffer P (n x kb) and eliminated column by column over all
// rows (one launch per column, below; for n <= kGjSmallRows panels of
// kGjSmallNb columns are eliminated in one workgroup instead); (2) its row swaps
// are applied to every other column; (3) with T = rows K of the other columns,
// every other column is updated as A[:,C] = [0 on rows K; A[O,C]] + P T, which
// is the block form of the Gauss-Jordan step; (4) the panel is written back.
// At the end the columns are permuted back in reverse pivot order.

__global__ void gj_panel_in_kernel(int64_t n, int64_t k0, int kb, const double* __restrict__ A,
                                   double* __restrict__ P) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int j = 0; j < kb; ++j) P[(int64_t)j * n + r] = A[r * n + k0 + j];
}

__global__ void gj_panel_out_kernel(int64_t n, int64_t k0, int kb, double* __restrict__ A,
                                    const double* __restrict__ P) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int j = 0; j < kb; ++j) A[r * n + k0 + j] = P[(int64_t)j * n + r];
}

// Panel elimination, one launch per column.  Workgroup b owns rows
// 64 b .. 64 b + 63 of the panel (one row per lane, the four waves take a
// quarter of the panel's columns each).  Step jc reads the panel from Pin and
// writes it whole to Pout (two copies, so no workgroup reads what another one
// is writing): the pivot row p of column jc comes from the per-block maxima
// left by the previous step (largest |P[jc][r]| over the rows r >= c not yet
// used as pivots, ties to the smaller row); the new row c is old row p scaled
// by 1 / pivot (its pivot entry becomes 1 / pivot), row p takes old row c, and
// every other row subtracts its column-jc entry times the new row c (its
// column-jc entry becomes -entry / pivot): the Gauss-Jordan step with the
// interchange folded in.  The wave holding column jc + 1 leaves its block's
// maximum for the next step.
constexpr int kGjQ = kGjNb / 4;  // panel columns per wave

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// block maxima of column 0 of the panel over the rows r >= k0
__global__ __launch_bounds__(64) void gj_partials0_kernel(int64_t n, int64_t k0,
                                                          const double* __restrict__ P,
                                                          double* __restrict__ bv,
                                                          int* __restrict__ bi) {
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  double v = (r < n && r >= k0) ? fabs(P[r]) : -1.0;
  int i = (int)r;
  wave_argmax(v, i);
  if (threadIdx.x == 0) {
    bv[blockIdx.x] = v;
    bi[blockIdx.x] = i;
  }
}

__global__ __launch_bounds__(256) void gj_panel_step_kernel(
    int64_t n, int64_t k0, int kb, int jc, const double* __restrict__ Pin, double* __restrict__ Pout,
    const double* __restrict__ bv_in, const int* __restrict__ bi_in, double* __restrict__ bv_out,
    int* __restrict__ bi_out, int nblk, int* piv, int* status) {
  __shared__ double oc[kGjNb], op[kGjNb];
  __shared__ double s_pv;
  __shared__ int s_p;
  const int64_t c = k0 + jc;
  const int t = threadIdx.x, lane = t & 63, q = t >> 6;
  if (t < 64) {
    double v = -1.0;
    int i = (int)c;
    for (int b = lane; b < nblk; b += 64) {
      const double w = bv_in[b];
      const int wi = bi_in[b];
      if (w > v || (w == v && wi < i)) {
        v = w;
        i = wi;
      }
    }
    wave_argmax(v, i);
    if (lane == 0) {
      const bool sing = !(v > 0.0);
      s_p = sing ? (int)c : i;
      s_pv = sing ? 1.0 : Pin[(int64_t)jc * n + i];
      if (blockIdx.x == 0) {
        piv[c] = s_p;
        if (sing) atomicOr(status, 2);
      }
    }
  }
  __syncthreads();
  const int64_t p = s_p;
  if (t < kb) {
    oc[t] = Pin[(int64_t)t * n + c];
    op[t] = Pin[(int64_t)t * n + p];
  }
  __syncthreads();
  const double dinv = 1.0 / s_pv;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  double mine = -1.0;
  if (r < n) {
    // all of this thread's loads first, then the update and the stores
    const int j0 = q * kGjQ;
    double v[kGjQ];
#pragma unroll
    for (int u = 0; u < kGjQ; ++u)
      v[u] = (j0 + u < kb && r != p) ? Pin[(int64_t)(j0 + u) * n + r] : 0.0;
    const double f = r == p ? oc[jc] : Pin[(int64_t)jc * n + r];
#pragma unroll
    for (int u = 0; u < kGjQ; ++u) {
      const int j = j0 + u;
      if (j >= kb) break;
      const double nc = (j == jc ? 1.0 : op[j]) * dinv;
      double out;
      if (r == c) {
        out = nc;
      } else {
        double base = r == p ? oc[j] : v[u];
        if (j == jc) base = 0.0;
        out = base - f * nc;
      }
      Pout[(int64_t)j * n + r] = out;
      if (j == jc + 1 && r > c) mine = fabs(out);
    }
  }
  if (jc + 1 < kb && q == (jc + 1) / kGjQ) {
    int i = (int)r;
    wave_argmax(mine, i);
    if (lane == 0) {
      bv_out[blockIdx.x] = mine;
      bi_out[blockIdx.x] = i;
    }
  }
}

// Small matrices (n <= kGjSmallRows, e.g. an 8 x 8 coarsest level): the
// elimination of a whole panel of kb <= kGjSmallNb columns in one workgroup,
// the panel held in registers (rows t and t + 1024 of thread t), instead of
// one launch per column.  Same pivot rule (largest |entry| over the rows
// r >= c, ties to the smaller row) and the same exchange step as
// gj_panel_step_kernel, column after column with workgroup barriers; the
// panel is read from A and written, eliminated, to P (column-major n x kb).
constexpr int kGjSmallNb = 16;
constexpr int kGjSmallThreads = 1024;
constexpr int kGjSmallR = 2;
constexpr int64_t kGjSmallRows = (int64_t)kGjSmallThreads * kGjSmallR;

// argmax of |value| over the wave, ties to the smaller row; carries the value
__device__ __forceinline__ void wave_argmax_val(double& a, int& i, double& val) {
  for (int off = 32; off > 0; off >>= 1) {
    const double oa = __shfl_xor(a, off);
    const int oi = __shfl_xor(i, off);
    const double ov = __shfl_xor(val, off);
    if (oa > a || (oa == a && oi < i)) {
      a = oa;
      i = oi;
      val = ov;
    }
  }
}

__global__ __launch_bounds__(kGjSmallThreads) void gj_panel_small_kernel(
    int64_t n, int64_t k0, int kb, const double* __restrict__ A, double* __restrict__ P,
    int* __restrict__ piv, int* __restrict__ status) {
  __shared__ double wa[kGjSmallThreads / 64], wvl[kGjSmallThreads / 64];
  __shared__ int wi[kGjSmallThreads / 64];
  __shared__ double oc[kGjSmallNb], op[kGjSmallNb];
  __shared__ double s_pv;
  __shared__ int s_p;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double v[kGjSmallR][kGjSmallNb];
  int64_t row[kGjSmallR];
#pragma unroll
  for (int i = 0; i < kGjSmallR; ++i) {
    row[i] = t + (int64_t)i * kGjSmallThreads;
#pragma unroll
    for (int j = 0; j < kGjSmallNb; ++j)
      v[i][j] = (row[i] < n && j < kb) ? A[row[i] * n + k0 + j] : 0.0;
  }
#pragma unroll
  for (int jc = 0; jc < kGjSmallNb; ++jc) {
    if (jc < kb) {  // uniform over the workgroup
    const int64_t c = k0 + jc;
    // pivot: largest |entry| of column jc over the rows r >= c
    double a = -1.0, val = 0.0;
    int bi = (int)c;
#pragma unroll
    for (int i = 0; i < kGjSmallR; ++i) {
      if (row[i] < n && row[i] >= c) {
        const double x = fabs(v[i][jc]);
        if (x > a || (x == a && row[i] < bi)) {
          a = x;
          bi = (int)row[i];
          val = v[i][jc];
        }
      }
    }
    wave_argmax_val(a, bi, val);
    if (lane == 0) {
      wa[w] = a;
      wi[w] = bi;
      wvl[w] = val;
    }
    __syncthreads();
    if (t < 64) {
      double aa = t < kGjSmallThreads / 64 ? wa[t] : -1.0;
      int ii = t < kGjSmallThreads / 64 ? wi[t] : (int)c;
      double vv = t < kGjSmallThreads / 64 ? wvl[t] : 0.0;
      wave_argmax_val(aa, ii, vv);
      if (t == 0) {
        const bool sing = !(aa > 0.0);
        s_p = sing ? (int)c : ii;
        s_pv = sing ? 1.0 : vv;
        piv[c] = s_p;
        if (sing) atomicOr(status, 2);
      }
    }
    __syncthreads();
    const int64_t p = s_p;
    // old rows c and p of the panel
#pragma unroll
    for (int i = 0; i < kGjSmallR; ++i) {
      if (row[i] == c) {
#pragma unroll
        for (int j = 0; j < kGjSmallNb; ++j) oc[j] = v[i][j];
      }
      if (row[i] == p) {
#pragma unroll
        for (int j = 0; j < kGjSmallNb; ++j) op[j] = v[i][j];
      }
    }
    __syncthreads();
    const double dinv = 1.0 / s_pv;
#pragma unroll
    for (int i = 0; i < kGjSmallR; ++i) {
      if (row[i] >= n) continue;
      const bool isc = row[i] == c, isp = row[i] == p;
      const double f = isp ? oc[jc] : v[i][jc];
#pragma unroll
      for (int j = 0; j < kGjSmallNb; ++j) {
        const double nc = (j == jc ? 1.0 : op[j]) * dinv;
        double out;
        if (isc) {
          out = nc;
        } else {
          double base = isp ? oc[j] : v[i][j];
          if (j == jc) base = 0.0;
          out = base - f * nc;
        }
        v[i][j] = out;
      }
    }
    __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < kGjSmallR; ++i) {
    if (row[i] >= n) continue;
#pragma unroll
    for (int j = 0; j < kGjSmallNb; ++j)
      if (j < kb) P[(int64_t)j * n + row[i]] = v[i][j];
  }
}

// row swaps of the panel applied to column j (outside the panel), in order;
// then T = rows K of that column
__global__ void gj_rowswap_copy_kernel(int64_t n, int64_t k0, int kb, double* __restrict__ A,
                                       const int* __restrict__ piv, double* __restrict__ T) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + kb)) return;
  for (int q = 0; q < kb; ++q) {
    const int64_t c = k0 + q, p = piv[c];
    if (p != c) {
      const double a = A[c * n + j];
      A[c * n + j] = A[p * n + j];
      A[p * n + j] = a;
    }
  }
  for (int q = 0; q < kb; ++q) T[(int64_t)q * n + j] = A[(k0 + q) * n + j];
}

// A[:,C] = [0 on rows K; A[O,C]] + P T on the FP64 matrix cores.  64 x 64
// output tile per workgroup (in the compressed column space that skips the
// panel), each wave a 32 x 32 quarter held as 2 x 2 accumulator tiles of
// v_mfma_f64_16x16x4f64: in a 16 x 16 tile lane l holds rows l/16 + 4 r
// (r = 0..3) of column l%16; the A operand of a 16 x 4 block is row l%16,
// k = l/16, the B operand of a 4 x 16 block k = l/16, column l%16.  The old
// entries (zero on the rows K) are loaded first into registers of their own
// and added after the products, so their latency overlaps the staging and the
// matrix-core work; the tile's rows of P and columns of T pass through LDS in
// chunks of 16 k,
// double-buffered: the loads of chunk c + 1 are in flight while the matrix
// cores work on chunk c (zero beyond kb and beyond the matrix).  32 KB of LDS
// and a small register budget let several workgroups share a CU.
// Tile order: workgroups are dealt round-robin to the 8 XCDs, so each XCD is
// given a contiguous run of a sequence that walks all row tiles for a group
// of kGjGc column tiles at a time (kGjGc consecutive tiles share a row tile):
// the group's T tiles stay in the XCD's L2 and each P tile is fetched once
// per group instead of once per tile.
typedef double gj_d4 __attribute__((ext_vector_type(4)));
constexpr int kGjKc = 16;  // k per staged chunk
constexpr int kGjGc = 8;   // column tiles per group

__global__ __launch_bounds__(256) void gj_update_kernel(int64_t n, int64_t k0, int kb,
                                                        double* __restrict__ A,
                                                        const double* __restrict__ P,
                                                        const double* __restrict__ T,
                                                        int row_tiles, int col_groups,
                                                        int col_tiles) {
  __shared__ double As[2][kGjKc][64];  // [buffer][k][row of the tile]
  __shared__ double Bs[2][kGjKc][64];  // [buffer][k][column of the tile]
  const int64_t seq = (int64_t)row_tiles * col_groups * kGjGc;
  const int64_t per_xcd = (seq + 7) >> 3;
  const int64_t pos = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (pos >= seq) return;
  const int64_t grp = pos / ((int64_t)row_tiles * kGjGc), rem = pos % ((int64_t)row_tiles * kGjGc);
  const int64_t ctile = grp * kGjGc + rem % kGjGc, rtile = rem / kGjGc;
  if (ctile >= col_tiles) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int lr = l >> 4, lc = l & 15;
  const int wr = w >> 1, wc = w & 1;
  const int64_t row0 = rtile * 64;
  const int64_t m = n - kb;  // > 0: the update is launched only then
  const int64_t ccol0 = ctile * 64;
  // column of A for a compressed column (clamped into [0, m))
  auto acol = [&](int64_t cc) -> int64_t {
    const int64_t c = cc < m ? cc : m - 1;
    return c < k0 ? c : c + kb;
  };
  double Aold[2][2][4];
  gj_d4 C[2][2];
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const int64_t col = acol(ccol0 + 32 * wc + 16 * J + lc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 32 * wr + 16 * I + lr + 4 * r;
        Aold[I][J][r] = A[(row < n ? row : n - 1) * n + col];
        C[I][J][r] = 0.0;
      }
    }
  // this thread's share of a chunk: entries e = t + 256 u of the 16 x 64
  // blocks of P and T
  constexpr int kU = kGjKc * 64 / 256;
  const int i0 = t & 63;
  const int64_t r_ld = row0 + i0, cc_ld = ccol0 + i0;
  const int64_t r_cl = r_ld < n ? r_ld : n - 1;
  const int64_t c_cl = acol(cc_ld);
  double pa[kU], tb[kU];
  auto load_chunk = [&](int ch) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = ch * kGjKc + (t >> 6) + 4 * u;
      const int kc = k < kb ? k : kb - 1;
      const double pv = P[(int64_t)kc * n + r_cl];
      const double tv = T[(int64_t)kc * n + c_cl];
      pa[u] = (k < kb && r_ld < n) ? pv : 0.0;
      tb[u] = (k < kb && cc_ld < m) ? tv : 0.0;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      As[buf][(t >> 6) + 4 * u][i0] = pa[u];
      Bs[buf][(t >> 6) + 4 * u][i0] = tb[u];
    }
  };
  const int nch = (kb + kGjKc - 1) / kGjKc;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) load_chunk(ch + 1);
#pragma unroll
    for (int q = 0; q < kGjKc / 4; ++q) {
      const int k = 4 * q + lr;
      const double a0 = As[buf][k][32 * wr + lc], a1 = As[buf][k][32 * wr + 16 + lc];
      const double b0 = Bs[buf][k][32 * wc + lc], b1 = Bs[buf][k][32 * wc + 16 + lc];
      C[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, C[0][0], 0, 0, 0);
      C[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, C[0][1], 0, 0, 0);
      C[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, C[1][0], 0, 0, 0);
      C[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, C[1][1], 0, 0, 0);
    }
    if (ch + 1 < nch) store_chunk(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const int64_t cc = ccol0 + 32 * wc + 16 * J + lc;
      if (cc >= m) continue;
      const int64_t col = acol(cc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 32 * wr + 16 * I + lr + 4 * r;
        const bool inK = row >= k0 && row < k0 + kb;
        if (row < n) A[row * n + col] = inK ? C[I][J][r] : Aold[I][J][r] + C[I][J][r];
      }
    }
}

// columns back in reverse pivot order (thread per row)
__global__ void gj_colperm_kernel(int64_t n, double* __restrict__ A, const int* __restrict__ piv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double* row = A + r * n;
  for (int64_t c = n - 1; c >= 0; --c) {
    const int64_t p = piv[c];
    if (p != c) {
      const double a = row[c];
      row[c] = row[p];
      row[p] = a;
    }
  }
}

__global__ __launch_bounds__(256) void form_fine_st_kernel(Grid g, FineEntry e, double* __restrict__ E) {
  const int64_t cell = blockIdx.x;
  for (int idx = threadIdx.x; idx < kNst * kNst; idx += blockDim.x)
    E[cell * (kNst * kNst) + idx] = e(cell, idx / kNst, idx % kNst);
}

}  // namespace

hipError_t launch_form_fine_st(const Grid& g, double tau, const double* Es0, const double* Es1,
                               double* E, hipStream_t s) {
  FineEntry e{g, tau, Es0, Es1};
  hipLaunchKernelGGL(form_fine_st_kernel, dim3((unsigned)g.nc), dim3(256), 0, s, g, e, E);
  return hipGetLastError();
}

hipError_t launch_element_matrices(const Grid& g, const Model& m, const double* u, int lslot,
                                   double* Es, hipStream_t s) {
  hipLaunchKernelGGL(element_matrix_kernel, dim3((unsigned)g.nc), dim3(256), 0, s, g, m, u, lslot,
                     Es);
  return hipGetLastError();
}

hipError_t launch_state_combine(int64_t n, const double* u0, const double* u1, double a0,
                                double a1, double* out, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, u0, u1,
                     a0, a1, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convert(int64_t n, const double* in, T* out, hipStream_t s) {
  hipLaunchKernelGGL(convert_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fine_patches(const Grid& g, double tau, const double* Es, const double* Sr,
                               const uint16_t* masks, T* inv, int* status, hipStream_t s) {
  hipLaunchKernelGGL(patch_complex_kernel<T>, dim3((unsigned)g.nc), dim3(64), 0, s, g, tau, Es,
                     Sr, masks, inv, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_exact_fine_patches(const Grid& g, double tau, const double* Es0,
                                     const double* Es1, const double* S, const uint16_t* masks,
                                     T* inv, int* status, hipStream_t s) {
  FineEntry e{g, tau, Es0, Es1};
  hipLaunchKernelGGL((patch_kernel<T, FineEntry>), dim3((unsigned)g.nc), dim3(64), 0, s, g, e, S,
                     masks, inv, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose_convert(const Grid& g, const double* E, T* Et, hipStream_t s) {
  const int64_t n = g.nc * kNst * kNst;
  hipLaunchKernelGGL(transpose_convert_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, g, E, Et);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_patches(const Grid& g, const double* E, const double* S, T* inv,
                                int* status, hipStream_t s) {
  StoredEntry e{E};
  hipLaunchKernelGGL((patch_kernel<T, StoredEntry>), dim3((unsigned)g.nc), dim3(64), 0, s, g, e, S,
                     (const uint16_t*)nullptr, inv, status);
  return hipGetLastError();
}

hipError_t launch_galerkin_from_fine(const Grid& gc, double tau, const double* Es0,
                                     const double* Es1, double* Ec, hipStream_t s) {
  Grid gf = make_grid(2 * gc.nx, 2 * gc.ny, 2 * gc.nx * (gc.hx / 2), 2 * gc.ny * (gc.hy / 2));
  FineEntry e{gf, tau, Es0, Es1};
  hipLaunchKernelGGL((galerkin_kernel<FineEntry>), dim3((unsigned)gc.nc), dim3(256), 0, s, gc, gf,
                     e, Ec);
  return hipGetLastError();
}

hipError_t launch_galerkin(const Grid& gc, const double* Ef, double* Ec, hipStream_t s) {
  Grid gf = make_grid(2 * gc.nx, 2 * gc.ny, 2 * gc.nx * (gc.hx / 2), 2 * gc.ny * (gc.hy / 2));
  StoredEntry e{Ef};
  hipLaunchKernelGGL((galerkin_kernel<StoredEntry>), dim3((unsigned)gc.nc), dim3(256), 0, s, gc,
                     gf, e, Ec);
  return hipGetLastError();
}

hipError_t launch_coarse_assemble(const Grid& g, const double* E, double* A, hipStream_t s) {
  hipLaunchKernelGGL(coarse_assemble_kernel, dim3((unsigned)((g.nst + 127) / 128)), dim3(128), 0,
                     s, g, E, A);
  return hipGetLastError();
}

hipError_t launch_pin(int64_t n, double* A, const int64_t* pin, int npin, hipStream_t s) {
  hipLaunchKernelGGL(pin_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, A, pin,
                     npin);
  return hipGetLastError();
}

// work: coarse_invert_work_doubles(n) doubles (two panel copies, the row block
// T, the per-block pivot candidates); piv: n ints
hipError_t coarse_invert(int64_t n, double* A, double* work, int* piv, int* status,
                         hipStream_t s) {
  double* P[2] = {work, work + (int64_t)2 * kGjNb * n};
  double* T = work + (int64_t)kGjNb * n;
  const int nblk = (int)((n + 63) / 64);
  double* bv[2] = {work + (int64_t)3 * kGjNb * n, work + (int64_t)3 * kGjNb * n + nblk};
  int* bi[2] = {(int*)(work + (int64_t)3 * kGjNb * n + 2 * nblk),
                (int*)(work + (int64_t)3 * kGjNb * n + 2 * nblk) + nblk};
  const unsigned nb = (unsigned)((n + 255) / 256);
  // small matrices: narrow panels eliminated in one workgroup each
  const bool small = n <= kGjSmallRows;
  const int width = small ? kGjSmallNb : kGjNb;
  for (int64_t k0 = 0; k0 < n; k0 += width) {
    const int kb = (int)((n - k0) < width ? (n - k0) : width);
    double* Pf;
    if (small) {
      hipLaunchKernelGGL(gj_panel_small_kernel, dim3(1), dim3(kGjSmallThreads), 0, s, n, k0, kb,
                         (const double*)A, P[0], piv, status);
      Pf = P[0];
    } else {
      hipLaunchKernelGGL(gj_panel_in_kernel, dim3(nb), dim3(256), 0, s, n, k0, kb, A, P[0]);
      hipLaunchKernelGGL(gj_partials0_kernel, dim3((unsigned)nblk), dim3(64), 0, s, n, k0,
                         (const double*)P[0], bv[0], bi[0]);
      for (int jc = 0; jc < kb; ++jc) {
        const int a = jc & 1, b = a ^ 1;
        hipLaunchKernelGGL(gj_panel_step_kernel, dim3((unsigned)nblk), dim3(256), 0, s, n, k0, kb,
                           jc, (const double*)P[a], P[b], (const double*)bv[a], (const int*)bi[a],
                           bv[b], bi[b], nblk, piv, status);
      }
      Pf = P[kb & 1];
    }
    const int64_t m = n - kb;
    if (m > 0) {
      hipLaunchKernelGGL(gj_rowswap_copy_kernel, dim3(nb), dim3(256), 0, s, n, k0, kb, A, piv, T);
      const int rt = (int)((n + 63) / 64), ct = (int)((m + 63) / 64);
      const int cg = (ct + kGjGc - 1) / kGjGc;
      const int64_t seq = (int64_t)rt * cg * kGjGc;
      const unsigned nwg = (unsigned)(((seq + 7) >> 3) * 8);
      hipLaunchKernelGGL(gj_update_kernel, dim3(nwg), dim3(256), 0, s, n, k0, kb, A,
                         (const double*)Pf, (const double*)T, rt, cg, ct);
    }
    hipLaunchKernelGGL(gj_panel_out_kernel, dim3(nb), dim3(256), 0, s, n, k0, kb, A,
                       (const double*)Pf);
  }
  hipLaunchKernelGGL(gj_colperm_kernel, dim3(nb), dim3(256), 0, s, n, A, piv);
  return hipGetLastError();
}

template hipError_t launch_convert<double>(int64_t, const double*, double*, hipStream_t);
template hipError_t launch_convert<float>(int64_t, const double*, float*, hipStream_t);
template hipError_t launch_fine_patches<double>(const Grid&, double, const double*, const double*,
                                                const uint16_t*, double*, int*, hipStream_t);
template hipError_t launch_fine_patches<float>(const Grid&, double, const double*, const double*,
                                               const uint16_t*, float*, int*, hipStream_t);
template hipError_t launch_exact_fine_patches<double>(const Grid&, double, const double*,
                                                      const double*, const double*,
                                                      const uint16_t*, double*, int*, hipStream_t);
template hipError_t launch_exact_fine_patches<float>(const Grid&, double, const double*,
                                                     const double*, const double*,
                                                     const uint16_t*, float*, int*, hipStream_t);
template hipError_t launch_transpose_convert<double>(const Grid&, const double*, double*, hipStream_t);
template hipError_t launch_transpose_convert<float>(const Grid&, const double*, float*, hipStream_t);
template hipError_t launch_level_patches<double>(const Grid&, const double*, const double*,
                                                 double*, int*, hipStream_t);
template hipError_t launch_level_patches<float>(const Grid&, const double*, const double*, float*,
                                                int*, hipStream_t);

}  // namespace pns
