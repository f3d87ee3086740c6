/*
 * pns_oracle.c -- plain FP64 CPU oracle for the space-time (p,delta)-Navier-Stokes
 * smoothing step.  TEST INFRASTRUCTURE ONLY: this file is compiled into
 * liboracle.so and loaded by tests, by the smoke check and by the CPU baseline
 * leg of the benchmark.  No product code links, loads or calls it, and it shares
 * no source, header, table or helper with the HIP path.
 *
 * What is computed (Margenberg & Mehlmann, arXiv 2603.28706):
 *   - the (p,delta) stress law, eq. (constitutive-law), and the three
 *     constitutive tangents: Picard eq. (local-tangent-picard), exact Newton
 *     eq. (local-tangent-exact), stress-clipped modified Newton
 *     eq. (local-tangent-clip) (Sec. 4.2-4.4);
 *   - the spatial linearisation J_mu of the slab residual on Q2 / P1disc,
 *     cell by cell, including the volume terms of eq. (pns-form) and the
 *     boundary terms of eq. (def-a-gam), eq. (Defc) and eq. (def-b-gam)
 *     (Sec. 3.2), for one Gauss-Radau node;
 *   - the slab Jacobian action eq. (slab-underint-jac) and the slab residual
 *     eq. (slab-underint) (Sec. 5.2);
 *
 * Style: per-cell quadrature loops that evaluate every basis function at every
 * quadrature point.  No sum factorisation, no blocking, no fusion.  Element
 * matrices are formed entry by entry from the bilinear form and then multiplied
 * by the local vector.
 *
 * Readings where the paper is silent (each one listed in the design notes):
 *   - Dirichlet data on all of the boundary, given by a lifting ghat_D: a Q2
 *     velocity field per Radau node (NULL: homogeneous data).  g_D is its
 *     trace; the frozen Nitsche coefficients of eq. (def-b-gam) are eta(G) and
 *     the exact stress derivative DS(G) at G = D ghat_D, evaluated at each face
 *     point from the boundary cell's field (G = 0 for homogeneous data:
 *     eta_D = nu_inf + nu*delta^(p-2), DS(0)B = eta_D B); the right-hand side
 *     carries B_gamma(g_D, w) of eq. (disc-residual);
 *   - 3-point Gauss-Legendre per direction on cells and faces;
 *   - P1disc basis {1, (x_k - c_k)/h_k};
 *   - h_F = cell size normal to the face;
 *   - pressure sign of B^s: qsign=+1 reads the q-term so that the continuity
 *     block is the transpose of the momentum pressure block, qsign=-1 keeps the
 *     printed "+q Id";
 *   - the inflow factor (u.n)^- is lagged (Sec. 4.3), in the residual it is
 *     evaluated at a given field ulag (NULL = the state itself).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PICARD 0
#define ORC_EXACT_NEWTON 1
#define ORC_MODIFIED_NEWTON 2

typedef struct {
  int dim;            /* 2 or 3 */
  int n[3];           /* cells per direction */
  double lo[3], hi[3];
  int nt;             /* number of Gauss-Radau nodes = k+1 */
  double kt[16];      /* reference K_t, nt x nt row-major, row = test, col = trial */
  double wt[4];       /* reference Radau weights = diagonal of reference M_t */
  double mt[4];       /* reference m_t = xi_i(0) */
  double tau;         /* slab length */
  double p, delta, nu, nu_inf;
  double gamma1, gamma2;
  double sigma_max;
  int convection;     /* 1: p-Navier-Stokes, 0: p-Stokes */
  int qsign;          /* +1 or -1, see header */
  int lin;            /* ORC_PICARD / ORC_EXACT_NEWTON / ORC_MODIFIED_NEWTON */
  double gamma_cip;   /* CIP weight gamma_CIP of eq. (scip-def); 0 = off */
  const double* ghat; /* Dirichlet lifting, nt blocks of d*num_nodes; NULL = 0 */
  const double* gnode;/* the lifting of the one time node an element-level call
                         works on (d*num_nodes); NULL = 0 */
} orc_problem;

/* ---------------------------------------------------------------- sizes */

static int ipow3(int d) { int r = 1; for (int k = 0; k < d; ++k) r *= 3; return r; }

int orc_num_nodes(const orc_problem* P) {
  int r = 1;
  for (int k = 0; k < P->dim; ++k) r *= 2 * P->n[k] + 1;
  return r;
}
int orc_num_cells(const orc_problem* P) {
  int r = 1;
  for (int k = 0; k < P->dim; ++k) r *= P->n[k];
  return r;
}
/* spatial unknowns of one time node: d velocity components on the Q2 nodes,
 * then d+1 P1disc coefficients per cell */
int orc_spatial_size(const orc_problem* P) {
  return P->dim * orc_num_nodes(P) + (P->dim + 1) * orc_num_cells(P);
}
int orc_local_size(const orc_problem* P) {
  return P->dim * ipow3(P->dim) + P->dim + 1;
}

/* ------------------------------------------------------------ 1D Q2 basis */
/* Lagrange polynomials on the nodes {0, 1/2, 1} of the reference interval */
static double q2_val(int a, double s) {
  if (a == 0) return 2.0 * (s - 0.5) * (s - 1.0);
  if (a == 1) return -4.0 * s * (s - 1.0);
  return 2.0 * s * (s - 0.5);
}
static double q2_der(int a, double s) {
  if (a == 0) return 4.0 * s - 3.0;
  if (a == 1) return -8.0 * s + 4.0;
  return 4.0 * s - 1.0;
}

/* 3-point Gauss-Legendre rule on [0,1] */
static void gauss3(double* x, double* w) {
  double r = 0.5 * sqrt(0.6);
  x[0] = 0.5 - r; x[1] = 0.5; x[2] = 0.5 + r;
  w[0] = 5.0 / 18.0; w[1] = 8.0 / 18.0; w[2] = 5.0 / 18.0;
}

/* ------------------------------------------------- constitutive law (L0) */

static double ddot(int d, const double* A, const double* B) {
  double s = 0.0;
  for (int i = 0; i < d * d; ++i) s += A[i] * B[i];
  return s;
}

/* eta(A) = nu_inf + nu (delta^2 + |A|^2)^((p-2)/2), eq. (constitutive-law) */
static double eta_of(const orc_problem* P, double a2) {
  return P->nu_inf + P->nu * pow(P->delta * P->delta + a2, 0.5 * (P->p - 2.0));
}

/* S(A) = eta(A) A */
void orc_stress(const orc_problem* P, const double* A, double* S) {
  int d = P->dim;
  double e = eta_of(P, ddot(d, A, A));
  for (int i = 0; i < d * d; ++i) S[i] = e * A[i];
}

/* T(B) for the tangent selected by `kind`, at the linearisation point A.
 *   Picard:  eta B                                       eq. (local-tangent-picard)
 *   exact:   eta B + (p-2) mu/Delta^2 (A:B) A            eq. (local-tangent-exact)
 *   clipped: eta B + s (p-2) mu/Delta^2 (A:B) A,
 *            s = min(1, sigma_max/|mu A|), s = 0 if mu A = 0   eq. (local-tangent-clip) */
void orc_tangent(const orc_problem* P, int kind, const double* A, const double* B, double* T) {
  int d = P->dim;
  double a2 = ddot(d, A, A);
  double D2 = P->delta * P->delta + a2;
  double mu = P->nu * pow(D2, 0.5 * (P->p - 2.0));
  double eta = P->nu_inf + mu;
  double kappa = 0.0;
  if (kind == ORC_EXACT_NEWTON) {
    kappa = (P->p - 2.0) * mu / D2;
  } else if (kind == ORC_MODIFIED_NEWTON) {
    double sig = mu * sqrt(a2);
    double s = 0.0;
    if (sig > 0.0) s = (P->sigma_max / sig < 1.0) ? P->sigma_max / sig : 1.0;
    kappa = s * (P->p - 2.0) * mu / D2;
  }
  double ab = ddot(d, A, B);
  for (int i = 0; i < d * d; ++i) T[i] = eta * B[i] + kappa * ab * A[i];
}

/* ----------------------------------------------------- cell geometry */

typedef struct {
  int d, nb;               /* dimension, nodes per cell (3^d) */
  int cidx[3];             /* cell multi-index */
  double h[3];             /* cell sizes */
  double vol;              /* cell measure */
} cellgeo;

static void cell_setup(const orc_problem* P, int cell, cellgeo* g) {
  g->d = P->dim;
  g->nb = ipow3(P->dim);
  int r = cell;
  g->vol = 1.0;
  for (int k = 0; k < P->dim; ++k) {
    g->cidx[k] = r % P->n[k];
    r /= P->n[k];
    g->h[k] = (P->hi[k] - P->lo[k]) / P->n[k];
    g->vol *= g->h[k];
  }
}

/* global node number of local node a of the cell */
static int global_node(const orc_problem* P, const cellgeo* g, int a) {
  int idx = 0, stride = 1;
  for (int k = 0; k < P->dim; ++k) {
    int ak = (a / (k == 0 ? 1 : (k == 1 ? 3 : 9))) % 3;
    idx += (2 * g->cidx[k] + ak) * stride;
    stride *= 2 * P->n[k] + 1;
  }
  return idx;
}

/* global spatial index of every local unknown: velocity (comp c, node a) at
 * c*nb + a, pressure coefficient j at d*nb + j */
void orc_local_dofs(const orc_problem* P, int cell, int* dofs) {
  cellgeo g;
  cell_setup(P, cell, &g);
  int nn = orc_num_nodes(P);
  for (int c = 0; c < g.d; ++c)
    for (int a = 0; a < g.nb; ++a) dofs[c * g.nb + a] = c * nn + global_node(P, &g, a);
  for (int j = 0; j <= g.d; ++j) dofs[g.d * g.nb + j] = g.d * nn + cell * (g.d + 1) + j;
}

/* Every basis function of the cell evaluated at the reference point xi:
 * velocity scalar basis values/gradients (physical), pressure basis values. */
typedef struct {
  double phi[27];
  double dphi[27][3];
  double psi[4];
} basis_at;

static void eval_basis(const cellgeo* g, const double* xi, basis_at* B) {
  for (int a = 0; a < g->nb; ++a) {
    int ak[3] = {a % 3, (a / 3) % 3, (a / 9) % 3};
    double v = 1.0;
    for (int k = 0; k < g->d; ++k) v *= q2_val(ak[k], xi[k]);
    B->phi[a] = v;
    for (int k = 0; k < g->d; ++k) {
      double t = q2_der(ak[k], xi[k]) / g->h[k];
      for (int m = 0; m < g->d; ++m)
        if (m != k) t *= q2_val(ak[m], xi[m]);
      B->dphi[a][k] = t;
    }
  }
  B->psi[0] = 1.0;
  for (int k = 0; k < g->d; ++k) B->psi[1 + k] = xi[k] - 0.5;
}

/* A local unknown seen as a field: velocity value v[d], gradient G[i][j] =
 * d v_i / d x_j, pressure value q.  `j` is the local index. */
typedef struct {
  double v[3];
  double G[9];
  double q;
} field;

static void unit_field(const cellgeo* g, const basis_at* B, int j, field* f) {
  memset(f, 0, sizeof(*f));
  int d = g->d, nb = g->nb;
  if (j < d * nb) {
    int c = j / nb, a = j % nb;
    f->v[c] = B->phi[a];
    for (int k = 0; k < d; ++k) f->G[c * d + k] = B->dphi[a][k];
  } else {
    f->q = B->psi[j - d * nb];
  }
}

/* the state (velocity only, local values u[c*nb + a]) at the point */
static void state_field(const cellgeo* g, const basis_at* B, const double* u, field* f) {
  memset(f, 0, sizeof(*f));
  int d = g->d, nb = g->nb;
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < nb; ++a) {
      f->v[c] += u[c * nb + a] * B->phi[a];
      for (int k = 0; k < d; ++k) f->G[c * d + k] += u[c * nb + a] * B->dphi[a][k];
    }
}

static void symgrad(int d, const double* G, double* D) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) D[i * d + j] = 0.5 * (G[i * d + j] + G[j * d + i]);
}

static double div_of(int d, const double* G) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) s += G[i * d + i];
  return s;
}

static double vdot(int d, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) s += a[i] * b[i];
  return s;
}

/* -------------------------------------------- linearised spatial form J_mu */

/* Volume integrand of J_mu(trial x, test w) at one point with state u:
 *   (T(Dx), Dw)                                    viscous, with the tangent
 *   - (x (x) u + u (x) x, grad w)   [Newton]        convection, eq. (Defc)
 *   - (x (x) u, grad w)             [Picard]
 *   - (div w) x_pi                                  b(w, x_pi)
 *   - (div x) w_pi                                  b(x, w_pi)
 * with (a (x) b)_ij = a_i b_j and (grad w)_ij = d w_i / d x_j.               */
static double vol_J(const orc_problem* P, const field* u, const double* A, const field* x,
                    const field* w) {
  int d = P->dim;
  double Bx[9], T[9], Dw[9];
  symgrad(d, x->G, Bx);
  orc_tangent(P, P->lin, A, Bx, T);
  symgrad(d, w->G, Dw);
  double s = ddot(d, T, Dw);
  if (P->convection) {
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double m = x->v[i] * u->v[j];
        if (P->lin != ORC_PICARD) m += u->v[i] * x->v[j];
        s -= m * w->G[i * d + j];
      }
  }
  s -= div_of(d, w->G) * x->q;
  s -= div_of(d, x->G) * w->q;
  return s;
}

/* B^s and B^r of eq. (def-b-gam) for the field x (value xv) and the test w,
 * coefficients frozen at G = D ghat_D:
 *   - (DS(G)(Dw) n).x + qsign (x.n) w_pi + gamma1 eta(G)/hF (x.w) + gamma2/hF (x.n)(w.n) */
static double nitsche_sr(const orc_problem* P, const double* G, const double* n, double hF,
                         const double* xv, const field* w) {
  int d = P->dim;
  double Dw[9], DSw[9];
  symgrad(d, w->G, Dw);
  orc_tangent(P, ORC_EXACT_NEWTON, G, Dw, DSw);
  double xn = vdot(d, xv, n), wn = vdot(d, w->v, n), xw = vdot(d, xv, w->v);
  double s = 0.0;
  for (int i = 0; i < d; ++i) {
    double Dn = 0.0;
    for (int j = 0; j < d; ++j) Dn += DSw[i * d + j] * n[j];
    s -= Dn * xv[i];
  }
  s += (double)P->qsign * xn * w->q;
  s += P->gamma1 * eta_of(P, ddot(d, G, G)) / hF * xw + P->gamma2 / hF * xn * wn;
  return s;
}

/* Boundary integrand of J_mu on a Dirichlet face with outward normal n, face
 * size hF, frozen Nitsche coefficients at G = D ghat_D:
 *   (x.n)(u.w) + (u.n)(x.w)   [Newton] / (u.n)(x.w) [Picard]  convective flux, eq. (Defc)
 *   - (T(Dx) n).w + x_pi (n.w)                  -<(S(Du) - pi I) n, w>, eq. (def-a-gam)
 *   - (ulag.n)^- (x.w)                          B^c, factor lagged
 *   - (DS(G)(Dw) n).x + qsign (x.n) w_pi        B^s
 *   + gamma1 eta(G) / hF (x.w) + gamma2 / hF (x.n)(w.n)   B^r                   */
static double face_J(const orc_problem* P, const field* u, const double* A, const double* n,
                     double hF, const double* G, const field* x, const field* w) {
  int d = P->dim;
  double Bx[9], T[9];
  symgrad(d, x->G, Bx);
  orc_tangent(P, P->lin, A, Bx, T);
  double un = vdot(d, u->v, n), xn = vdot(d, x->v, n), wn = vdot(d, w->v, n);
  double xw = vdot(d, x->v, w->v);
  double s = 0.0;
  if (P->convection) {
    s += un * xw;
    if (P->lin != ORC_PICARD) s += xn * vdot(d, u->v, w->v);
    double neg = 0.5 * (fabs(un) - un);
    s -= neg * xw;
  }
  for (int i = 0; i < d; ++i) {
    double Tn = 0.0;
    for (int j = 0; j < d; ++j) Tn += T[i * d + j] * n[j];
    s -= Tn * w->v[i];
  }
  s += x->q * wn;
  s += nitsche_sr(P, G, n, hF, x->v, w);
  return s;
}

/* Quadrature points of the cell volume (reference coordinates, weights
 * including the cell measure). Returns the count. */
static int volume_rule(const cellgeo* g, double (*xi)[3], double* w) {
  double gx[3], gw[3];
  gauss3(gx, gw);
  int nq = ipow3(g->d);
  for (int q = 0; q < nq; ++q) {
    int qk[3] = {q % 3, (q / 3) % 3, (q / 9) % 3};
    w[q] = g->vol;
    for (int k = 0; k < 3; ++k) xi[q][k] = 0.0;
    for (int k = 0; k < g->d; ++k) {
      xi[q][k] = gx[qk[k]];
      w[q] *= gw[qk[k]];
    }
  }
  return nq;
}

/* Quadrature points on face (direction k, side s) of the cell, if that face
 * lies on the domain boundary.  Returns the count (0 for an interior face). */
static int face_rule(const orc_problem* P, const cellgeo* g, int k, int s, double (*xi)[3],
                     double* w, double* n, double* hF) {
  if (s == 0 && g->cidx[k] != 0) return 0;
  if (s == 1 && g->cidx[k] != P->n[k] - 1) return 0;
  double gx[3], gw[3];
  gauss3(gx, gw);
  int nq = ipow3(g->d - 1);
  double area = g->vol / g->h[k];
  for (int q = 0; q < nq; ++q) {
    int qt[2] = {q % 3, (q / 3) % 3};
    int t = 0;
    w[q] = area;
    for (int m = 0; m < g->d; ++m) {
      if (m == k) {
        xi[q][m] = (double)s;
      } else {
        xi[q][m] = gx[qt[t]];
        w[q] *= gw[qt[t]];
        ++t;
      }
    }
    for (int m = g->d; m < 3; ++m) xi[q][m] = 0.0;
  }
  for (int m = 0; m < 3; ++m) n[m] = 0.0;
  n[k] = s ? 1.0 : -1.0;
  *hF = g->h[k];
  return nq;
}

/* local values of the lifting P->gnode on the cell (0 without one) */
static void lift_local(const orc_problem* P, int cell, double* gloc) {
  int nb = ipow3(P->dim);
  if (!P->gnode) {
    memset(gloc, 0, sizeof(double) * P->dim * nb);
    return;
  }
  int dofs[85];
  orc_local_dofs(P, cell, dofs);
  for (int i = 0; i < P->dim * nb; ++i) gloc[i] = P->gnode[dofs[i]];
}

/* Element matrix of J_mu on one cell: E[i*nloc + j] = J_mu(trial j, test i),
 * state given by the local velocity values u[c*nb + a]; Nitsche coefficients
 * frozen at the lifting P->gnode. */
void orc_element_matrix(const orc_problem* P, int cell, const double* u, double* E) {
  cellgeo g;
  cell_setup(P, cell, &g);
  int d = g.d, nloc = orc_local_size(P);
  memset(E, 0, sizeof(double) * nloc * nloc);
  double gloc[81];
  lift_local(P, cell, gloc);
  double xi[27][3], w[27];
  field* fx = (field*)malloc(sizeof(field) * nloc);
  /* volume */
  int nq = volume_rule(&g, xi, w);
  for (int q = 0; q < nq; ++q) {
    basis_at B;
    eval_basis(&g, xi[q], &B);
    field us;
    state_field(&g, &B, u, &us);
    double A[9];
    symgrad(d, us.G, A);
    for (int j = 0; j < nloc; ++j) unit_field(&g, &B, j, &fx[j]);
    for (int i = 0; i < nloc; ++i)
      for (int j = 0; j < nloc; ++j) E[i * nloc + j] += w[q] * vol_J(P, &us, A, &fx[j], &fx[i]);
  }
  /* Dirichlet faces (the whole boundary) */
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      double n[3], hF;
      int nf = face_rule(P, &g, k, s, xi, w, n, &hF);
      for (int q = 0; q < nf; ++q) {
        basis_at B;
        eval_basis(&g, xi[q], &B);
        field us, gs;
        state_field(&g, &B, u, &us);
        state_field(&g, &B, gloc, &gs);
        double A[9], G[9];
        symgrad(d, us.G, A);
        symgrad(d, gs.G, G);
        for (int j = 0; j < nloc; ++j) unit_field(&g, &B, j, &fx[j]);
        for (int i = 0; i < nloc; ++i)
          for (int j = 0; j < nloc; ++j)
            E[i * nloc + j] += w[q] * face_J(P, &us, A, n, hF, G, &fx[j], &fx[i]);
      }
    }
  free(fx);
}

/* Scalar Q2 mass matrix of the cell: M[a*nb + b] = (phi_b, phi_a). */
void orc_element_mass(const orc_problem* P, int cell, double* M) {
  cellgeo g;
  cell_setup(P, cell, &g);
  memset(M, 0, sizeof(double) * g.nb * g.nb);
  double xi[27][3], w[27];
  int nq = volume_rule(&g, xi, w);
  for (int q = 0; q < nq; ++q) {
    basis_at B;
    eval_basis(&g, xi[q], &B);
    for (int a = 0; a < g.nb; ++a)
      for (int b = 0; b < g.nb; ++b) M[a * g.nb + b] += w[q] * B.phi[a] * B.phi[b];
  }
}

/* gather the local velocity values of one time node from a spatial vector */
static void gather_velocity(const orc_problem* P, const int* dofs, const double* vec, double* loc) {
  int nb = ipow3(P->dim);
  for (int i = 0; i < P->dim * nb; ++i) loc[i] = vec[dofs[i]];
}

/* All element matrices of J_mu at the spatial velocity state u (d*num_nodes
 * values), E[cell][nloc][nloc]. */
void orc_all_element_matrices(const orc_problem* P, const double* u, double* E) {
  int nc = orc_num_cells(P), nloc = orc_local_size(P);
  int dofs[85];
  double uloc[81];
  for (int c = 0; c < nc; ++c) {
    orc_local_dofs(P, c, dofs);
    gather_velocity(P, dofs, u, uloc);
    orc_element_matrix(P, c, uloc, E + (size_t)c * nloc * nloc);
  }
}

/* ------------------------------------------------------ CIP stabilisation */

/* Interior faces: direction k (normal e_k), between cell L = c - e_k and cell
 * R = c (c_k >= 1).  Faces are numbered direction by direction, within a
 * direction by the index of cell R in the mesh with n_k - 1 cells along k. */
int orc_cip_count(const orc_problem* P) {
  int total = 0;
  for (int k = 0; k < P->dim; ++k) {
    int m = 1;
    for (int j = 0; j < P->dim; ++j) m *= (j == k ? P->n[j] - 1 : P->n[j]);
    total += m;
  }
  return total;
}

/* Local matrix of the CIP form of eq. (scip-def) on interior face f,
 *   s_F(uw; x, v) = gamma_CIP h_F^2 int_F |uw . n_F| [grad x n_F] . [grad v n_F] ds,
 * [g] = g|_L - g|_R, the weight field uw (d*num_nodes velocity values of one
 * time node) evaluated on the face, h_F the cell size normal to the face,
 * 3^(d-1) Gauss points.  Local unknowns: velocity (component c, node a) of L
 * at c*nb + a, of R at d*nb + c*nb + a; dofs[] receives their global spatial
 * indices, M the (2 d nb)^2 matrix, row = test. */
void orc_cip_face(const orc_problem* P, const double* uw, int f, int* dofs, double* M) {
  int d = P->dim, nb = ipow3(d), nl = 2 * d * nb;
  int k = 0;
  for (; k < d; ++k) {
    int m = 1;
    for (int j = 0; j < d; ++j) m *= (j == k ? P->n[j] - 1 : P->n[j]);
    if (f < m) break;
    f -= m;
  }
  /* cell R from f over the mesh with n_k - 1 cells along k, shifted by one */
  int idx[3] = {0, 0, 0}, r = f;
  for (int j = 0; j < d; ++j) {
    int nj = (j == k ? P->n[j] - 1 : P->n[j]);
    idx[j] = r % nj + (j == k ? 1 : 0);
    r /= nj;
  }
  int cR = 0, cL = 0, stride = 1;
  for (int j = 0; j < d; ++j) {
    cR += idx[j] * stride;
    cL += (idx[j] - (j == k ? 1 : 0)) * stride;
    stride *= P->n[j];
  }
  int dl[85], dr[85];
  orc_local_dofs(P, cL, dl);
  orc_local_dofs(P, cR, dr);
  for (int i = 0; i < d * nb; ++i) {
    dofs[i] = dl[i];
    dofs[d * nb + i] = dr[i];
  }
  memset(M, 0, sizeof(double) * nl * nl);
  cellgeo gL, gR;
  cell_setup(P, cL, &gL);
  cell_setup(P, cR, &gR);
  double gx[3], gw[3];
  gauss3(gx, gw);
  double hF = gL.h[k];
  double area = gL.vol / gL.h[k];
  int nq = ipow3(d - 1);
  double uwl[81];
  for (int i = 0; i < d * nb; ++i) uwl[i] = uw[dl[i]];
  double* jn = (double*)malloc(sizeof(double) * nl);
  for (int q = 0; q < nq; ++q) {
    int qt[2] = {q % 3, (q / 3) % 3};
    double xiL[3] = {0, 0, 0}, xiR[3] = {0, 0, 0}, w = area;
    int t = 0;
    for (int m = 0; m < d; ++m) {
      if (m == k) {
        xiL[m] = 1.0;
        xiR[m] = 0.0;
      } else {
        xiL[m] = xiR[m] = gx[qt[t]];
        w *= gw[qt[t]];
        ++t;
      }
    }
    basis_at BL, BR;
    eval_basis(&gL, xiL, &BL);
    eval_basis(&gR, xiR, &BR);
    field uf;
    state_field(&gL, &BL, uwl, &uf);
    double un = fabs(uf.v[k]);   /* n_F = e_k */
    double wq = P->gamma_cip * hF * hF * un * w;
    /* normal derivative of each local unknown, with the sign of the jump */
    for (int c = 0; c < d; ++c)
      for (int a = 0; a < nb; ++a) {
        jn[c * nb + a] = BL.dphi[a][k];
        jn[d * nb + c * nb + a] = -BR.dphi[a][k];
      }
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        int ci = (i % (d * nb)) / nb, cj = (j % (d * nb)) / nb;
        if (ci == cj) M[i * nl + j] += wq * jn[i] * jn[j];
      }
  }
  free(jn);
}

/* y_mu += tau wt[mu] s_CIP(uw_mu; x_mu, .) over every interior face, the
 * weight fields uw given per time node (nt blocks of d*num_nodes). */
static void cip_add(const orc_problem* P, const double* uw, const double* x, double* y,
                    double sign) {
  int d = P->dim, nb = ipow3(d), nl = 2 * d * nb, nn = orc_num_nodes(P);
  int ns = orc_spatial_size(P), nf = orc_cip_count(P);
  int dofs[162];
  double* M = (double*)malloc(sizeof(double) * nl * nl);
  for (int mu = 0; mu < P->nt; ++mu)
    for (int f = 0; f < nf; ++f) {
      orc_cip_face(P, uw + (size_t)mu * d * nn, f, dofs, M);
      const double* xm = x + (size_t)mu * ns;
      double* ym = y + (size_t)mu * ns;
      double scale = sign * P->tau * P->wt[mu];
      for (int i = 0; i < nl; ++i) {
        double s = 0.0;
        for (int j = 0; j < nl; ++j) s += M[i * nl + j] * xm[dofs[j]];
        ym[dofs[i]] += scale * s;
      }
    }
  free(M);
}

/* ---------------------------------------------------------- slab apply */

/* Contributions of cell c to y = J_n x, eq. (slab-underint-jac):
 *   y_v,mu += sum_nu Kt[mu][nu] (M_x x_v,nu) + tau wt[mu] (J_mu x_mu)_v
 *   y_p,mu += tau wt[mu] (J_mu x_mu)_p
 * restricted to the cell (its element matrices times its local values).
 * E: scratch of nloc^2 doubles. */
static void apply_cell(const orc_problem* P, int c, const double* uk, const double* x,
                       double* y, double* E) {
  int d = P->dim, nb = ipow3(d), nloc = orc_local_size(P);
  int nn = orc_num_nodes(P), ns = orc_spatial_size(P);
  double M[729];
  int dofs[85];
  double uloc[81];
  orc_local_dofs(P, c, dofs);
  orc_element_mass(P, c, M);
  for (int mu = 0; mu < P->nt; ++mu) {
    orc_problem Pm = *P;
    Pm.gnode = P->ghat ? P->ghat + (size_t)mu * d * nn : NULL;
    gather_velocity(P, dofs, uk + (size_t)mu * d * nn, uloc);
    orc_element_matrix(&Pm, c, uloc, E);
    const double* xm = x + (size_t)mu * ns;
    double* ym = y + (size_t)mu * ns;
    double scale = P->tau * P->wt[mu];
    for (int i = 0; i < nloc; ++i) {
      double s = 0.0;
      for (int j = 0; j < nloc; ++j) s += E[i * nloc + j] * xm[dofs[j]];
      ym[dofs[i]] += scale * s;
    }
    /* temporal mass coupling, velocity only */
    for (int nu = 0; nu < P->nt; ++nu) {
      double kmn = P->kt[mu * P->nt + nu];
      const double* xn = x + (size_t)nu * ns;
      for (int cc = 0; cc < d; ++cc)
        for (int a = 0; a < nb; ++a) {
          double s = 0.0;
          for (int b = 0; b < nb; ++b) s += M[a * nb + b] * xn[dofs[cc * nb + b]];
          ym[dofs[cc * nb + a]] += kmn * s;
        }
    }
  }
}

/* y = J_n x, eq. (slab-underint-jac), element by element.
 * uk holds the velocity state at every Radau node (nt blocks of d*num_nodes),
 * x and y hold nt blocks of spatial_size. */
void orc_apply(const orc_problem* P, const double* uk, const double* x, double* y) {
  int nloc = orc_local_size(P), nc = orc_num_cells(P), ns = orc_spatial_size(P);
  memset(y, 0, sizeof(double) * (size_t)ns * P->nt);
  double* E = (double*)malloc(sizeof(double) * nloc * nloc);
  for (int c = 0; c < nc; ++c) apply_cell(P, c, uk, x, y, E);
  free(E);
  /* CIP with the weight lagged at u_k (every linearisation) */
  if (P->gamma_cip > 0.0) cip_add(P, uk, x, y, 1.0);
}

/* The same action on `nthreads` host threads (CPU timing only): the cells are
 * visited in 2^d parity classes (cells of one class share no node and no
 * pressure coefficient), each class split over the threads.  Per cell the
 * arithmetic is that of orc_apply; only the order in which the cells add to a
 * shared node differs. */
void orc_apply_threads(const orc_problem* P, const double* uk, const double* x, double* y,
                       int nthreads) {
  int d = P->dim, nloc = orc_local_size(P), nc = orc_num_cells(P), ns = orc_spatial_size(P);
  memset(y, 0, sizeof(double) * (size_t)ns * P->nt);
  for (int color = 0; color < (1 << d); ++color) {
#pragma omp parallel num_threads(nthreads)
    {
      double* E = (double*)malloc(sizeof(double) * nloc * nloc);
#pragma omp for schedule(static)
      for (int c = 0; c < nc; ++c) {
        int cx = c % P->n[0], cy = (c / P->n[0]) % P->n[1];
        int cz = d == 3 ? c / (P->n[0] * P->n[1]) : 0;
        int cl = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
        if (cl == color) apply_cell(P, c, uk, x, y, E);
      }
      free(E);
    }
  }
  if (P->gamma_cip > 0.0) cip_add(P, uk, x, y, 1.0);
}

/* ------------------------------------------------------------ load vector */

/* Right-hand side of the volume force on the slab, the f-term of eq.
 * (disc-residual) under the Radau rule of eq. (slab-underint):
 *   F_v,mu[i] = tau wt[mu] (f(t_mu), phi_i)_Omega,   F_p = 0,
 * each cell integrated with its 3^d-point Gauss rule.  f_qp holds f at those
 * points: f_qp[((mu * cells + cell) * 3^d + q) * d + comp], q = qx + 3 qy
 * (+ 9 qz), the points ordered as in volume_rule. */
void orc_load(const orc_problem* P, const double* f_qp, double* F) {
  int d = P->dim, nb = ipow3(d), nc = orc_num_cells(P), ns = orc_spatial_size(P);
  memset(F, 0, sizeof(double) * (size_t)ns * P->nt);
  int dofs[85];
  double xi[27][3], w[27];
  for (int c = 0; c < nc; ++c) {
    cellgeo g;
    cell_setup(P, c, &g);
    orc_local_dofs(P, c, dofs);
    int nq = volume_rule(&g, xi, w);
    for (int mu = 0; mu < P->nt; ++mu) {
      double* Fm = F + (size_t)mu * ns;
      double scale = P->tau * P->wt[mu];
      for (int q = 0; q < nq; ++q) {
        basis_at B;
        eval_basis(&g, xi[q], &B);
        const double* f = f_qp + (((size_t)mu * nc + c) * nq + q) * d;
        for (int cc = 0; cc < d; ++cc)
          for (int a = 0; a < nb; ++a) Fm[dofs[cc * nb + a]] += scale * w[q] * f[cc] * B.phi[a];
      }
    }
  }
}

/* --------------------------------------------------------- slab residual */

/* Nonlinear left-hand-side form A_gamma(u,pi)(w) at one point (volume part):
 *   S(Du):Dw - (u (x) u):grad w - (div w) pi - (div u) w_pi                   */
static double vol_A(const orc_problem* P, const field* u, const field* w) {
  int d = P->dim;
  double A[9], S[9], Dw[9];
  symgrad(d, u->G, A);
  orc_stress(P, A, S);
  symgrad(d, w->G, Dw);
  double s = ddot(d, S, Dw);
  if (P->convection)
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) s -= u->v[i] * u->v[j] * w->G[i * d + j];
  s -= div_of(d, w->G) * u->q;
  s -= div_of(d, u->G) * w->q;
  return s;
}

/* boundary part of A_gamma on a Dirichlet face, Nitsche coefficients frozen
 * at G = D ghat_D:
 *   (u.n)(u.w) - (S(Du) n).w + pi (n.w) - (ulag.n)^- (u.w)
 *   - (DS(G)(Dw) n).u + qsign (u.n) w_pi + gamma1 eta(G)/hF (u.w) + gamma2/hF (u.n)(w.n) */
static double face_A(const orc_problem* P, const field* u, const field* ulag, const double* n,
                     double hF, const double* G, const field* w) {
  int d = P->dim;
  double A[9], S[9];
  symgrad(d, u->G, A);
  orc_stress(P, A, S);
  double un = vdot(d, u->v, n), wn = vdot(d, w->v, n), uw = vdot(d, u->v, w->v);
  double s = 0.0;
  if (P->convection) {
    double ln = vdot(d, ulag->v, n);
    s += un * uw;
    s -= 0.5 * (fabs(ln) - ln) * uw;
  }
  for (int i = 0; i < d; ++i) {
    double Sn = 0.0;
    for (int j = 0; j < d; ++j) Sn += S[i * d + j] * n[j];
    s -= Sn * w->v[i];
  }
  s += u->q * wn;
  s += nitsche_sr(P, G, n, hF, u->v, w);
  return s;
}

/* B_gamma(g_D, w) of eq. (def-b-gam) at a face point, g the lifting's value
 * there (its trace), G = D ghat_D:
 *   - (g.n)^- (g.w) [with convection] + B^s(g, w) + B^r(g, w)              */
static double face_B(const orc_problem* P, const double* g, const double* n, double hF,
                     const double* G, const field* w) {
  int d = P->dim;
  double s = 0.0;
  if (P->convection) {
    double gn = vdot(d, g, n);
    s -= 0.5 * (fabs(gn) - gn) * vdot(d, g, w->v);
  }
  return s + nitsche_sr(P, G, n, hF, g, w);
}

/* Local vector of A_gamma at state (u, pi) on one cell: F[i] = A_gamma(u,pi)(test i).
 * uloc: velocity local values, ploc: d+1 pressure coefficients, lagloc: local
 * velocity values of the field in the lagged inflow factor. */
void orc_element_form(const orc_problem* P, int cell, const double* uloc, const double* ploc,
                      const double* lagloc, double* F) {
  cellgeo g;
  cell_setup(P, cell, &g);
  int d = g.d, nloc = orc_local_size(P);
  memset(F, 0, sizeof(double) * nloc);
  double gloc[81];
  lift_local(P, cell, gloc);
  double xi[27][3], w[27];
  int nq = volume_rule(&g, xi, w);
  for (int q = 0; q < nq; ++q) {
    basis_at B;
    eval_basis(&g, xi[q], &B);
    field us;
    state_field(&g, &B, uloc, &us);
    for (int j = 0; j <= d; ++j) us.q += ploc[j] * B.psi[j];
    for (int i = 0; i < nloc; ++i) {
      field fw;
      unit_field(&g, &B, i, &fw);
      F[i] += w[q] * vol_A(P, &us, &fw);
    }
  }
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      double n[3], hF;
      int nf = face_rule(P, &g, k, s, xi, w, n, &hF);
      for (int q = 0; q < nf; ++q) {
        basis_at B;
        eval_basis(&g, xi[q], &B);
        field us, ul, gs;
        state_field(&g, &B, uloc, &us);
        state_field(&g, &B, lagloc, &ul);
        state_field(&g, &B, gloc, &gs);
        for (int j = 0; j <= d; ++j) us.q += ploc[j] * B.psi[j];
        double G[9];
        symgrad(d, gs.G, G);
        for (int i = 0; i < nloc; ++i) {
          field fw;
          unit_field(&g, &B, i, &fw);
          F[i] += w[q] * face_A(P, &us, &ul, n, hF, G, &fw);
        }
      }
    }
}

/* Local vector of B_gamma(g_D, .) on one cell (zero unless the cell has a
 * boundary face and P->gnode is set): F[i] = B_gamma(g_D, test i). */
void orc_element_lift(const orc_problem* P, int cell, double* F) {
  cellgeo g;
  cell_setup(P, cell, &g);
  int d = g.d, nloc = orc_local_size(P);
  memset(F, 0, sizeof(double) * nloc);
  if (!P->gnode) return;
  double gloc[81];
  lift_local(P, cell, gloc);
  double xi[27][3], w[27];
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      double n[3], hF;
      int nf = face_rule(P, &g, k, s, xi, w, n, &hF);
      for (int q = 0; q < nf; ++q) {
        basis_at B;
        eval_basis(&g, xi[q], &B);
        field gs;
        state_field(&g, &B, gloc, &gs);
        double G[9];
        symgrad(d, gs.G, G);
        for (int i = 0; i < nloc; ++i) {
          field fw;
          unit_field(&g, &B, i, &fw);
          F[i] += w[q] * face_B(P, gs.v, n, hF, G, &fw);
        }
      }
    }
}

/* Slab residual, eq. (slab-underint), right-hand side minus left-hand side with
 * f = 0 and the Dirichlet data of the lifting P->ghat (NULL: g_D = 0):
 *   R_v,mu = -( sum_nu Kt[mu][nu] M_x V_nu - mt[mu] M_x vprev )
 *            + tau wt[mu] (B_gamma(g_D(t_mu)) - A_gamma(U_mu))_v
 *   R_p,mu = tau wt[mu] (B_gamma(g_D(t_mu)) - A_gamma(U_mu))_p
 * U: nt spatial blocks; vprev: left trace (velocity, d*num_nodes), may be NULL
 * (zero); ulag: nt velocity blocks for the inflow factor, NULL = U itself. */
void orc_residual(const orc_problem* P, const double* U, const double* vprev, const double* ulag,
                  double* R) {
  int d = P->dim, nb = ipow3(d), nloc = orc_local_size(P);
  int nc = orc_num_cells(P), nn = orc_num_nodes(P), ns = orc_spatial_size(P);
  memset(R, 0, sizeof(double) * (size_t)ns * P->nt);
  double M[729], F[85];
  int dofs[85];
  double uloc[81], lloc[81], ploc[4];
  for (int c = 0; c < nc; ++c) {
    orc_local_dofs(P, c, dofs);
    orc_element_mass(P, c, M);
    for (int mu = 0; mu < P->nt; ++mu) {
      const double* Um = U + (size_t)mu * ns;
      double* Rm = R + (size_t)mu * ns;
      for (int i = 0; i < d * nb; ++i) uloc[i] = Um[dofs[i]];
      for (int j = 0; j <= d; ++j) ploc[j] = Um[dofs[d * nb + j]];
      if (ulag) {
        for (int i = 0; i < d * nb; ++i) lloc[i] = ulag[(size_t)mu * d * nn + dofs[i]];
      } else {
        memcpy(lloc, uloc, sizeof(double) * d * nb);
      }
      orc_problem Pm = *P;
      Pm.gnode = P->ghat ? P->ghat + (size_t)mu * d * nn : NULL;
      orc_element_form(&Pm, c, uloc, ploc, lloc, F);
      double scale = P->tau * P->wt[mu];
      for (int i = 0; i < nloc; ++i) Rm[dofs[i]] -= scale * F[i];
      if (Pm.gnode) {
        orc_element_lift(&Pm, c, F);
        for (int i = 0; i < nloc; ++i) Rm[dofs[i]] += scale * F[i];
      }
      for (int cc = 0; cc < d; ++cc)
        for (int a = 0; a < nb; ++a) {
          double s = 0.0;
          for (int b = 0; b < nb; ++b) {
            double tb = 0.0;
            for (int nu = 0; nu < P->nt; ++nu)
              tb += P->kt[mu * P->nt + nu] * U[(size_t)nu * ns + dofs[cc * nb + b]];
            if (vprev) tb -= P->mt[mu] * vprev[dofs[cc * nb + b]];
            s += M[a * nb + b] * tb;
          }
          Rm[dofs[cc * nb + a]] -= s;
        }
    }
  }
  /* CIP, eq. (scip-def): s_CIP(u; u, v) with the weight at the state itself,
   * or at ulag (the lagged weight of the linearisations) when given */
  if (P->gamma_cip > 0.0) {
    double* uw = (double*)malloc(sizeof(double) * (size_t)P->nt * d * nn);
    for (int mu = 0; mu < P->nt; ++mu)
      for (int i = 0; i < d * nn; ++i)
        uw[(size_t)mu * d * nn + i] = ulag ? ulag[(size_t)mu * d * nn + i] : U[(size_t)mu * ns + i];
    cip_add(P, uw, U, R, -1.0);
    free(uw);
  }
}
