/*
 * pnsmg.h -- C-ABI of the MI355X space-time multigrid smoothing step for the
 * time-dependent (p,delta)-Navier-Stokes equations
 * (Margenberg & Mehlmann, arXiv 2603.28706).
 *
 * Discretisation (Sec. 3): uniform quadrilateral mesh of a box, Q2 velocity /
 * P1disc pressure in space, dG(1) in time with the two right Gauss-Radau nodes
 * t = 1/3, 1 of the reference slab (Sec. 3.1, Sec. 5.2).  Dirichlet data are
 * imposed weakly by Nitsche terms on the whole boundary (Sec. 3.2,
 * eq. def-b-gam) with homogeneous data.
 *
 * Vector layout ("canonical"), identical for every vector argument:
 *   one block per Radau node mu = 0, 1; inside a block the d velocity
 *   components, each over the (2 n_x + 1)(2 n_y + 1) Q2 nodes in lexicographic
 *   order (x fastest), then 3 P1disc coefficients per cell (cells
 *   lexicographic, coefficients of 1, (x - x_c)/h_x, (y - y_c)/h_y).
 *   A level-l vector has the same layout on the level-l mesh.
 *
 * Precision: the context precision (PNS_FP64 or PNS_FP32) is the element type
 * of every x, y, r, d argument.  The linearisation state u_k is always given
 * in FP64.  The constitutive power law is evaluated in FP64 in both modes.
 * PNS_BF16 (hexahedral meshes, one level, the action only): the state is
 * stored in BF16 (rounded to nearest even from the FP64 u_k), x of
 * pns_cell_apply / pns_cell_defect is BF16 (uint16 bit patterns of bfloat16),
 * y and b are FP32, the arithmetic is FP32 with the power law in FP64; every
 * smoother, V-cycle, residual and solve entry point returns PNS_EUNSUPPORTED.
 *
 * Memory: every pointer named *_dev is a device pointer owned by the caller.
 * The library allocates no device memory; it works in one caller-provided
 * workspace (query its size, bind it once).  All calls are asynchronous on the
 * stream given at creation; they return after enqueueing.  Calls on one
 * context must not overlap (one stream, one caller at a time).
 *
 * Errors: every int-returning call returns PNS_OK (0) or a negative code; the
 * message of the last error of a context is returned by pns_last_error.  On
 * error nothing is enqueued and the outputs are unchanged.
 */
#ifndef PNSMG_H
#define PNSMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PNS_OK = 0,
  PNS_EINVAL = -1,      /* invalid argument (sizes, model parameters, NULL) */
  PNS_EWORKSPACE = -2,  /* no workspace bound, or too small / misaligned */
  PNS_EHIP = -3,        /* a HIP runtime call failed */
  PNS_ESTATE = -4,      /* call order: no state set / smoother not set up */
  PNS_ESINGULAR = -5,   /* a patch or the coarse matrix had a zero pivot */
  PNS_EUNSUPPORTED = -6, /* configuration outside what this build implements */
  PNS_ENOTCONV = -7,    /* a slab solve stopped without reaching its tolerance */
  PNS_ENONFINITE = -8   /* a slab solve met a NaN or infinite residual or Krylov value */
};

/* Constitutive tangent of the linearisation (Sec. 4.2-4.4). */
typedef enum {
  PNS_PICARD = 0,          /* eta B, eq. (local-tangent-picard) */
  PNS_EXACT_NEWTON = 1,    /* D S(A) B, eq. (local-tangent-exact) */
  PNS_MODIFIED_NEWTON = 2  /* stress-clipped rank one, eq. (local-tangent-clip) */
} pns_lin_kind;

typedef enum { PNS_FP64 = 0, PNS_FP32 = 1, PNS_BF16 = 2 } pns_precision;

/* How the level-0 action obtains the constitutive tangent at each quadrature
 * point (same operator, same FP64 tangent arithmetic; only where it happens):
 *   RECOMPUTE: from u_k inside every action (nothing stored);
 *   CACHED: once per pns_set_state, six coefficients per point and Radau node
 *   (eta, the rank-one direction scaled by sqrt(-kappa), the advecting
 *   velocity, all times the quadrature weight) stored in the workspace in the
 *   context precision and read by every action. */
typedef enum { PNS_APPLY_RECOMPUTE = 0, PNS_APPLY_CACHED = 1 } pns_apply_mode;

/* Patch matrices of the finest-level Vanka smoother (Sec. 6.3):
 *   SURROGATE: every state-dependent coefficient frozen at the slab midpoint,
 *   eq. (surrogate-diag), solved in time-diagonal form (one complex 21x21
 *   inverse per cell);
 *   EXACT: the exact patch matrices R_K A R_K^T of the slab operator with the
 *   coefficients of each Radau node (real 42x42 inverse per cell), as on the
 *   coarse levels. */
typedef enum { PNS_PATCH_SURROGATE = 0, PNS_PATCH_EXACT = 1 } pns_patch_kind;

/* Box [lo, hi] with n_cells[k] uniform cells per direction.  dim = 2
 * (quadrilaterals; n_cells[2], lo[2], hi[2] unused) or dim = 3 (hexahedra).
 * Canonical layout of one Radau node's spatial block: velocity component c
 * at c*nn + node, nodes lexicographic with x fastest over the (2n_k+1) Q2
 * nodes per direction (nn nodes); then the d+1 P1disc coefficients of each
 * cell (cells lexicographic, x fastest) in the basis 1, (x_k - xc_k)/h_k. */
typedef struct {
  int dim;
  int n_cells[3];
  double lo[3], hi[3];
} pns_mesh;

/* Q_{k_space} / P_{k_space-1}^disc x dG(k_time) on the slab (t0, t0 + tau].
 * This build implements k_space = 2, k_time = 1. */
typedef struct {
  int k_space;
  int k_time;
  double t0, tau;
} pns_discretization;

/* Model of Sec. 2 / Sec. 3.2:
 *   S(D) = eta(D) D, eta(D) = nu_inf + nu (delta^2 + |D|^2)^((p-2)/2),
 *   1 < p <= 2, delta > 0, nu > 0, nu_inf >= 0  (eq. constitutive-law);
 *   Nitsche penalties gamma1, gamma2 > 0 with h_F = cell size normal to the
 *   face (eq. def-b-gam); sigma_max >= 0 the stress clip of modified Newton
 *   (Sec. 4.4); convection = 1 for p-Navier-Stokes, 0 for p-Stokes;
 *   nitsche_q_sign = +1 makes the Nitsche pressure coupling the transpose of
 *   the momentum one (-q I in B^s), -1 keeps the printed +q I;
 *   lin = pns_lin_kind of the Jacobian action;
 *   gamma_cip > 0 adds the convection-aligned CIP stabilisation of Sec. 3.2,
 *   eq. (scip-def): on every interior face F, gamma_cip h_F^2 int_F
 *   |u^ . n_F| [grad u n_F] . [grad v n_F], h_F the cell size normal to F; in
 *   the residual the weight u^ is the state itself, in the Jacobian action of
 *   every linearisation it is lagged at u_k (eq. Amu-decomp), which keeps the
 *   term symmetric positive semidefinite.  The Vanka patches and the coarse
 *   Galerkin operators are formed from the cell terms only (the CIP face
 *   coupling enters the action and the residual, so the solve converges to
 *   the stabilised solution; the V-cycle preconditions it without the face
 *   term).  Hexahedral contexts return PNS_EUNSUPPORTED for gamma_cip > 0. */
typedef struct {
  double p, delta, nu, nu_inf;
  double gamma1, gamma2;
  double sigma_max;
  int convection;
  int nitsche_q_sign;
  int lin;
  double gamma_cip;  /* CIP weight of eq. (scip-def), >= 0; 0 = off (quadrilaterals only) */
} pns_model;

typedef struct pns_ctx pns_ctx;

/* Create a context for `n_levels` nested meshes (level 0 = the given mesh,
 * level l has n_cells / 2^l cells per direction, every level keeps dG(1)).
 * n_cells must be divisible by 2^(n_levels-1).  The dense coarsest solve
 * (and so pns_vcycle) is available when the coarsest level has at most 40000
 * space-time unknowns; larger coarsest levels still allow the apply and the
 * smoother.  `stream` is a hipStream_t (NULL =
 * default stream).  A dim = 3 mesh (hexahedra, n_cells divisible by
 * 2^(n_levels-1) in every direction) supports every entry point below except
 * node masks in pns_vanka_setup; pns_vcycle and pns_solve need at least two
 * levels (the dense coarsest inverse is formed only then).
 * Returns PNS_EINVAL / PNS_EUNSUPPORTED on bad input. */
int pns_ctx_create(const pns_mesh* mesh, const pns_discretization* disc, int n_levels,
                   int precision, void* stream, pns_ctx** out);

void pns_ctx_destroy(pns_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* pns_last_error(const pns_ctx* ctx);

/* Sizes of level `level`: out[0] = space-time unknowns, out[1] = cells,
 * out[2] = velocity unknowns per Radau node, out[3] = spatial unknowns per
 * Radau node. */
int pns_level_sizes(const pns_ctx* ctx, int level, int64_t out[4]);

/* Bytes of device workspace the context needs (all levels, smoother data,
 * coarse inverse) and its required alignment (256).  On hexahedra the
 * level-0 smoother storage follows the patch kind selected at the time of
 * the query (FP64 per cell: ~173 KB surrogate, ~347 KB exact, plus 58 KB of
 * second-node cell matrices with two or more levels), so select the kind
 * first. */
size_t pns_workspace_bytes(const pns_ctx* ctx);

/* Bind a caller-owned device buffer of at least pns_workspace_bytes bytes,
 * 256-byte aligned; it must stay valid until the context is destroyed or
 * another buffer is bound.  Binding invalidates state and smoother data. */
int pns_bind_workspace(pns_ctx* ctx, void* ws_dev, size_t bytes);

/* Set the linearisation point: u_k_dev holds the velocity (FP64) at both
 * Radau nodes, 2 blocks of d*nn values in the canonical velocity layout.  Copies it into the workspace.  Invalidates the smoother. */
int pns_set_state(pns_ctx* ctx, const pns_model* model, const double* u_k_dev);

/* Select the apply mode (default PNS_APPLY_RECOMPUTE).  Switching to CACHED
 * after pns_set_state builds the cache from the current state; returns
 * PNS_EINVAL for an unknown mode, PNS_EUNSUPPORTED for CACHED on a 3D
 * context (3D actions always recompute the tangent). */
int pns_set_apply_mode(pns_ctx* ctx, int mode);

/* Select the finest-level patch matrices (default PNS_PATCH_SURROGATE); a
 * change takes effect at the next pns_vanka_setup (until then the context has
 * no smoother).  PNS_EINVAL for an unknown kind.  On a hexahedral context
 * with a workspace bound that is too small for the new kind's level-0
 * storage: PNS_EWORKSPACE, kind unchanged (state and action data are kept
 * either way).  PNS_PATCH_EXACT restricts
 * the exact slab operator (each Radau node with its own state); on hexahedra
 * it is needed when the velocity varies by O(1) across the slab, where the
 * midpoint-frozen surrogate stops preconditioning. */
int pns_set_patch_kind(pns_ctx* ctx, int kind);

/* Storage precision of the Jacobian action that pns_solve's FGMRES applies
 * (Sec. 6.1; the mixed-precision pattern of iterative refinement): PNS_BF16 on
 * a hexahedral PNS_FP32 context stores the Krylov vector and the state u_k in
 * BF16 (rounded to nearest even from FP64) for that action, with FP32
 * arithmetic (power law in FP64) and an FP32 result widened to FP64; the
 * V-cycle preconditioner stays FP32 with its FP64 coarsest solve, the
 * residual, norms and Krylov vectors FP64.  The context precision (the
 * default) switches it back.  Query pns_solve_workspace_bytes after setting
 * it (the BF16 staging adds 2 N_st + 4 n_v bytes).  PNS_EINVAL for an unknown
 * precision; PNS_EUNSUPPORTED for BF16 on other contexts or for a precision
 * other than the context's. */
int pns_set_jacobian_precision(pns_ctx* ctx, int precision);

/* y = J_n(u_k) x on level 0, eq. (slab-underint-jac): the temporal mass
 * coupling K_t (x) M_x plus tau M_t (x) diag(J_1, J_2), each J_mu the spatial
 * linearisation of Sec. 5.2 (viscous volume term with the selected tangent,
 * convection, pressure coupling, boundary flux and Nitsche terms) at u_k of
 * Radau node mu.  Matrix-free; x, y in the context precision, canonical
 * layout, must not alias.  On quadrilaterals the cell contributions inside
 * a tile are summed with LDS atomics by default, so the last bits of y may
 * vary from call to call (pns_set_reproducible selects a fixed order); on
 * hexahedra every sum has a fixed order (bitwise reproducible). */
int pns_cell_apply(pns_ctx* ctx, const void* x_dev, void* y_dev);

/* Summation order of the quadrilateral action, defect and FP64 residual
 * (a property of the implementation, not of the method): on = 1 sums the
 * cell contributions of each tile in a fixed order (the four parity classes
 * of cells one after the other, boundary faces side by side), so repeated
 * calls on the same inputs give bitwise equal results; on = 0 (the default)
 * uses LDS atomics, which is faster.  Both agree with the oracle to rounding.
 * Hexahedral contexts always sum in a fixed order.  PNS_EINVAL for on other
 * than 0 or 1. */
int pns_set_reproducible(pns_ctx* ctx, int on);

/* Same operator as pns_cell_apply, y = b - J_n x (the global defect). */
int pns_cell_defect(pns_ctx* ctx, const void* b_dev, const void* x_dev, void* y_dev);

/* Build the smoother of every level (Sec. 6.3): level 0 patch matrices from
 * the surrogate operator with all state-dependent coefficients frozen at the
 * slab midpoint, eq. (surrogate-diag); coarse operators A_{l+1} = P^T A_l P
 * formed element by element; exact coarse patch matrices; LU-based inverses
 * of every patch; dense inverse of the coarsest operator with the constant
 * pressure coefficient of cell 0 pinned at each Radau node.
 * node_masks (host, may be NULL): one uint16 per level-0 cell, bit a set if
 * local Q2 node a (a = ax + 3 ay) belongs to that cell's patch; dropped nodes
 * are removed from the patch (uneven patches).  Returns PNS_ESINGULAR if a
 * patch has a zero pivot.
 * 3D contexts: the 85 x 85 spatial cell matrices at the midpoint
 * state are formed in FP64, each cell patch (27 nodes x 3 components + 4
 * pressure coefficients per Radau node, 170 unknowns) is summed from the 27
 * cells around it and inverted in time-diagonal form (one complex 85 x 85
 * Gauss-Jordan inversion with partial pivoting, FP64, stored in the context
 * precision), or with PNS_PATCH_EXACT real 170 x 170 patches of the exact
 * operator (FP64 Gauss-Jordan); coarse levels as above with real 170 x 170
 * patches, the coarsest level without patches; node_masks must be NULL
 * (PNS_EUNSUPPORTED otherwise). */
int pns_vanka_setup(pns_ctx* ctx, const uint16_t* node_masks);

/* n_sweeps additive Vanka steps on level `level`, eq. (stmg-vanka-update):
 * d <- d + omega sum_K R_K^T A_K^{-1} R_K (r - A_l d), in place on d.
 * PNS_EINVAL for the coarsest level of a 3D context with two or more levels
 * (it holds the dense inverse, no patches). */
int pns_vanka_smooth(pns_ctx* ctx, int level, int n_sweeps, double omega, const void* r_dev,
                     void* d_dev);

/* For callers that cannot allocate device memory or reserve per-context
 * scratch (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same n_sweeps additive Vanka steps as
 * pns_vanka_smooth (same kernels, same arguments, d updated in place), with
 * the buffers that are neither inputs nor outputs -- the defect r - A_l d of
 * each step, the tile-edge partial sums of the quadrilateral level-0 action,
 * the per-patch result slots of the quadrilateral coarse levels, the per-cell
 * result slots of the hexahedral actions -- taken from a static
 * device array of the library (64 MiB, one per GPU, held until the process
 * ends) instead of the bound workspace.  Allocates nothing: no hipMalloc, no
 * allocating library call.  Nothing in that array has to start at zero (every
 * call writes each scratch value before reading it).  All calls on one GPU
 * share the array, so calls that overlap on one GPU (several streams, several
 * threads, or a pns_vanka_smooth_static of another context still running)
 * race; serialise them.  PNS_EINVAL, before any device work, when the level
 * needs more than 64 MiB of scratch (the defect is N_st values of the context
 * precision, plus 2D level 0: 3 KB per 16 x 8 tile; 2D coarser levels: 42
 * values per cell; 3D: 170 values per cell;
 * e.g. a 256 x 256 FP64 level 0 needs 13.2 MB, 512 x 512 FP64 53 MB, 32^3
 * FP64 60 MB), otherwise the errors of pns_vanka_smooth. */
int pns_vanka_smooth_static(pns_ctx* ctx, int level, int n_sweeps, double omega,
                            const void* r_dev, void* d_dev);

/* Tile shapes of the batched patch sweeps (Sec. 6.3 additive Vanka step),
 * chosen on the device by an autotuner.  Each patch form has several kernel
 * variants that compute
 * the same additive step with different workgroup sizes (waves per
 * workgroup), column loads in flight and rows per lane; the first
 * pns_vanka_setup in a process that meets a level shape (cells in x and y,
 * patch form, precision) runs every variant of every level once on zero
 * vectors, times three further runs with events on the context stream and
 * keeps the fastest; later setups and contexts with the same shapes reuse
 * the choices without timing.  Variants differ only in time and in the
 * summation order inside a patch.
 *   pns_sweep_variant: out = {chosen variant, number of variants of the
 *     level's form, waves per workgroup, column loads in flight, rows per
 *     lane};
 *   pns_sweep_variant_time: the autotuner's mean time (ms) of one step of
 *     `variant` on `level` in this context (0 if the context reused an
 *     earlier choice or has not been set up);
 *   pns_set_sweep_variant: use `variant` on `level` until the next
 *     pns_vanka_setup (drops a captured V-cycle graph).
 * PNS_EINVAL for a bad level or variant and on 3D contexts. */
int pns_sweep_variant(const pns_ctx* ctx, int level, int out[5]);
int pns_sweep_variant_time(const pns_ctx* ctx, int level, int variant, double* ms);
int pns_set_sweep_variant(pns_ctx* ctx, int level, int variant);

/* d = V(r): one V-cycle over all levels (Sec. 6.3 "Hierarchy and coarse
 * operators": levels l = 0 .. L-1 with A_{l+1} = P^T A_l P; Sec. 6.3 "Vanka
 * smoothing": nu1 pre- and nu2 post-smoothing steps of eq. stmg-vanka-update
 * on every level but the coarsest).  From d = 0: nu1 steps, restriction
 * P^T of the defect, recursion, coarsest dense solve, prolongation-add,
 * nu2 steps.  r_dev, d_dev: level-0 vectors in the context precision,
 * canonical layout, caller-owned, must not alias; d is overwritten.
 * PNS_EUNSUPPORTED if the coarsest level exceeds the dense-solve limit, and
 * on 3D contexts with one level.  On hexahedra each vertex lies in 8 cell
 * patches; the additive step needs a smaller omega there (about 0.15) than on
 * quadrilaterals for the V-cycle to precondition well. */
int pns_vcycle(pns_ctx* ctx, int nu1, int nu2, double omega, const void* r_dev, void* d_dev);

/* enable = 1: pns_vcycle (and so the preconditioner of pns_solve) replays one
 * HIP graph holding the whole V-cycle of the operator sequence above, instead
 * of launching its ~100 kernels one by one; the launch overhead of the small
 * coarse-level grids goes away, the arithmetic is the same.  The graph is
 * captured at the first V-cycle on a stream the library creates (default
 * priority), is keyed on (nu1, nu2, omega) and is dropped by pns_set_state,
 * pns_vanka_setup, pns_set_apply_mode, pns_set_patch_kind and
 * pns_bind_workspace; r and d pass through two workspace vectors (two copies
 * per V-cycle).  enable = 0 returns to eager launches.  PNS_EINVAL for other
 * values, PNS_EUNSUPPORTED on BF16 contexts (no V-cycle). */
int pns_set_vcycle_graph(pns_ctx* ctx, int enable);

/* y = A_l x with the level-l operator (level 0: pns_cell_apply; coarser:
 * the Galerkin operator applied element by element).  Needs pns_vanka_setup
 * for level > 0. */
int pns_level_apply(pns_ctx* ctx, int level, const void* x_dev, void* y_dev);

/* Transfers between level l (fine) and l+1 (coarse): rc = P^T rf and
 * df += P dc, P the nested Q2 interpolation / P1disc restriction. */
int pns_restrict(pns_ctx* ctx, int level, const void* rf_dev, void* rc_dev);
int pns_prolongate_add(pns_ctx* ctx, int level, const void* dc_dev, void* df_dev);

/* ------------------------------------------------------------- slab solve */

/* R = R_n(U), the slab residual of eq. (slab-underint) with f = 0 and g_D = 0
 * (Sec. 5.2), in FP64 whatever the context precision:
 *   R_v,mu = -( sum_nu K_t[mu][nu] M_x u_nu - m_t[mu] M_x v_prev ) - tau w_mu A_gamma(U_mu)_v,
 *   R_p,mu = - tau w_mu A_gamma(U_mu)_p,
 * with A_gamma the nonlinear form of eqs. pns-form, def-a-gam, def-b-gam and the
 * inflow factor (u.n)^- of B^c evaluated at U itself.
 * U_dev, R_dev: FP64 device vectors, canonical layout of level 0, must not
 * alias.  v_prev_dev: FP64 device vector of the left-trace velocity
 * (component 0 over the Q2 nodes, then component 1), or NULL for zero.
 * Needs a bound workspace, not a state.  Asynchronous on the context stream.
 * Hexahedra: v_prev holds 3 components; R is evaluated as the Picard
 * linearisation at U applied to U (which reproduces every nonlinear term of
 * A_gamma, the inflow factor included) plus the left-trace term, in FP64. */
int pns_residual(pns_ctx* ctx, const pns_model* model, const double* U_dev,
                 const double* v_prev_dev, double* R_dev);

/* Volume force (the f-term of eq. disc-residual on one slab, with the Radau
 * rule of eq. slab-underint): F_v,mu = tau w_mu (f(t_mu), phi)_Omega, each
 * cell integrated with its 3^d-point Gauss rule; F_p = 0.  f_qp_dev (FP64,
 * device): f at the Gauss points of every cell at both Radau nodes,
 * f_qp[((mu * cells + cell) * 3^d + q) * d + comp], cells lexicographic
 * (x fastest), q = qx + 3 qy (+ 9 qz) over the points x_c + h (g_qx, g_qy
 * [, g_qz]) - x_c the cell's low corner, g = 1/2 - sqrt(3/5)/2, 1/2,
 * 1/2 + sqrt(3/5)/2 -, t_mu = t0 + tau (1/3, 1).  F_dev: FP64 device vector
 * of N_st values (canonical layout), overwritten.  Needs no workspace. */
int pns_load_vector(pns_ctx* ctx, const double* f_qp_dev, double* F_dev);

/* Register a load vector F (FP64 device vector of N_st values, e.g. from
 * pns_load_vector; caller-owned, read at every use) that pns_residual,
 * pns_solve and pns_march add to every slab residual, R_n(U) + F; NULL (the
 * default) for f = 0.  pns_march adds the same F to each of its slabs. */
int pns_set_load(pns_ctx* ctx, const double* F_dev);

/* Inhomogeneous Dirichlet data (Sec. 3.2, eq. def-b-gam; the B_gamma(g_D, .)
 * term of eq. disc-residual).  ghat_dev (FP64, device, caller-owned, read at
 * every use): a lifting ghat_D of the data as a Q2 velocity field per Radau
 * node, 2 N_v values (node 0's velocity layout, then node 1's) on the level-0
 * mesh; g_D is its trace on the boundary.  The viscous Nitsche coefficients
 * are frozen at G = D ghat_D, evaluated at each boundary face point from the
 * boundary cell's field: eta(G) in the penalty and the exact stress
 * derivative DS(G) in the symmetry term, in the Jacobian action, the residual,
 * the patches and the Galerkin coarse operators (the surrogate patches take
 * the lifting at the slab midpoint); the residual adds B_gamma(g_D, .) (inflow,
 * symmetry and penalty terms at the trace).  NULL (the default): homogeneous
 * data, eta_D = eta(0).  The lifting is evaluated at the boundary face points
 * (a small table in the workspace) for the model of pns_set_state and of each
 * pns_residual / pns_solve call, so it is read again at each of those calls.
 * A smoother built before the call is invalidated (pns_vanka_setup again).
 * Needs a bound workspace (PNS_EWORKSPACE); rebinding one clears the state, not
 * the registration.  Quadrilaterals and hexahedra (the 3D action, residual,
 * smoother and solve); PNS_EUNSUPPORTED in a BF16 context.  Serving requests
 * use homogeneous data. */
int pns_set_dirichlet(pns_ctx* ctx, const double* ghat_dev);

/* Parameters of pns_solve. */
typedef struct {
  int max_newton;     /* nonlinear iterations */
  int max_krylov;     /* FGMRES iterations per linear solve */
  int restart;        /* FGMRES restart length (Krylov vectors kept), 1..200 */
  double rtol, atol;  /* stop at ||R||_M <= max(atol, rtol ||R(U^0)||_M), eq. (nk-stop) */
  double eta0;        /* forcing term of the first linear solve */
  double eta_max;     /* upper bound of the forcing terms */
  double rho;         /* refresh the smoother when ||R_{m+1}||_M / ||R_m||_M > rho */
  int nu1, nu2;       /* Vanka steps before / after the coarse correction */
  double omega;       /* Vanka damping */
} pns_solve_params;

/* What pns_solve did. */
typedef struct {
  int newton_iterations;    /* accepted Newton steps */
  int krylov_iterations;    /* FGMRES iterations, all steps */
  int smoother_setups;      /* smoother (re)builds */
  int backtracks;           /* Armijo halvings, all steps */
  double residual_initial;  /* ||R(U^0)||_M */
  double residual_final;    /* ||R(U)||_M on return */
} pns_solve_info;

/* Device bytes of the pns_solve work buffer for FGMRES restart length `restart`
 * ((2 restart + 7) vectors of N_st doubles, plus FP32 staging in an FP32
 * context); 0 for a NULL context or restart outside 1..200. */
size_t pns_solve_workspace_bytes(const pns_ctx* ctx, int restart);

/* Newton-Krylov solve of R_n(U) = 0 on the slab (Sec. 6 eq. nk-newton-lin; Sec. 6.1
 * eq. nk-inexact-newton; Sec. 6.2 eq. nk-stop): at each iterate U^m the linearisation model->lin
 * acts matrix-free as J_n; FGMRES, right-preconditioned by one V-cycle,
 * solves J_n dU = R_n(U^m) until ||J_n dU - R_n||_M <= eta_m ||R_n||_M, with
 * Eisenstat-Walker forcing terms (choice 2, gamma 0.9, exponent 2) and FP64
 * classical Gram-Schmidt with one reorthogonalisation in the block mass inner
 * product of the time step (tau M_t (x) blockdiag(M_x, M_p)), whose norm
 * ||.||_M measures every residual; then U^{m+1} = U^m + lambda dU, lambda
 * halved until ||R(U^{m+1})||_M <= (1 - 1e-4 lambda (1 - eta_m)) ||R(U^m)||_M
 * (Armijo on ||R||_M^2 / 2).  The smoother is built at the first step and
 * rebuilt at the state of a later step when the previous step's residual
 * ratio exceeded rho or its FGMRES count more than doubled (Sec. 6.3,
 * "Interpretation and refresh strategy"), and once more, with the linear
 * solve repeated, when a solve with a smoother from an earlier iterate misses
 * its forcing term; the Jacobian action always uses the current iterate.  In an FP32 context the Jacobian action and the V-cycle run
 * in FP32 (coarsest solve in FP64) while the residual, the norms and the
 * Krylov vectors stay FP64.
 * U_dev: FP64 device vector, the initial guess on entry, the last iterate on
 * return.  v_prev_dev as for pns_residual.  work_dev: device buffer, 256-byte
 * aligned, of at least pns_solve_workspace_bytes(ctx, prm->restart) bytes.
 * Overwrites the context's state and smoother.  Synchronous: returns when the
 * solve has finished on the context stream; *info is filled when non-NULL.
 * Returns PNS_OK on convergence; PNS_ENOTCONV when max_newton is reached, the
 * line search fails or a linear solve misses its forcing term within
 * max_krylov iterations; PNS_ENONFINITE when the initial residual, a trial
 * residual of every backtracking step or the FGMRES residual estimate is not
 * finite (a NaN or infinity in U, v_prev or the model's output): U is then
 * left at the last finite iterate; PNS_EUNSUPPORTED when the coarsest level
 * is too large for the dense coarse solve. */
int pns_solve(pns_ctx* ctx, const pns_model* model, const double* v_prev_dev, double* U_dev,
              const pns_solve_params* prm, void* work_dev, size_t work_bytes,
              pns_solve_info* info);

/* Time marching over n_slabs consecutive slabs of length tau (Sec. 3.1: the
 * dG(1) slabs are coupled only through the left trace v^-): for each slab,
 * U starts from v at both Radau nodes with zero pressure, pns_solve runs with
 * v as v^-, and the velocity at the second Radau node (the slab's end point,
 * which the right Radau rule contains) becomes v for the next slab.
 * v_dev (FP64, n_v values): in, the velocity at the start; out, at the end of
 * the last solved slab.  U_dev (FP64, N_st): out, the last slab's solution.
 * work as for pns_solve.  info: the sums of the iteration counts over the
 * slabs, residual_initial of the first and residual_final of the last slab
 * solved.  Returns the first failing pns_solve code (PNS_ENOTCONV: the
 * slab that did not converge is left in U_dev and v_dev holds the start of
 * that slab); n_slabs = 0 leaves v_dev unchanged. */
int pns_march(pns_ctx* ctx, const pns_model* model, double* v_dev, int n_slabs, double* U_dev,
              const pns_solve_params* prm, void* work_dev, size_t work_bytes,
              pns_solve_info* info);

/* ---------------------------------------------------------------- serving */

/* A request server for independent slab solves (each one the Newton-Krylov
 * solve of pns_solve on its own mesh and model).  `slots` requests run at
 * once, each on its own HIP stream driven by its own host worker thread, so
 * the kernels of different requests overlap on the device.  Requests are
 * admitted in arrival order as a slot and room in the device arena free up;
 * a request that does not fit yet lets smaller later ones start (backfill).
 * The server allocates no device memory: every running request takes its
 * workspace, Krylov vectors and solution vector from the caller's arena and
 * returns them on completion.  All entry points are thread-safe. */
typedef struct pns_server pns_server;

typedef struct {
  int n_cells[2];            /* mesh n_x x n_y of the box [lo, hi] */
  double lo[2], hi[2];
  double tau;                /* slab length */
  int n_levels;              /* multigrid levels; the coarsest must fit the dense solve */
  int precision;             /* PNS_FP64, or PNS_FP32 for the mixed-precision solve */
  int patch_kind;            /* pns_patch_kind of the finest level */
  pns_model model;
  pns_solve_params params;
  const double* v_prev_host; /* left-trace velocity, host, 2 (2n_x+1)(2n_y+1) doubles; copied
                                at submission, the copy released once it is on the device */
  double* U_host;            /* host buffer of N_st doubles receiving the last iterate */
  int vcycle_graph;          /* 1: the request's V-cycles replay a captured HIP graph
                                (pns_set_vcycle_graph), 0: eager launches */
} pns_request;

enum { PNS_REQ_QUEUED = 0, PNS_REQ_RUNNING = 1, PNS_REQ_DONE = 2 };

typedef struct {
  int state;                 /* PNS_REQ_QUEUED / RUNNING / DONE */
  int status;                /* return code of the solve once DONE */
  pns_solve_info info;
  double t_submit, t_start, t_done;  /* seconds on the server's steady clock */
  size_t footprint;          /* arena bytes the request holds while running */
} pns_result;

/* Arena bytes one request needs (context workspace, solve work buffer, U and
 * v_prev, alignment); 0 if the request is invalid. */
size_t pns_request_footprint(const pns_request* req);

/* Create a server on the current device with `slots` (1..16) concurrent
 * solves working in [arena_dev, arena_dev + arena_bytes) (device memory,
 * 256-byte aligned, owned by the caller, untouched outside running requests).
 * PNS_EINVAL for bad arguments, PNS_EHIP if a stream cannot be created. */
int pns_server_create(int slots, void* arena_dev, size_t arena_bytes, pns_server** out);

/* Queue a request (Sec. 6-6.2 slab solve, as pns_solve); the request struct and
 * v_prev_host are copied, U_host must stay valid until the request is DONE.
 * The solve starts from U = 0; if that attempt stops with PNS_ENOTCONV, a
 * second one starts from the left trace at both Radau nodes (zero pressure),
 * and the result's status, residuals and iterate are the second attempt's,
 * its iteration counts the sums over both.
 * *ticket identifies it.  PNS_EINVAL if the request is invalid,
 * PNS_EWORKSPACE if its footprint exceeds the whole arena. */
int pns_solve_request(pns_server* srv, const pns_request* req, uint64_t* ticket);

/* State of a request, without blocking; PNS_EINVAL for an unknown ticket. */
int pns_poll(pns_server* srv, uint64_t ticket, pns_result* out);

/* Block until the request is DONE, then as pns_poll. */
int pns_wait(pns_server* srv, uint64_t ticket, pns_result* out);

/* Forget a finished request: its result can no longer be polled and the
 * server's host memory for it is freed (a long-running server calls this
 * for every ticket it has waited for).  PNS_EINVAL for an unknown ticket,
 * PNS_ESTATE if the request is not DONE yet (nothing changes then). */
int pns_release(pns_server* srv, uint64_t ticket);

/* Finish every queued and running request, then release the streams and
 * worker threads. */
void pns_server_destroy(pns_server* srv);

#ifdef __cplusplus
}
#endif
#endif
