// Newton-Krylov slab solve (Sec. 6, eq. nk-newton-lin; Sec. 6.1 Krylov solver,
// Sec. 6.2 globalisation and stopping): FP64 residual and norms, FGMRES with a
// V-cycle preconditioner, Eisenstat-Walker forcing, Armijo backtracking,
// smoother refresh on deterioration (Sec. 6.3).  Host-side sequencing of
// device kernels on the context stream; the small Hessenberg least-squares
// problem of FGMRES is solved on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace pns;

namespace {

constexpr int kMaxRestart = 200;
constexpr double kArmijo = 1e-4;
constexpr int kMaxBacktrack = 30;
constexpr double kEwGamma = 0.9;  // Eisenstat-Walker choice 2: gamma (r_m / r_{m-1})^2

int fail(pns_ctx* c, int code, const std::string& msg) { return fail_msg(&c->err, code, msg); }

struct Work {
  int m = 0;
  int64_t n = 0;
  double* V = nullptr;   // m + 1 Krylov vectors
  double* Z = nullptr;   // m preconditioned vectors
  double* R = nullptr;   // residual at U
  double* Rt = nullptr;  // residual at the trial point
  double* Ut = nullptr;  // trial point
  double* dU = nullptr;  // Newton correction
  double* w = nullptr;   // Arnoldi vector
  double* Mw = nullptr;  // mass times a vector
  double* uk = nullptr;  // velocity blocks of U (linearisation state)
  double* part = nullptr;
  double* h = nullptr;   // device scalars
  float* x32 = nullptr;  // FP32 staging (FP32 context)
  float* y32 = nullptr;
  uint16_t* x16 = nullptr;   // BF16 Jacobian action: the Krylov vector and the state in BF16
  uint16_t* uk16 = nullptr;
};

size_t work_layout(const pns_ctx* c, int m, char* base, Work* w) {
  const Grid& g = c->lev[0].g;
  const int64_t n = g.nst;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + kAlign - 1) / kAlign * kAlign;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  Work t;
  t.m = m;
  t.n = n;
  t.V = (double*)take((size_t)(m + 1) * n * 8);
  t.Z = (double*)take((size_t)m * n * 8);
  t.R = (double*)take(n * 8);
  t.Rt = (double*)take(n * 8);
  t.Ut = (double*)take(n * 8);
  t.dU = (double*)take(n * 8);
  t.w = (double*)take(n * 8);
  t.Mw = (double*)take(n * 8);
  t.uk = (double*)take(2 * g.nv * 8);
  t.part = (double*)take((size_t)(m + 2) * dot_partials() * 8);
  t.h = (double*)take((size_t)(2 * m + 8) * 8);
  if (c->es == 4) {
    t.x32 = (float*)take(n * 4);
    t.y32 = (float*)take(n * 4);
  }
  if (c->jac_bf16) {
    t.x16 = (uint16_t*)take(n * 2);
    t.uk16 = (uint16_t*)take(2 * g.nv * 2);
  }
  if (w) *w = t;
  return (off + kAlign - 1) / kAlign * kAlign;
}

// Hexahedra: the FP64 slab residual from the fixed-point form of the Picard
// linearisation.  With the state taken at U itself (tangent eta(DU) I,
// advecting field U, inflow factor (U.n)^- at U) the Picard operator applied
// to U reproduces every term of the nonlinear form, so
//   R(U) = [m_t (x) M_x v_prev ; 0] - J_Picard(U) U,
// one FP64 3D action in defect mode with b = the left-trace term.
int residual3d(pns_ctx* c, const Model& m, const double* U, const double* vprev, double* R) {
  const Level& L = c->lev[0];
  const Grid3& g = L.g3;
  hipStream_t s = c->stream;
  if (vprev) {
    // stage (v_prev, 0, v_prev, 0) in R, then b = (m_t[0] M v, 0, m_t[1] M v, 0)
    PNS_HIP(c, launch_fill<double>(g.nst, 0.0, R, s));
    PNS_HIP(c, launch_copy<double>(g.nv, vprev, R, s));
    PNS_HIP(c, launch_copy<double>(g.nv, vprev, R + g.ns, s));
    PNS_HIP(c, launch_mass3(g, 1.5, -0.5, 0.0, R, c->r3b, s));
  } else {
    PNS_HIP(c, launch_fill<double>(g.nst, 0.0, c->r3b, s));
  }
  if (m.lift) {
    // b += B_gamma(g_D, .): the data term per cell into the slots, gathered as
    // b - sum with slots holding its negative
    PNS_HIP(c, launch_lift3_rhs(g, m, c->disc.tau, m.lift, c->r3slot, s));
    PNS_HIP(c, launch_gather3<double>(g, c->r3slot, c->r3b, c->r3b, s));
  }
  PNS_HIP(c, hipMemcpyAsync(c->r3u, U, g.nv * 8, hipMemcpyDeviceToDevice, s));
  PNS_HIP(c, hipMemcpyAsync(c->r3u + g.nv, U + g.ns, g.nv * 8, hipMemcpyDeviceToDevice, s));
  Model mp = m;
  mp.lin = PNS_PICARD;
  PNS_HIP(c, launch_cell_apply3d<double>(g, mp, c->disc.tau, c->r3u, U, c->r3b, R, c->r3slot, 1,
                                         s));
  return PNS_OK;
}

struct Solver {
  pns_ctx* c;
  const pns_model* md;
  Model model;
  const double* vprev;
  Work W;
  Grid g;
  hipStream_t s;
  pns_solve_params prm;

  // ||x||_M; h[0] receives x . M x
  // W.Mw = M x, the block mass of the time step (the inner product of FGMRES)
  hipError_t mass(const double* x) {
    if (c->dim == 3)
      return launch_mass3(c->lev[0].g3, c->disc.tau * kWt[0], c->disc.tau * kWt[1], 1.0, x, W.Mw,
                          s);
    return launch_mass(g, c->disc.tau, x, W.Mw, s);
  }

  int mnorm(const double* x, double* out) {
    PNS_HIP(c, mass(x));
    PNS_HIP(c, launch_multi_dot(W.n, 1, x, W.n, W.Mw, W.part, W.h, s));
    double v = 0.0;
    PNS_HIP(c, hipMemcpyAsync(&v, W.h, 8, hipMemcpyDeviceToHost, s));
    PNS_HIP(c, hipStreamSynchronize(s));
    *out = std::sqrt(std::max(v, 0.0));
    return PNS_OK;
  }

  int residual(const double* U, double* R) {
    if (c->dim == 3) {
      const int rc = residual3d(c, model, U, vprev, R);
      if (rc != PNS_OK) return rc;
    } else {
      PNS_HIP(c, launch_residual(g, model, c->disc.tau, U, vprev, R, s));
      if (model.gamma_cip > 0.0)
        PNS_HIP(c, launch_cip<double>(g, model, c->disc.tau, U, g.ns, U, R, -1.0, c->cipG, s));
    }
    if (c->load) PNS_HIP(c, launch_add(W.n, c->load, R, s));
    return PNS_OK;
  }

  // z = V-cycle(v) in the context precision
  int precondition(const double* v, double* z) {
    int rc;
    if (c->es == 8) return pns_vcycle(c, prm.nu1, prm.nu2, prm.omega, v, z);
    PNS_HIP(c, launch_narrow(W.n, v, W.x32, s));
    if ((rc = pns_vcycle(c, prm.nu1, prm.nu2, prm.omega, W.x32, W.y32)) != PNS_OK) return rc;
    PNS_HIP(c, launch_widen(W.n, W.y32, z, s));
    return PNS_OK;
  }

  // y = J_n x in the context precision (x and u_k in BF16 with FP32
  // arithmetic when the context asks for it)
  int jacobian(const double* x, double* y) {
    int rc;
    if (c->es == 8) return pns_cell_apply(c, x, y);
    if (c->jac_bf16) {
      PNS_HIP(c, launch_to_bf16(W.n, x, W.x16, s));
      PNS_HIP(c, launch_cell_apply3d_bf16(c->g3, c->model, c->disc.tau, W.uk16, W.x16, nullptr,
                                          W.y32, (float*)c->E3, 0, s));
      PNS_HIP(c, launch_widen(W.n, W.y32, y, s));
      return PNS_OK;
    }
    PNS_HIP(c, launch_narrow(W.n, x, W.x32, s));
    if ((rc = pns_cell_apply(c, W.x32, W.y32)) != PNS_OK) return rc;
    PNS_HIP(c, launch_widen(W.n, W.y32, y, s));
    return PNS_OK;
  }

  // linearisation state: the velocity blocks of U at both Radau nodes
  int set_state(const double* U, bool keep_smoother) {
    const bool had = c->has_smoother;
    PNS_HIP(c, hipMemcpyAsync(W.uk, U, g.nv * 8, hipMemcpyDeviceToDevice, s));
    PNS_HIP(c, hipMemcpyAsync(W.uk + g.nv, U + g.ns, g.nv * 8, hipMemcpyDeviceToDevice, s));
    int rc = pns_set_state(c, md, W.uk);
    if (rc != PNS_OK) return rc;
    if (c->jac_bf16) PNS_HIP(c, launch_to_bf16(2 * g.nv, W.uk, W.uk16, s));
    // the smoother's patch inverses and coarse operators are untouched by a
    // new state; keep them when no refresh is due
    if (keep_smoother) c->has_smoother = had;
    return PNS_OK;
  }

  // FGMRES(m) for J dU = b (dU = 0 initially), stops at ||b - J dU||_M <= tol
  int fgmres(const double* b, double bnorm, double tol, int* its, double* achieved) {
    const int m = W.m;
    const int64_t n = W.n;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gvec(m + 1), y(m), hv(m + 1);
    PNS_HIP(c, launch_fill<double>(n, 0.0, W.dU, s));
    *its = 0;
    double beta = bnorm;
    *achieved = beta;
    if (beta <= tol) return PNS_OK;
    const double* r = b;
    while (true) {
      PNS_HIP(c, launch_axpby(n, 1.0 / beta, r, 0.0, nullptr, W.V, s));
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(gvec.begin(), gvec.end(), 0.0);
      gvec[0] = beta;
      int j = 0, jend = 0;
      double res = beta;
      for (j = 0; j < m; ++j) {
        double* vj = W.V + (int64_t)j * n;
        double* zj = W.Z + (int64_t)j * n;
        int rc;
        if ((rc = precondition(vj, zj)) != PNS_OK) return rc;
        if ((rc = jacobian(zj, W.w)) != PNS_OK) return rc;
        // classical Gram-Schmidt in the M inner product, twice
        for (int pass = 0; pass < 2; ++pass) {
          PNS_HIP(c, mass(W.w));
          PNS_HIP(c, launch_multi_dot(n, j + 1, W.V, n, W.Mw, W.part, W.h, s));
          PNS_HIP(c, launch_combine(n, j + 1, W.V, n, W.h, -1.0, 1.0, W.w, s));
          PNS_HIP(c, hipMemcpyAsync(hv.data(), W.h, (j + 1) * 8, hipMemcpyDeviceToHost, s));
          PNS_HIP(c, hipStreamSynchronize(s));
          for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] += hv[i];
        }
        double hn;
        if ((rc = mnorm(W.w, &hn)) != PNS_OK) return rc;
        H[(size_t)(j + 1) * m + j] = hn;
        // Givens rotations of the Hessenberg column
        for (int i = 0; i < j; ++i) {
          const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
          H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
        }
        const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
        const double rr = std::hypot(a, bb);
        cs[j] = rr > 0.0 ? a / rr : 1.0;
        sn[j] = rr > 0.0 ? bb / rr : 0.0;
        H[(size_t)j * m + j] = rr;
        H[(size_t)(j + 1) * m + j] = 0.0;
        gvec[j + 1] = -sn[j] * gvec[j];
        gvec[j] = cs[j] * gvec[j];
        res = std::fabs(gvec[j + 1]);
        ++*its;
        jend = j + 1;
        if (res <= tol || *its >= prm.max_krylov || !(hn > 0.0)) break;
        PNS_HIP(c, launch_axpby(n, 1.0 / hn, W.w, 0.0, nullptr, W.V + (int64_t)(j + 1) * n, s));
      }
      // y = H^{-1} g (upper triangular), dU += Z y
      for (int i = jend - 1; i >= 0; --i) {
        double t = gvec[i];
        for (int k = i + 1; k < jend; ++k) t -= H[(size_t)i * m + k] * y[k];
        const double d = H[(size_t)i * m + i];
        y[i] = d != 0.0 ? t / d : 0.0;
      }
      PNS_HIP(c, hipMemcpyAsync(W.h, y.data(), jend * 8, hipMemcpyHostToDevice, s));
      PNS_HIP(c, launch_combine(n, jend, W.Z, n, W.h, 1.0, 1.0, W.dU, s));
      PNS_HIP(c, hipStreamSynchronize(s));  // y is read by the copy above
      *achieved = res;
      if (res <= tol || *its >= prm.max_krylov) break;
      // restart from the true residual b - J dU
      int rc;
      if ((rc = jacobian(W.dU, W.w)) != PNS_OK) return rc;
      PNS_HIP(c, launch_axpby(n, 1.0, b, -1.0, W.w, W.Rt, s));
      if ((rc = mnorm(W.Rt, &beta)) != PNS_OK) return rc;
      *achieved = beta;
      if (beta <= tol) break;
      r = W.Rt;
    }
    return PNS_OK;
  }
};

}  // namespace

extern "C" {

int pns_residual(pns_ctx* ctx, const pns_model* md, const double* U, const double* vprev,
                 double* R) {
  if (!ctx) return PNS_EINVAL;
  if (ctx->prec == PNS_BF16) return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (!ctx->ws) return fail(ctx, PNS_EWORKSPACE, "no workspace bound");
  if (!md || !U || !R || U == R || R == ctx->load)
    return fail(ctx, PNS_EINVAL, "NULL model or vectors, U == R, or R is the load vector");
  Model m;
  const int rc = make_model(md, &m, &ctx->err);
  if (rc != PNS_OK) return rc;
  if (ctx->dim == 3 && m.gamma_cip > 0.0)
    return fail(ctx, PNS_EUNSUPPORTED, "CIP stabilisation is built for quadrilaterals only");
  m.lift = nullptr;
  if (ctx->lift) {
    if (ctx->dim == 3)
      PNS_HIP(ctx, launch_lift3_table(ctx->g3, m, ctx->lift, ctx->ltab_r, ctx->stream));
    else
      PNS_HIP(ctx, launch_lift_table(ctx->lev[0].g, m, ctx->lift, ctx->ltab_r, ctx->stream));
    m.lift = ctx->ltab_r;
  }
  m.ordered = ctx->ordered ? 1 : 0;
  if (ctx->dim == 3) {
    const int rc = residual3d(ctx, m, U, vprev, R);
    if (rc != PNS_OK) return rc;
  } else {
    const Grid& g0 = ctx->lev[0].g;
    PNS_HIP(ctx, launch_residual(g0, m, ctx->disc.tau, U, vprev, R, ctx->stream));
    if (m.gamma_cip > 0.0)
      PNS_HIP(ctx, launch_cip<double>(g0, m, ctx->disc.tau, U, g0.ns, U, R, -1.0, ctx->cipG,
                                      ctx->stream));
  }
  if (ctx->load) PNS_HIP(ctx, launch_add(ctx->lev[0].g.nst, ctx->load, R, ctx->stream));
  return PNS_OK;
}

size_t pns_solve_workspace_bytes(const pns_ctx* ctx, int restart) {
  if (!ctx || ctx->prec == PNS_BF16 || restart < 1 || restart > kMaxRestart) return 0;
  return work_layout(ctx, restart, nullptr, nullptr);
}

int pns_solve(pns_ctx* ctx, const pns_model* md, const double* vprev, double* U,
              const pns_solve_params* prm, void* work, size_t work_bytes, pns_solve_info* info) {
  if (!ctx) return PNS_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  if (ctx->prec == PNS_BF16) return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (!ctx->ws) return fail(ctx, PNS_EWORKSPACE, "no workspace bound");
  if (!md || !U || !prm) return fail(ctx, PNS_EINVAL, "NULL model, U or parameters");
  if (prm->restart < 1 || prm->restart > kMaxRestart || prm->max_newton < 1 ||
      prm->max_krylov < 1 || prm->nu1 < 0 || prm->nu2 < 0 || !(prm->rtol >= 0.0) ||
      !(prm->atol >= 0.0) || !(prm->eta0 > 0.0 && prm->eta0 < 1.0) ||
      !(prm->eta_max >= prm->eta0 && prm->eta_max < 1.0) || !(prm->rho > 0.0))
    return fail(ctx, PNS_EINVAL, "invalid solve parameters");
  if (!ctx->has_coarse)
    return fail(ctx, PNS_EUNSUPPORTED, "coarsest level too large for the dense coarse solve");
  if (!work || ((uintptr_t)work % kAlign) != 0 ||
      work_bytes < work_layout(ctx, prm->restart, nullptr, nullptr))
    return fail(ctx, PNS_EWORKSPACE, "solve work buffer NULL, misaligned or too small");
  Solver S;
  S.c = ctx;
  S.md = md;
  int rc = make_model(md, &S.model, &ctx->err);
  if (rc != PNS_OK) return rc;
  S.model.lift = nullptr;
  if (ctx->lift) {
    if (ctx->dim == 3)
      PNS_HIP(ctx, launch_lift3_table(ctx->g3, S.model, ctx->lift, ctx->ltab_r, ctx->stream));
    else
      PNS_HIP(ctx, launch_lift_table(ctx->lev[0].g, S.model, ctx->lift, ctx->ltab_r,
                                     ctx->stream));
    S.model.lift = ctx->ltab_r;
  }
  S.model.ordered = ctx->ordered ? 1 : 0;
  S.vprev = vprev;
  S.g = ctx->lev[0].g;
  S.s = ctx->stream;
  S.prm = *prm;
  work_layout(ctx, prm->restart, (char*)work, &S.W);
  const int64_t n = S.W.n;
  hipStream_t s = ctx->stream;

  pns_solve_info inf{};
  if ((rc = S.residual(U, S.W.R)) != PNS_OK) return rc;
  double rnorm;
  if ((rc = S.mnorm(S.W.R, &rnorm)) != PNS_OK) return rc;
  if (!std::isfinite(rnorm)) {
    inf.residual_initial = inf.residual_final = rnorm;
    if (info) *info = inf;
    return fail(ctx, PNS_ENONFINITE, "initial residual is not finite (NaN or Inf in U or v_prev)");
  }
  const double r0 = rnorm;
  const double stop = std::max(prm->atol, prm->rtol * r0);
  inf.residual_initial = inf.residual_final = r0;
  bool refresh = true;
  int prev_its = 0;
  double eta = prm->eta0, rprev = r0;
  const char* why = "maximal number of Newton iterations reached";
  for (int it = 0; it < prm->max_newton && rnorm > stop; ++it) {
    if ((rc = S.set_state(U, !refresh)) != PNS_OK) return rc;
    if (refresh) {
      if ((rc = pns_vanka_setup(ctx, nullptr)) != PNS_OK) return rc;
      ++inf.smoother_setups;
    }
    if (it > 0) {
      // Eisenstat-Walker choice 2 with safeguard; never solve below what the
      // nonlinear stopping test needs
      double e = kEwGamma * (rnorm / rprev) * (rnorm / rprev);
      const double sg = kEwGamma * eta * eta;
      if (sg > 0.1) e = std::max(e, sg);
      eta = std::min(prm->eta_max, std::max(e, 0.5 * stop / rnorm));
    }
    int its = 0;
    double achieved = 0.0;
    if ((rc = S.fgmres(S.W.R, rnorm, eta * rnorm, &its, &achieved)) != PNS_OK) return rc;
    inf.krylov_iterations += its;
    if (!std::isfinite(achieved)) {
      PNS_HIP(ctx, hipStreamSynchronize(s));
      if (info) *info = inf;
      return fail(ctx, PNS_ENONFINITE, "FGMRES residual estimate is not finite");
    }
    if (achieved > eta * rnorm && !refresh) {
      // the smoother was built at an earlier iterate: rebuild it here and
      // solve again before declaring the linear solve failed
      if ((rc = S.set_state(U, false)) != PNS_OK) return rc;
      if ((rc = pns_vanka_setup(ctx, nullptr)) != PNS_OK) return rc;
      ++inf.smoother_setups;
      if ((rc = S.fgmres(S.W.R, rnorm, eta * rnorm, &its, &achieved)) != PNS_OK) return rc;
      inf.krylov_iterations += its;
      if (!std::isfinite(achieved)) {
        PNS_HIP(ctx, hipStreamSynchronize(s));
        if (info) *info = inf;
        return fail(ctx, PNS_ENONFINITE, "FGMRES residual estimate is not finite");
      }
    }
    if (achieved > eta * rnorm) {
      why = "FGMRES missed its forcing term within max_krylov iterations";
      break;
    }
    // Armijo backtracking on ||R||_M^2 / 2
    double lam = 1.0, rt = 0.0;
    bool ok = false, finite = false;
    for (int bt = 0; bt <= kMaxBacktrack; ++bt) {
      PNS_HIP(ctx, launch_axpby(n, 1.0, U, lam, S.W.dU, S.W.Ut, s));
      if ((rc = S.residual(S.W.Ut, S.W.Rt)) != PNS_OK) return rc;
      if ((rc = S.mnorm(S.W.Rt, &rt)) != PNS_OK) return rc;
      finite = finite || std::isfinite(rt);
      if (rt <= (1.0 - kArmijo * lam * (1.0 - eta)) * rnorm) {
        ok = true;
        break;
      }
      lam *= 0.5;
      ++inf.backtracks;
    }
    if (!ok && !finite) {
      PNS_HIP(ctx, hipStreamSynchronize(s));
      if (info) *info = inf;
      return fail(ctx, PNS_ENONFINITE, "every trial residual of the line search is not finite");
    }
    if (!ok) {
      why = "line search failed";
      break;
    }
    PNS_HIP(ctx, hipMemcpyAsync(U, S.W.Ut, n * 8, hipMemcpyDeviceToDevice, s));
    PNS_HIP(ctx, hipMemcpyAsync(S.W.R, S.W.Rt, n * 8, hipMemcpyDeviceToDevice, s));
    ++inf.newton_iterations;
    refresh = (rt / rnorm > prm->rho) || (prev_its > 0 && its > 2 * prev_its);
    prev_its = its;
    rprev = rnorm;
    rnorm = rt;
    inf.residual_final = rnorm;
  }
  PNS_HIP(ctx, hipStreamSynchronize(s));
  if (info) *info = inf;
  if (rnorm <= stop) return PNS_OK;
  return fail(ctx, PNS_ENOTCONV, why);
}

int pns_march(pns_ctx* ctx, const pns_model* md, double* v, int n_slabs, double* U,
              const pns_solve_params* prm, void* work, size_t work_bytes, pns_solve_info* info) {
  if (!ctx) return PNS_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  if (!md || !v || !U || !prm || n_slabs < 0 || (const void*)v == (const void*)U)
    return fail(ctx, PNS_EINVAL, "NULL model, vectors or parameters, or n_slabs < 0");
  if (!ctx->ws) return fail(ctx, PNS_EWORKSPACE, "no workspace bound");
  const Grid& g = ctx->lev[0].g;
  hipStream_t s = ctx->stream;
  pns_solve_info tot{};
  for (int k = 0; k < n_slabs; ++k) {
    // initial guess of the slab: the left trace at both Radau nodes, zero pressure
    PNS_HIP(ctx, launch_fill<double>(g.nst, 0.0, U, s));
    PNS_HIP(ctx, launch_copy<double>(g.nv, v, U, s));
    PNS_HIP(ctx, launch_copy<double>(g.nv, v, U + g.ns, s));
    pns_solve_info si{};
    const int rc = pns_solve(ctx, md, v, U, prm, work, work_bytes, &si);
    tot.newton_iterations += si.newton_iterations;
    tot.krylov_iterations += si.krylov_iterations;
    tot.smoother_setups += si.smoother_setups;
    tot.backtracks += si.backtracks;
    if (k == 0) tot.residual_initial = si.residual_initial;
    tot.residual_final = si.residual_final;
    if (info) *info = tot;
    if (rc != PNS_OK) return rc;
    // the right Radau rule ends at the slab's end: its second node's velocity
    // is the left trace of the next slab
    PNS_HIP(ctx, launch_copy<double>(g.nv, U + g.ns, v, s));
  }
  PNS_HIP(ctx, hipStreamSynchronize(s));
  if (info) *info = tot;
  return PNS_OK;
}

}  // extern "C"
