// C-ABI entry points: argument checking, workspace layout, sequencing of the
// kernels of one smoothing step / V-cycle on the context stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ctx.h"
#include "hex3.h"

using namespace pns;

namespace pns {
hipError_t launch_pin(int64_t n, double* A, const int64_t* pin, int npin, hipStream_t s);
hipError_t launch_form_fine_st(const Grid& g, double tau, const double* Es0, const double* Es1,
                               double* E, hipStream_t s);
}  // namespace pns

namespace {

int fail(pns_ctx* c, int code, const std::string& msg) {
  return fail_msg(c ? &c->err : nullptr, code, msg);
}

// Lay out (bind == false: only measure) every buffer of the context.
size_t layout(pns_ctx* c, bool bind) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + kAlign - 1) / kAlign * kAlign;
    char* p = bind ? c->ws + off : nullptr;
    off += bytes;
    return p;
  };
  const Grid& g0 = c->lev[0].g;
  const size_t es = c->es;
  if (c->prec == PNS_BF16) {  // hexahedral action only: state in BF16, slots in FP32
    c->uk = take(2 * g0.nv * 2);
    c->uk64 = (double*)take(2 * g0.nv * 8);
    c->E3 = take(g0.nc * 170 * 4);
    return (off + kAlign - 1) / kAlign * kAlign;
  }
  c->uk = take(2 * g0.nv * es);
  c->uk64 = (double*)take(2 * g0.nv * 8);
  if (c->dim == 3) {  // action, smoother of every level, dense coarsest inverse
    constexpr int64_t kE = 170 * 170;
    c->E3 = take(g0.nc * 170 * es);
    c->r3u = (double*)take(2 * g0.nv * 8);
    c->r3b = (double*)take(g0.nst * 8);
    c->r3slot = (double*)take(g0.nc * 170 * 8);
    c->ltab = (double*)take(lift3_table_doubles(c->g3) * 8);
    c->ltab_r = (double*)take(lift3_table_doubles(c->g3) * 8);
    if (c->nlev >= 2) {  // right-hand side and correction of graph-replayed V-cycles
      c->gr = take(g0.nst * es);
      c->gd = take(g0.nst * es);
    }
    // Level-0 smoother storage follows the patch kind current at sizing time
    // (it dominates the footprint): the surrogate's midpoint cell matrices
    // share the buffer of the Radau-node-1 matrices (they are consumed before
    // those are formed), the Radau-node-2 matrices exist only for exact
    // patches or for the Galerkin product of a second level.
    const bool exact = c->patch_kind == PNS_PATCH_EXACT;
    c->urep = (double*)take(g0.nv * 8);
    c->status = (int*)take(sizeof(int) * 4);
    c->Es0 = (double*)take(g0.nc * 85 * 85 * 8);
    c->Esr = c->Es0;
    c->Es1 = (exact || c->nlev >= 2) ? (double*)take(g0.nc * 85 * 85 * 8) : nullptr;
    for (int l = 0; l < c->nlev; ++l) {
      Level& L = c->lev[l];
      const bool coarsest = l == c->nlev - 1;
      L.res = take(L.g.nst * es);
      if (l == 0) {
        // real 170 x 170 exact inverses or complex 85 x 85 time-diagonal ones
        L.inv = take(L.g.nc * (exact ? kE : 2 * 85 * 85) * es);
        continue;
      }
      L.E64 = (double*)take(L.g.nc * kE * 8);
      L.E = take(L.g.nc * kE * es);
      L.r = take(L.g.nst * es);
      L.d = take(L.g.nst * es);
      if (!coarsest) L.inv = take(L.g.nc * kE * es);
    }
    if (c->has_coarse) {
      const int64_t n = c->lev.back().g.nst;
      c->Adense = (double*)take((size_t)n * n * 8);
      if (es == 4) c->Adense32 = (float*)take((size_t)n * n * 4);
      c->gjwork = (double*)take((size_t)coarse_invert_work_doubles(n) * 8);
      c->gjpiv = (int*)take((size_t)n * sizeof(int));
    }
    return (off + kAlign - 1) / kAlign * kAlign;
  }
  c->urep = (double*)take(g0.nv * 8);
  c->ltab = (double*)take(lift_table_doubles(g0) * 8);
  c->ltab_r = (double*)take(lift_table_doubles(g0) * 8);
  c->Es0 = (double*)take(g0.nc * kNs * kNs * 8);
  c->Es1 = (double*)take(g0.nc * kNs * kNs * 8);
  c->Esr = (double*)take(g0.nc * kNs * kNs * 8);
  c->masks = (uint16_t*)take(g0.nc * sizeof(uint16_t));
  c->tcache = take(g0.nc * 18 * 6 * es);
  c->edge2 = (double*)take(cell_apply_edge_doubles(g0) * 8);
  c->cipG = (double*)take(cip_face_doubles(g0) * 8);
  c->Sr = (double*)take(cip_face_count(g0) * 9 * 8);
  c->gr = take(g0.nst * es);
  c->gd = take(g0.nst * es);
  c->status = (int*)take(sizeof(int) * 4);
  // 42 results per cell of the largest coarse level
  if (c->nlev >= 2) c->slot2 = take(c->lev[1].g.nc * kNst * es);
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    const bool coarsest = (l == c->nlev - 1);
    // level 0 holds either the complex 21x21 or the real 42x42 inverses
    L.inv = take(L.g.nc * kNst * kNst * es);
    L.res = take(L.g.nst * es);
    L.S = (double*)take(cip_face_count(L.g) * 18 * 8);
    if (l >= 1 || coarsest) L.E64 = (double*)take(L.g.nc * kNst * kNst * 8);
    if (l >= 1) L.E = take(L.g.nc * kNst * kNst * es);
    if (l >= 1) {
      L.r = take(L.g.nst * es);
      L.d = take(L.g.nst * es);
    }
    if (coarsest && c->has_coarse) {
      const int64_t n = L.g.nst;
      c->Adense = (double*)take((size_t)n * n * 8);
      if (es == 4) c->Adense32 = (float*)take((size_t)n * n * 4);
      c->gjwork = (double*)take((size_t)coarse_invert_work_doubles(n) * 8);
      c->gjpiv = (int*)take((size_t)n * sizeof(int));
    }
  }
  return (off + kAlign - 1) / kAlign * kAlign;
}

bool check_ctx(pns_ctx* c, bool need_state, bool need_smoother) {
  if (!c) return false;
  if (!c->ws) {
    fail(c, PNS_EWORKSPACE, "no workspace bound");
    return false;
  }
  if (need_state && !c->has_state) {
    fail(c, PNS_ESTATE, "pns_set_state has not been called");
    return false;
  }
  if (need_smoother && !c->has_smoother) {
    fail(c, PNS_ESTATE, "pns_vanka_setup has not been called");
    return false;
  }
  return true;
}

int ctx_code(pns_ctx* c, bool need_state, bool need_smoother) {
  if (!c) return PNS_EINVAL;
  if (!c->ws) return PNS_EWORKSPACE;
  if (need_state && !c->has_state) return PNS_ESTATE;
  if (need_smoother && !c->has_smoother) return PNS_ESTATE;
  return PNS_OK;
}

template <typename T>
const T* tangent_cache(pns_ctx* c) {
  return c->apply_mode == PNS_APPLY_CACHED ? (const T*)c->tcache : nullptr;
}

// Buffers of one smoothing call that are neither inputs nor outputs: the
// defect r - A_l d, the tile-edge partial sums of the 2D level-0 action and the
// per-cell result slots of the 3D actions.  By default the context's own (in
// the bound workspace); pns_vanka_smooth_static points them into the static
// device array below.
struct SmoothScratch {
  void* res;
  double* edge;
  void* slot;
  double* cip;
};

// The coarse 2D levels sum their patch results through per-patch slots and a
// node gather (two launches a step); level 0 keeps the colour launches.
template <typename T>
T* coarse_slot(const pns_ctx* c, int l, const SmoothScratch* sc) {
  if (c->dim == 3 || l == 0) return nullptr;
  return (T*)(sc ? sc->slot : c->slot2);
}

template <typename T>
hipError_t defect(pns_ctx* c, int l, const T* b, const T* x, T* y,
                  const SmoothScratch* sc = nullptr) {
  Level& L = c->lev[l];
  double* edge = sc ? sc->edge : c->edge2;
  T* slot = (T*)(sc ? sc->slot : c->E3);
  if (c->dim == 3 && l == 0)
    return launch_cell_apply3d<T>(c->g3, c->model, c->disc.tau, (const T*)c->uk, x, b, y,
                                  slot, 1, c->stream);
  if (c->dim == 3)
    return launch_ebe_apply3d<T>(L.g3, (const T*)L.E, x, b, y, slot, c->stream);
  if (l == 0) {
    hipError_t e = launch_cell_apply<T>(L.g, c->model, c->disc.tau, (const T*)c->uk,
                                        tangent_cache<T>(c), x, b, y, edge, 1, c->stream);
    if (e != hipSuccess || !(c->model.gamma_cip > 0.0)) return e;
    return launch_cip<T>(L.g, c->model, c->disc.tau, (const T*)c->uk, L.g.nv, x, y, -1.0,
                         sc ? sc->cip : c->cipG, c->stream);
  }
  hipError_t e = launch_ebe_apply<T>(L.g, (const T*)L.E, x, b, y, 1, c->sweep_var[l],
                                     coarse_slot<T>(c, l, sc), c->stream);
  if (e != hipSuccess || !(c->model.gamma_cip > 0.0)) return e;
  return launch_cip_level<T>(L.g, L.S, x, y, -1.0, sc ? sc->cip : c->cipG, c->stream);
}

template <typename T>
hipError_t apply_level(pns_ctx* c, int l, const T* x, T* y) {
  Level& L = c->lev[l];
  if (c->dim == 3 && l == 0)
    return launch_cell_apply3d<T>(c->g3, c->model, c->disc.tau, (const T*)c->uk, x, x, y,
                                  (T*)c->E3, 0, c->stream);
  if (c->dim == 3)
    return launch_ebe_apply3d<T>(L.g3, (const T*)L.E, x, (const T*)nullptr, y, (T*)c->E3,
                                 c->stream);
  if (l == 0) {
    hipError_t e = launch_cell_apply<T>(L.g, c->model, c->disc.tau, (const T*)c->uk,
                                        tangent_cache<T>(c), x, x, y, c->edge2, 0, c->stream);
    if (e != hipSuccess || !(c->model.gamma_cip > 0.0)) return e;
    return launch_cip<T>(L.g, c->model, c->disc.tau, (const T*)c->uk, L.g.nv, x, y, 1.0, c->cipG,
                         c->stream);
  }
  hipError_t e = launch_ebe_apply<T>(L.g, (const T*)L.E, x, x, y, 0, c->sweep_var[l],
                                     coarse_slot<T>(c, l, nullptr), c->stream);
  if (e != hipSuccess || !(c->model.gamma_cip > 0.0)) return e;
  return launch_cip_level<T>(L.g, L.S, x, y, 1.0, c->cipG, c->stream);
}

hipError_t build_tangent_cache(pns_ctx* c) {
  const Grid& g0 = c->lev[0].g;
  if (c->es == 8)
    return launch_tangent_cache<double>(g0, c->model, c->disc.tau, c->uk64, (double*)c->tcache,
                                        c->stream);
  return launch_tangent_cache<float>(g0, c->model, c->disc.tau, c->uk64, (float*)c->tcache,
                                     c->stream);
}

// level l holds complex 21x21 time-diagonal patch inverses (else real 42x42)
bool complex_patches(const pns_ctx* c, int l) {
  return l == 0 && c->patch_kind == PNS_PATCH_SURROGATE;
}

template <typename T>
hipError_t smooth(pns_ctx* c, int l, int nsweeps, double omega, const T* r, T* d, bool d_is_zero,
                  const SmoothScratch* sc = nullptr) {
  Level& L = c->lev[l];
  T* resbuf = (T*)(sc ? sc->res : L.res);
  for (int s = 0; s < nsweeps; ++s) {
    const T* res = r;
    if (!(s == 0 && d_is_zero)) {
      hipError_t e = defect<T>(c, l, r, d, resbuf, sc);
      if (e != hipSuccess) return e;
      res = (const T*)resbuf;
    }
    if (c->dim == 3) {
      hipError_t e = complex_patches(c, l)
                         ? launch_patch_sweep3<T>(L.g3, (const T*)L.inv, res, d, omega, c->stream)
                         : launch_patch_sweep3r<T>(L.g3, (const T*)L.inv, res, d, omega, c->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    hipError_t e = complex_patches(c, l)
                       ? launch_patch_sweep_c<T>(L.g, (const T*)L.inv, res, d, omega,
                                                 c->sweep_var[l], c->stream)
                       : launch_patch_sweep<T>(L.g, (const T*)L.inv, res, d, omega,
                                               c->sweep_var[l], coarse_slot<T>(c, l, sc),
                                               c->stream, s == 0 && d_is_zero);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t vcycle_level(pns_ctx* c, int l, int nu1, int nu2, double omega, const T* r, T* d) {
  Level& L = c->lev[l];
  hipError_t e;
  if (l == c->nlev - 1) {
    const int npin = 2;
    // the inverse in the context's precision: FP32 contexts read its FP32 copy
    const T* A = sizeof(T) == 8 ? (const T*)(const void*)c->Adense
                                : (const T*)(const void*)c->Adense32;
    return launch_dense_gemv<T>(L.g.nst, A, r, d, c->pin, npin, c->stream);
  }
  // d starts at zero; on a coarse level the first sweep's gather writes all of
  // it, so only level 0 (colour launches adding into d) needs the fill
  const bool first_sweep_sets_d = nu1 > 0 && coarse_slot<T>(c, l, nullptr) && l > 0;
  if (!first_sweep_sets_d && (e = launch_fill<T>(L.g.nst, (T)0, d, c->stream)) != hipSuccess)
    return e;
  if ((e = smooth<T>(c, l, nu1, omega, r, d, true)) != hipSuccess) return e;
  const T* res = r;
  if (nu1 > 0) {
    if ((e = defect<T>(c, l, r, d, (T*)L.res)) != hipSuccess) return e;
    res = (const T*)L.res;
  }
  Level& C = c->lev[l + 1];
  e = c->dim == 3 ? launch_restrict3<T>(L.g3, C.g3, res, (T*)C.r, c->stream)
                  : launch_restrict<T>(L.g, C.g, res, (T*)C.r, c->stream);
  if (e != hipSuccess) return e;
  if ((e = vcycle_level<T>(c, l + 1, nu1, nu2, omega, (const T*)C.r, (T*)C.d)) != hipSuccess)
    return e;
  e = c->dim == 3 ? launch_prolong_add3<T>(L.g3, C.g3, (const T*)C.d, d, c->stream)
                  : launch_prolong_add<T>(L.g, C.g, (const T*)C.d, d, c->stream);
  if (e != hipSuccess) return e;
  return smooth<T>(c, l, nu2, omega, r, d, false);
}

// Autotuner of the patch sweeps: on every level, each variant of that level's
// patch form runs one additive step (level 0: 4 colour launches; coarse levels:
// slot launch + gather) on zero vectors, once to warm up and three times timed
// with events on the context stream; the fastest is kept.  The variants compute
// the same step, so the choice changes the time and the summation order within
// a patch only.  The choice depends on the level's shape, not on its data: it
// is made once per (cells in x, cells in y, patch form, precision, colour or
// slot form) in a process and reused by later setups and contexts (smoother
// refreshes inside a solve, served requests).
struct TunedShapes {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int, int>, int> best;
};
TunedShapes& tuned_shapes() {
  static TunedShapes t;
  return t;
}

template <typename T>
int autotune_sweeps(pns_ctx* c) {
  {
    // every level already tuned in this process: reuse the choices
    TunedShapes& ts = tuned_shapes();
    std::lock_guard<std::mutex> lk(ts.mu);
    bool all = true;
    for (int l = 0; l < c->nlev && all; ++l) {
      const Grid& g = c->lev[l].g;
      auto it = ts.best.find({g.nx, g.ny, complex_patches(c, l) ? 1 : 0, (int)c->es, l >= 1 ? 1 : 0});
      if (it == ts.best.end()) all = false;
    }
    if (all) {
      for (int l = 0; l < c->nlev; ++l) {
        const Grid& g = c->lev[l].g;
        c->sweep_var[l] = ts.best[{g.nx, g.ny, complex_patches(c, l) ? 1 : 0, (int)c->es, l >= 1 ? 1 : 0}];
      }
      return PNS_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PNS_HIP(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, PNS_EHIP, "hipEventCreate failed");
  }
  int rc = PNS_OK;
  for (int l = 0; l < c->nlev && rc == PNS_OK; ++l) {
    Level& L = c->lev[l];
    const bool cx = complex_patches(c, l);
    const int nv = sweep_variant_count(cx);
    T* res = (T*)L.res;
    T* d = l == 0 ? (T*)c->gd : (T*)L.d;
    float best = 0.0f;
    if (launch_fill<T>(L.g.nst, (T)0, res, c->stream) != hipSuccess ||
        launch_fill<T>(L.g.nst, (T)0, d, c->stream) != hipSuccess) {
      rc = fail(c, PNS_EHIP, "fill failed in the sweep autotuner");
      break;
    }
    for (int v = 0; v < nv && rc == PNS_OK; ++v) {
      auto run = [&]() {
        return cx ? launch_patch_sweep_c<T>(L.g, (const T*)L.inv, res, d, 1.0, v, c->stream)
                  : launch_patch_sweep<T>(L.g, (const T*)L.inv, res, d, 1.0, v,
                                          coarse_slot<T>(c, l, nullptr), c->stream);
      };
      float ms = 0.0f;
      if (run() != hipSuccess || hipEventRecord(e0, c->stream) != hipSuccess ||
          run() != hipSuccess || run() != hipSuccess || run() != hipSuccess ||
          hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = fail(c, PNS_EHIP, "sweep autotuner launch failed");
        break;
      }
      ms /= 3.0f;
      c->sweep_ms[l][v] = ms;
      if (v == 0 || ms < best) {
        best = ms;
        c->sweep_var[l] = v;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == PNS_OK) {
    TunedShapes& ts = tuned_shapes();
    std::lock_guard<std::mutex> lk(ts.mu);
    for (int l = 0; l < c->nlev; ++l) {
      const Grid& g = c->lev[l].g;
      ts.best[{g.nx, g.ny, complex_patches(c, l) ? 1 : 0, (int)c->es, l >= 1 ? 1 : 0}] = c->sweep_var[l];
    }
  }
  return rc;
}

// 3D: surrogate patches of the finest level only (time-diagonal form)
// 3D: level 0 surrogate patches in time-diagonal form; coarse levels: Galerkin
// element matrices (from the exact level-0 element matrices of both Radau
// nodes), exact real patches (all but the coarsest), dense coarsest inverse
template <typename T>
int vanka_setup3d(pns_ctx* c) {
  hipStream_t s = c->stream;
  const Grid3& g0 = c->lev[0].g3;
  PNS_HIP(c, hipMemsetAsync(c->status, 0, sizeof(int), s));
  const bool exact = c->patch_kind == PNS_PATCH_EXACT;
  if (!exact) {
    // level 0: surrogate patches, all state-dependent coefficients at t_rep;
    // Esr is the buffer of Es0, so this comes first (stream order)
    PNS_HIP(c, launch_element_matrices3d(g0, c->model, c->urep, 2, c->Esr, s));
    PNS_HIP(c, launch_patches3d<T>(g0, c->disc.tau, c->Esr, (T*)c->lev[0].inv, c->status, s));
  }
  if (c->nlev >= 2 || exact) {
    PNS_HIP(c, launch_element_matrices3d(g0, c->model, c->uk64, 0, c->Es0, s));
    PNS_HIP(c, launch_element_matrices3d(g0, c->model, c->uk64 + g0.nv, 1, c->Es1, s));
  }
  if (exact) {
    // level 0: exact patches, each Radau node with its own spatial matrices
    PNS_HIP(c, launch_exact_fine_patches3d<T>(g0, c->disc.tau, c->Es0, c->Es1,
                                              (T*)c->lev[0].inv, c->status, s));
  }
  for (int l = 1; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    if (l == 1)
      PNS_HIP(c, launch_galerkin3d_from_fine(L.g3, g0, c->disc.tau, c->Es0, c->Es1, L.E64, s));
    else
      PNS_HIP(c, launch_galerkin3d(L.g3, c->lev[l - 1].g3, c->lev[l - 1].E64, L.E64, s));
    PNS_HIP(c, launch_transpose_convert3<T>(L.g.nc, L.E64, (T*)L.E, s));
    if (l < c->nlev - 1)
      PNS_HIP(c, launch_level_patches3d<T>(L.g3, L.E64, (T*)L.inv, c->status, s));
  }
  int st = 0;
  if (c->has_coarse) {
    Level& Lc = c->lev[c->nlev - 1];
    const int64_t n = Lc.g.nst;
    PNS_HIP(c, hipMemsetAsync(c->Adense, 0, (size_t)n * n * 8, s));
    PNS_HIP(c, launch_coarse_assemble3(Lc.g3, Lc.E64, c->Adense, s));
    c->pin[0] = Lc.g.nv;
    c->pin[1] = Lc.g.ns + Lc.g.nv;
    PNS_HIP(c, hipMemcpyAsync(c->gjwork, c->pin, sizeof(c->pin), hipMemcpyHostToDevice, s));
    PNS_HIP(c, hipStreamSynchronize(s));
    PNS_HIP(c, launch_pin(n, c->Adense, (const int64_t*)c->gjwork, 2, s));
    PNS_HIP(c, coarse_invert(n, c->Adense, c->gjwork, c->gjpiv, c->status, s));
    if (c->Adense32) PNS_HIP(c, launch_convert<float>(n * n, c->Adense, c->Adense32, s));
  }
  PNS_HIP(c, hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, s));
  PNS_HIP(c, hipStreamSynchronize(s));
  if (st & 1) return fail(c, PNS_ESINGULAR, "a patch matrix has a zero pivot");
  if (st & 2) return fail(c, PNS_ESINGULAR, "the coarsest matrix has a zero pivot");
  c->has_smoother = true;
  return PNS_OK;
}

template <typename T>
int vanka_setup_impl(pns_ctx* c, const uint16_t* masks) {
  hipStream_t s = c->stream;
  const Level& L0 = c->lev[0];
  PNS_HIP(c, hipMemsetAsync(c->status, 0, sizeof(int), s));
  if (masks) {
    PNS_HIP(c, hipMemcpyAsync(c->masks, masks, L0.g.nc * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    PNS_HIP(c, hipStreamSynchronize(s));
  }
  const double* u0 = c->uk64;
  const double* u1 = c->uk64 + L0.g.nv;
  // with Dirichlet data, the Nitsche coefficients of each Radau node's lifting,
  // and at t_rep for the surrogate patches (time slots 0, 1, 2 of the table)
  PNS_HIP(c, launch_element_matrices(L0.g, c->model, u0, 0, c->Es0, s));
  PNS_HIP(c, launch_element_matrices(L0.g, c->model, u1, 1, c->Es1, s));
  if (c->patch_kind == PNS_PATCH_SURROGATE)  // the midpoint matrices feed only those patches
    PNS_HIP(c, launch_element_matrices(L0.g, c->model, c->urep, 2, c->Esr, s));
  // CIP face matrices: at each Radau node's velocity (level-0 operator, with
  // tau w_mu) and at t_rep (time-diagonal patches, unscaled)
  const bool cip = c->model.gamma_cip > 0.0;
  if (cip) {
    PNS_HIP(c, launch_cip_face_matrices(L0.g, c->model, u0, L0.g.nv, 2, c->disc.tau * kWt[0],
                                        c->disc.tau * kWt[1], L0.S, s));
    PNS_HIP(c, launch_cip_face_matrices(L0.g, c->model, c->urep, 0, 1, 1.0, 1.0, c->Sr, s));
  }
  if (c->patch_kind == PNS_PATCH_SURROGATE) {
    // level 0: surrogate patches, all state-dependent coefficients at t_rep
    PNS_HIP(c, launch_fine_patches<T>(L0.g, c->disc.tau, c->Esr, cip ? c->Sr : nullptr,
                                      masks ? c->masks : nullptr, (T*)L0.inv, c->status, s));
  } else {
    // level 0: exact patches, each Radau node with its own spatial matrices
    PNS_HIP(c, launch_exact_fine_patches<T>(L0.g, c->disc.tau, c->Es0, c->Es1,
                                            cip ? L0.S : nullptr, masks ? c->masks : nullptr,
                                            (T*)L0.inv, c->status, s));
  }
  // coarse levels: Galerkin element matrices and CIP face matrices, exact patches
  for (int l = 1; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    if (l == 1)
      PNS_HIP(c, launch_galerkin_from_fine(L.g, c->disc.tau, c->Es0, c->Es1, L.E64, s));
    else
      PNS_HIP(c, launch_galerkin(L.g, c->lev[l - 1].E64, L.E64, s));
    if (cip) PNS_HIP(c, launch_cip_restrict(L.g, c->lev[l - 1].g, c->lev[l - 1].S, L.S, s));
    PNS_HIP(c, launch_transpose_convert<T>(L.g, L.E64, (T*)L.E, s));
    PNS_HIP(c, launch_level_patches<T>(L.g, L.E64, cip ? L.S : nullptr, (T*)L.inv, c->status,
                                       s));
  }
  // coarsest level: dense operator, pinned, inverted
  Level& Lc = c->lev[c->nlev - 1];
  if (c->nlev == 1) {
    PNS_HIP(c, launch_form_fine_st(Lc.g, c->disc.tau, c->Es0, c->Es1, Lc.E64, s));
  }
  int st = 0;
  if (!c->has_coarse) {
    PNS_HIP(c, hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, s));
    PNS_HIP(c, hipStreamSynchronize(s));
    if (st & 1) return fail(c, PNS_ESINGULAR, "a patch matrix has a zero pivot");
    const int rc = autotune_sweeps<T>(c);
    if (rc != PNS_OK) return rc;
    c->has_smoother = true;
    return PNS_OK;
  }
  const int64_t n = Lc.g.nst;
  PNS_HIP(c, hipMemsetAsync(c->Adense, 0, (size_t)n * n * 8, s));
  PNS_HIP(c, launch_coarse_assemble(Lc.g, Lc.E64, c->Adense, s));
  if (cip) PNS_HIP(c, launch_cip_dense(Lc.g, Lc.S, c->Adense, s));
  c->pin[0] = Lc.g.nv;
  c->pin[1] = Lc.g.ns + Lc.g.nv;
  // pin indices must be in device memory for the pin kernel
  PNS_HIP(c, hipMemcpyAsync(c->gjwork, c->pin, sizeof(c->pin), hipMemcpyHostToDevice, s));
  PNS_HIP(c, hipStreamSynchronize(s));
  PNS_HIP(c, launch_pin(n, c->Adense, (const int64_t*)c->gjwork, 2, s));
  PNS_HIP(c, coarse_invert(n, c->Adense, c->gjwork, c->gjpiv, c->status, s));
  if (c->Adense32) PNS_HIP(c, launch_convert<float>(n * n, c->Adense, c->Adense32, s));
  PNS_HIP(c, hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, s));
  PNS_HIP(c, hipStreamSynchronize(s));
  if (st & 1) return fail(c, PNS_ESINGULAR, "a patch matrix has a zero pivot");
  if (st & 2) return fail(c, PNS_ESINGULAR, "the coarsest matrix has a zero pivot");
  const int rc = autotune_sweeps<T>(c);
  if (rc != PNS_OK) return rc;
  c->has_smoother = true;
  return PNS_OK;
}

// One V-cycle d = V(r) replayed from a graph captured on the library's own
// stream (the context stream may be the legacy default stream, which cannot
// capture): r is copied into c->gr, the graph runs vcycle_level on
// (c->gr, c->gd), c->gd is copied out.  Captured on first use and again when
// nu1, nu2 or omega change; dropped by everything that changes the data the
// kernels read or their arguments.
template <typename T>
int vcycle_graph(pns_ctx* c, int nu1, int nu2, double omega, const T* r, T* d) {
  const int64_t n = c->lev[0].g.nst;
  if (c->vgraph && (c->g_nu1 != nu1 || c->g_nu2 != nu2 || c->g_omega != omega)) c->drop_graph();
  if (!c->vgraph) {
    if (!c->cap_stream)
      PNS_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    PNS_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    const hipError_t e = vcycle_level<T>(c, 0, nu1, nu2, omega, (const T*)c->gr, (T*)c->gd);
    c->stream = saved;
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
    PNS_HIP(c, e);
    PNS_HIP(c, e2);
    const hipError_t e3 = hipGraphInstantiate(&c->vgraph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) c->vgraph = nullptr;
    PNS_HIP(c, e3);
    c->g_nu1 = nu1;
    c->g_nu2 = nu2;
    c->g_omega = omega;
  }
  PNS_HIP(c, launch_copy<T>(n, r, (T*)c->gr, c->stream));
  PNS_HIP(c, hipGraphLaunch(c->vgraph, c->stream));
  PNS_HIP(c, launch_copy<T>(n, (const T*)c->gd, d, c->stream));
  return PNS_OK;
}

// 3D context: hexahedra (action, smoother, V-cycle over n_levels nested meshes)
int create3d(const pns_mesh* mesh, const pns_discretization* disc, int n_levels, int precision,
             void* stream, pns_ctx** out) {
  if (disc->k_space != 2 || disc->k_time != 1) return PNS_EUNSUPPORTED;
  if (precision != PNS_FP64 && precision != PNS_FP32 && precision != PNS_BF16) return PNS_EINVAL;
  if (precision == PNS_BF16 && n_levels != 1) return PNS_EUNSUPPORTED;  // action only
  if (!(disc->tau > 0.0) || n_levels < 1 || n_levels > 10) return PNS_EINVAL;
  const int nx = mesh->n_cells[0], ny = mesh->n_cells[1], nz = mesh->n_cells[2];
  if (nx < 1 || ny < 1 || nz < 1) return PNS_EINVAL;
  const int f = 1 << (n_levels - 1);
  if (nx % f || ny % f || nz % f) return PNS_EINVAL;
  double len[3];
  for (int k = 0; k < 3; ++k) {
    len[k] = mesh->hi[k] - mesh->lo[k];
    if (!(len[k] > 0.0)) return PNS_EINVAL;
  }
  // one workgroup per cell in a 1D grid
  if ((int64_t)nx * ny * nz > ((int64_t)1 << 31) - 1) return PNS_EUNSUPPORTED;
  pns_ctx* c = new pns_ctx();
  c->dim = 3;
  c->mesh = *mesh;
  c->disc = *disc;
  c->prec = precision;
  c->es = precision == PNS_FP64 ? 8 : 4;  // BF16: y, b and the slots in FP32
  c->nlev = n_levels;
  c->stream = (hipStream_t)stream;
  c->g3 = make_grid3(nx, ny, nz, len[0], len[1], len[2]);
  for (int l = 0; l < n_levels; ++l) {
    Level L{};
    L.g3 = make_grid3(nx >> l, ny >> l, nz >> l, len[0], len[1], len[2]);
    L.g.nx = L.g3.nx;
    L.g.ny = L.g3.ny;
    L.g.hx = L.g3.hx;
    L.g.hy = L.g3.hy;
    L.g.ihx = L.g3.ihx;
    L.g.ihy = L.g3.ihy;
    L.g.nn = L.g3.nn;
    L.g.nc = L.g3.nc;
    L.g.nv = L.g3.nv;
    L.g.ns = L.g3.ns;
    L.g.nst = L.g3.nst;
    c->lev.push_back(L);
  }
  // dense coarsest inverse (and so the V-cycle) with at least two levels
  c->has_coarse = n_levels >= 2 && c->lev.back().g.nst <= kMaxCoarse;
  *out = c;
  return PNS_OK;
}

// Scratch of pns_vanka_smooth_static: one array per GPU the library runs on,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device array: its device address is taken once per device
// with hipGetSymbolAddress and only that address is passed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the device of `stream` (looked up with that
// device current, then kept).
hipError_t static_scratch(hipStream_t stream, void** out) {
  int dev = -1;
  hipError_t e = hipStreamGetDevice(stream, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    int cur = -1;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// Bytes of static scratch one smoothing call on `level` uses: the defect, the
// 2D level-0 tile-edge partial sums, the 2D CIP per-face values, the 3D
// per-cell result slots.
size_t static_scratch_need(const pns_ctx* c, int level) {
  auto up = [](size_t b) { return (b + kAlign - 1) / kAlign * kAlign; };
  const Level& L = c->lev[level];
  size_t need = up(L.g.nst * c->es);
  if (c->dim == 3)
    need += up(L.g.nc * 170 * c->es);
  else
    need += (level == 0 ? up(cell_apply_edge_doubles(L.g) * 8) : up(L.g.nc * kNst * c->es)) +
            (c->model.gamma_cip > 0.0 ? up(cip_face_doubles(L.g) * 8) : 0);
  return need;
}

}  // namespace

int pns::make_model(const pns_model* md, Model* m, std::string* err) {
  if (!(md->p > 1.0 && md->p <= 2.0)) return fail_msg(err, PNS_EINVAL, "p must lie in (1, 2]");
  if (!(md->delta > 0.0)) return fail_msg(err, PNS_EINVAL, "delta must be > 0");
  if (!(md->nu > 0.0) || !(md->nu_inf >= 0.0))
    return fail_msg(err, PNS_EINVAL, "need nu > 0, nu_inf >= 0");
  if (!(md->gamma1 >= 0.0) || !(md->gamma2 >= 0.0))
    return fail_msg(err, PNS_EINVAL, "negative penalty");
  if (!(md->sigma_max >= 0.0)) return fail_msg(err, PNS_EINVAL, "sigma_max must be >= 0");
  if (md->lin < 0 || md->lin > 2) return fail_msg(err, PNS_EINVAL, "unknown linearisation kind");
  if (md->nitsche_q_sign != 1 && md->nitsche_q_sign != -1)
    return fail_msg(err, PNS_EINVAL, "nitsche_q_sign must be +1 or -1");
  if (!(md->gamma_cip >= 0.0)) return fail_msg(err, PNS_EINVAL, "gamma_cip must be >= 0");
  m->p = md->p;
  m->delta2 = md->delta * md->delta;
  m->nu = md->nu;
  m->nu_inf = md->nu_inf;
  m->expo = 0.5 * (md->p - 2.0);
  m->sigma_max = md->sigma_max;
  m->etaD = md->nu_inf + md->nu * std::pow(md->delta, md->p - 2.0);  // eta(D g_D), g_D = 0
  m->gamma1 = md->gamma1;
  m->gamma2 = md->gamma2;
  m->qsign = (double)md->nitsche_q_sign;
  m->lin = md->lin;
  m->convection = md->convection ? 1 : 0;
  m->gamma_cip = md->gamma_cip;
  m->lift = nullptr;  // the context's lifting and summation mode are attached by the caller
  m->ordered = 0;
  return PNS_OK;
}

extern "C" {

int pns_ctx_create(const pns_mesh* mesh, const pns_discretization* disc, int n_levels,
                   int precision, void* stream, pns_ctx** out) {
  if (!out) return PNS_EINVAL;
  *out = nullptr;
  if (!mesh || !disc) return PNS_EINVAL;
  if (mesh->dim == 3) return create3d(mesh, disc, n_levels, precision, stream, out);
  if (mesh->dim != 2 || disc->k_space != 2 || disc->k_time != 1) return PNS_EUNSUPPORTED;
  if (precision != PNS_FP64 && precision != PNS_FP32) return PNS_EINVAL;
  if (!(disc->tau > 0.0) || n_levels < 1 || n_levels > 12) return PNS_EINVAL;
  const int nx = mesh->n_cells[0], ny = mesh->n_cells[1];
  if (nx < 1 || ny < 1) return PNS_EINVAL;
  const double lx = mesh->hi[0] - mesh->lo[0], ly = mesh->hi[1] - mesh->lo[1];
  if (!(lx > 0.0) || !(ly > 0.0)) return PNS_EINVAL;
  const int f = 1 << (n_levels - 1);
  if (nx % f || ny % f || nx / f < 1 || ny / f < 1) return PNS_EINVAL;
  // tile grid of the level-0 kernel and int cell indices
  if ((int64_t)nx * ny > (int64_t)1 << 30) return PNS_EUNSUPPORTED;
  pns_ctx* c = new pns_ctx();
  c->mesh = *mesh;
  c->disc = *disc;
  c->prec = precision;
  c->es = precision == PNS_FP64 ? 8 : 4;
  c->nlev = n_levels;
  c->stream = (hipStream_t)stream;
  for (int l = 0; l < n_levels; ++l) {
    Level L;
    L.g = make_grid(nx >> l, ny >> l, lx, ly);
    c->lev.push_back(L);
  }
  c->has_coarse = c->lev.back().g.nst <= kMaxCoarse;
  *out = c;
  return PNS_OK;
}

void pns_ctx_destroy(pns_ctx* ctx) { delete ctx; }

int pns_sweep_variant(const pns_ctx* ctx, int level, int out[5]) {
  if (!ctx || !out || level < 0 || level >= ctx->nlev || ctx->dim == 3) return PNS_EINVAL;
  const bool cx = complex_patches(ctx, level);
  out[0] = ctx->sweep_var[level];
  out[1] = sweep_variant_count(cx);
  sweep_variant_shape(cx, out[0], out + 2);
  return PNS_OK;
}

int pns_sweep_variant_time(const pns_ctx* ctx, int level, int variant, double* ms) {
  if (!ctx || !ms || level < 0 || level >= ctx->nlev || ctx->dim == 3) return PNS_EINVAL;
  if (variant < 0 || variant >= sweep_variant_count(complex_patches(ctx, level)))
    return PNS_EINVAL;
  *ms = ctx->sweep_ms[level][variant];
  return PNS_OK;
}

int pns_set_sweep_variant(pns_ctx* ctx, int level, int variant) {
  if (!ctx) return PNS_EINVAL;
  if (level < 0 || level >= ctx->nlev || ctx->dim == 3)
    return fail(ctx, PNS_EINVAL, "bad level");
  if (variant < 0 || variant >= sweep_variant_count(complex_patches(ctx, level)))
    return fail(ctx, PNS_EINVAL, "bad sweep variant");
  ctx->sweep_var[level] = variant;
  ctx->drop_graph();
  return PNS_OK;
}

int pns_set_vcycle_graph(pns_ctx* ctx, int enable) {
  if (!ctx) return PNS_EINVAL;
  if (enable != 0 && enable != 1) return fail(ctx, PNS_EINVAL, "enable must be 0 or 1");
  if (enable && ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  ctx->graph_mode = enable == 1;
  if (!enable) ctx->drop_graph();
  return PNS_OK;
}

const char* pns_last_error(const pns_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pns_level_sizes(const pns_ctx* ctx, int level, int64_t out[4]) {
  if (!ctx || !out || level < 0 || level >= ctx->nlev) return PNS_EINVAL;
  const Grid& g = ctx->lev[level].g;
  out[0] = g.nst;
  out[1] = g.nc;
  out[2] = g.nv;
  out[3] = g.ns;
  return PNS_OK;
}

size_t pns_workspace_bytes(const pns_ctx* ctx) {
  if (!ctx) return 0;
  pns_ctx tmp = *ctx;
  // the copy measures the layout only; it does not own the graph or its stream
  tmp.vgraph = nullptr;
  tmp.cap_stream = nullptr;
  return layout(&tmp, false);
}

int pns_bind_workspace(pns_ctx* ctx, void* ws, size_t bytes) {
  if (!ctx) return PNS_EINVAL;
  if (!ws || ((uintptr_t)ws % kAlign) != 0)
    return fail(ctx, PNS_EWORKSPACE, "workspace pointer NULL or not 256-byte aligned");
  const size_t need = pns_workspace_bytes(ctx);
  if (bytes < need)
    return fail(ctx, PNS_EWORKSPACE,
                "workspace too small: need " + std::to_string(need) + " bytes");
  ctx->ws = (char*)ws;
  ctx->ws_bytes = bytes;
  ctx->drop_graph();
  layout(ctx, true);
  ctx->has_state = ctx->has_smoother = false;
  ctx->model.lift = nullptr;  // the boundary tables moved with the workspace
  return PNS_OK;
}

int pns_set_state(pns_ctx* ctx, const pns_model* md, const double* u_k) {
  if (!check_ctx(ctx, false, false)) return ctx_code(ctx, false, false);
  if (!md || !u_k) return fail(ctx, PNS_EINVAL, "NULL model or state");
  Model m;
  const int rc = make_model(md, &m, &ctx->err);
  if (rc != PNS_OK) return rc;
  if (ctx->dim == 3 && m.gamma_cip > 0.0)
    return fail(ctx, PNS_EUNSUPPORTED, "CIP stabilisation is built for quadrilaterals only");
  m.lift = nullptr;
  if (ctx->lift) {
    if (ctx->dim == 3)
      PNS_HIP(ctx, launch_lift3_table(ctx->g3, m, ctx->lift, ctx->ltab, ctx->stream));
    else
      PNS_HIP(ctx, launch_lift_table(ctx->lev[0].g, m, ctx->lift, ctx->ltab, ctx->stream));
    m.lift = ctx->ltab;
  }
  m.ordered = ctx->ordered ? 1 : 0;
  ctx->model = m;
  ctx->drop_graph();
  const Grid& g0 = ctx->lev[0].g;
  hipStream_t s = ctx->stream;
  PNS_HIP(ctx, hipMemcpyAsync(ctx->uk64, u_k, 2 * g0.nv * 8, hipMemcpyDeviceToDevice, s));
  if (ctx->prec == PNS_BF16) {
    PNS_HIP(ctx, launch_to_bf16(2 * g0.nv, ctx->uk64, (uint16_t*)ctx->uk, s));
    ctx->has_state = true;
    ctx->has_smoother = false;
    return PNS_OK;
  }
  if (ctx->es == 8)
    PNS_HIP(ctx, hipMemcpyAsync(ctx->uk, u_k, 2 * g0.nv * 8, hipMemcpyDeviceToDevice, s));
  else
    PNS_HIP(ctx, launch_convert<float>(2 * g0.nv, ctx->uk64, (float*)ctx->uk, s));
  PNS_HIP(ctx, launch_state_combine(g0.nv, ctx->uk64, ctx->uk64 + g0.nv, kXiMid[0], kXiMid[1],
                                    ctx->urep, s));
  if (ctx->dim == 2 && ctx->apply_mode == PNS_APPLY_CACHED) PNS_HIP(ctx, build_tangent_cache(ctx));
  ctx->has_state = true;
  ctx->has_smoother = false;
  return PNS_OK;
}

int pns_set_apply_mode(pns_ctx* ctx, int mode) {
  if (!ctx) return PNS_EINVAL;
  if (mode != PNS_APPLY_RECOMPUTE && mode != PNS_APPLY_CACHED)
    return fail(ctx, PNS_EINVAL, "unknown apply mode");
  if (ctx->dim == 3 && mode != PNS_APPLY_RECOMPUTE)
    return fail(ctx, PNS_EUNSUPPORTED, "3D contexts recompute the tangent");
  const bool rebuild = mode == PNS_APPLY_CACHED && ctx->apply_mode != mode && ctx->has_state;
  if (mode != ctx->apply_mode) ctx->drop_graph();
  ctx->apply_mode = mode;
  if (rebuild) PNS_HIP(ctx, build_tangent_cache(ctx));
  return PNS_OK;
}

int pns_set_patch_kind(pns_ctx* ctx, int kind) {
  if (!ctx) return PNS_EINVAL;
  if (kind != PNS_PATCH_SURROGATE && kind != PNS_PATCH_EXACT)
    return fail(ctx, PNS_EINVAL, "unknown patch kind");
  if (kind == ctx->patch_kind) return PNS_OK;
  if (ctx->dim == 3 && ctx->ws) {
    // the level-0 smoother storage depends on the kind; everything laid out
    // before it (state, action buffers) keeps its place
    const int old = ctx->patch_kind;
    ctx->patch_kind = kind;
    const size_t need = pns_workspace_bytes(ctx);  // measures on a copy
    if (need > ctx->ws_bytes) {
      ctx->patch_kind = old;
      return fail(ctx, PNS_EWORKSPACE,
                  "bound workspace too small for this patch kind: need " + std::to_string(need) +
                      " bytes (select the kind before pns_workspace_bytes)");
    }
    layout(ctx, true);
  }
  ctx->has_smoother = false;
  ctx->drop_graph();
  ctx->patch_kind = kind;
  return PNS_OK;
}

int pns_set_jacobian_precision(pns_ctx* ctx, int precision) {
  if (!ctx) return PNS_EINVAL;
  if (precision != PNS_FP64 && precision != PNS_FP32 && precision != PNS_BF16)
    return fail(ctx, PNS_EINVAL, "unknown precision");
  if (precision == PNS_BF16) {
    if (ctx->dim != 3 || ctx->prec != PNS_FP32)
      return fail(ctx, PNS_EUNSUPPORTED,
                  "a BF16 Jacobian action needs a hexahedral FP32 context");
    ctx->jac_bf16 = true;
    return PNS_OK;
  }
  if (precision != ctx->prec)
    return fail(ctx, PNS_EUNSUPPORTED, "the Jacobian action runs in the context precision or BF16");
  ctx->jac_bf16 = false;
  return PNS_OK;
}

int pns_load_vector(pns_ctx* ctx, const double* f_qp, double* F) {
  if (!ctx) return PNS_EINVAL;
  if (!f_qp || !F) return fail(ctx, PNS_EINVAL, "NULL f or F");
  if (ctx->dim == 3)
    PNS_HIP(ctx, launch_load3(ctx->g3, ctx->disc.tau, f_qp, F, ctx->stream));
  else
    PNS_HIP(ctx, launch_load2(ctx->lev[0].g, ctx->disc.tau, f_qp, F, ctx->stream));
  return PNS_OK;
}

int pns_set_load(pns_ctx* ctx, const double* F) {
  if (!ctx) return PNS_EINVAL;
  ctx->load = F;
  return PNS_OK;
}

int pns_set_reproducible(pns_ctx* ctx, int on) {
  if (!ctx) return PNS_EINVAL;
  if (on != 0 && on != 1) return fail(ctx, PNS_EINVAL, "on must be 0 or 1");
  ctx->ordered = on == 1;
  ctx->model.ordered = on;
  ctx->drop_graph();
  return PNS_OK;
}

int pns_set_dirichlet(pns_ctx* ctx, const double* ghat) {
  if (!ctx) return PNS_EINVAL;
  if (ghat && ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (ghat && !ctx->ws) return fail(ctx, PNS_EWORKSPACE, "no workspace bound");
  ctx->lift = ghat;
  ctx->model.lift = nullptr;
  if (ghat && ctx->has_state) {  // the action sees the data at once
    if (ctx->dim == 3)
      PNS_HIP(ctx, launch_lift3_table(ctx->g3, ctx->model, ghat, ctx->ltab, ctx->stream));
    else
      PNS_HIP(ctx, launch_lift_table(ctx->lev[0].g, ctx->model, ghat, ctx->ltab, ctx->stream));
    ctx->model.lift = ctx->ltab;
  }
  ctx->drop_graph();
  ctx->has_smoother = false;  // the patches and coarse operators depend on it
  return PNS_OK;
}

int pns_cell_apply(pns_ctx* ctx, const void* x, void* y) {
  if (!check_ctx(ctx, true, false)) return ctx_code(ctx, true, false);
  if (!x || !y || x == y) return fail(ctx, PNS_EINVAL, "x, y must be distinct non-NULL");
  if (ctx->prec == PNS_BF16)
    PNS_HIP(ctx, launch_cell_apply3d_bf16(ctx->g3, ctx->model, ctx->disc.tau,
                                          (const uint16_t*)ctx->uk, (const uint16_t*)x, nullptr,
                                          (float*)y, (float*)ctx->E3, 0, ctx->stream));
  else if (ctx->es == 8)
    PNS_HIP(ctx, apply_level<double>(ctx, 0, (const double*)x, (double*)y));
  else
    PNS_HIP(ctx, apply_level<float>(ctx, 0, (const float*)x, (float*)y));
  return PNS_OK;
}

int pns_cell_defect(pns_ctx* ctx, const void* b, const void* x, void* y) {
  if (!check_ctx(ctx, true, false)) return ctx_code(ctx, true, false);
  if (!b || !x || !y || x == y) return fail(ctx, PNS_EINVAL, "b, x, y non-NULL, x != y");
  if (ctx->prec == PNS_BF16)
    PNS_HIP(ctx, launch_cell_apply3d_bf16(ctx->g3, ctx->model, ctx->disc.tau,
                                          (const uint16_t*)ctx->uk, (const uint16_t*)x,
                                          (const float*)b, (float*)y, (float*)ctx->E3, 1,
                                          ctx->stream));
  else if (ctx->es == 8)
    PNS_HIP(ctx, defect<double>(ctx, 0, (const double*)b, (const double*)x, (double*)y));
  else
    PNS_HIP(ctx, defect<float>(ctx, 0, (const float*)b, (const float*)x, (float*)y));
  return PNS_OK;
}

int pns_vanka_setup(pns_ctx* ctx, const uint16_t* node_masks) {
  if (ctx && ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (!check_ctx(ctx, true, false)) return ctx_code(ctx, true, false);
  ctx->has_smoother = false;
  ctx->drop_graph();
  if (ctx->dim == 3) {
    if (node_masks) return fail(ctx, PNS_EUNSUPPORTED, "3D patches are not truncated");
    return ctx->es == 8 ? vanka_setup3d<double>(ctx) : vanka_setup3d<float>(ctx);
  }
  return ctx->es == 8 ? vanka_setup_impl<double>(ctx, node_masks)
                      : vanka_setup_impl<float>(ctx, node_masks);
}

int pns_vanka_smooth(pns_ctx* ctx, int level, int n_sweeps, double omega, const void* r, void* d) {
  if (ctx && ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (!check_ctx(ctx, true, true)) return ctx_code(ctx, true, true);
  if (level < 0 || level >= ctx->nlev || n_sweeps < 0 || !r || !d || r == d)
    return fail(ctx, PNS_EINVAL, "bad level, sweep count or vectors");
  if (ctx->dim == 3 && level >= 1 && level == ctx->nlev - 1)
    return fail(ctx, PNS_EINVAL, "the coarsest 3D level has no patches (dense solve)");
  if (ctx->es == 8)
    PNS_HIP(ctx, smooth<double>(ctx, level, n_sweeps, omega, (const double*)r, (double*)d, false));
  else
    PNS_HIP(ctx, smooth<float>(ctx, level, n_sweeps, omega, (const float*)r, (float*)d, false));
  return PNS_OK;
}

int pns_vanka_smooth_static(pns_ctx* ctx, int level, int n_sweeps, double omega, const void* r,
                            void* d) {
  if (!ctx) return PNS_EINVAL;
  if (ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (level < 0 || level >= ctx->nlev || n_sweeps < 0 || !r || !d || r == d)
    return fail(ctx, PNS_EINVAL, "bad level, sweep count or vectors");
  const size_t need = static_scratch_need(ctx, level);
  if (need > kStaticScratchBytes)
    return fail(ctx, PNS_EINVAL,
                "level too large for the static scratch: needs " + std::to_string(need) +
                    " bytes, the limit is " + std::to_string(kStaticScratchBytes));
  if (!check_ctx(ctx, true, true)) return ctx_code(ctx, true, true);
  if (ctx->dim == 3 && level >= 1 && level == ctx->nlev - 1)
    return fail(ctx, PNS_EINVAL, "the coarsest 3D level has no patches (dense solve)");
  void* base = nullptr;
  PNS_HIP(ctx, static_scratch(ctx->stream, &base));
  const Level& L = ctx->lev[level];
  const size_t res_bytes = (L.g.nst * ctx->es + kAlign - 1) / kAlign * kAlign;
  const size_t edge_bytes =
      (ctx->dim == 2 && level == 0)
          ? (cell_apply_edge_doubles(L.g) * 8 + kAlign - 1) / kAlign * kAlign
          : 0;
  const size_t slot_bytes =
      (ctx->dim == 2 && level >= 1) ? (L.g.nc * kNst * ctx->es + kAlign - 1) / kAlign * kAlign
                                    : 0;
  SmoothScratch sc;
  sc.res = base;
  sc.edge = (ctx->dim == 2 && level == 0) ? (double*)((char*)base + res_bytes) : nullptr;
  // 3D: per-cell results of the action; 2D coarse levels: per-patch results
  sc.slot = (ctx->dim == 3 || level >= 1) ? (void*)((char*)base + res_bytes) : nullptr;
  sc.cip = ctx->dim == 2 ? (double*)((char*)base + res_bytes + edge_bytes + slot_bytes) : nullptr;
  if (ctx->es == 8)
    PNS_HIP(ctx, smooth<double>(ctx, level, n_sweeps, omega, (const double*)r, (double*)d, false,
                                &sc));
  else
    PNS_HIP(ctx, smooth<float>(ctx, level, n_sweeps, omega, (const float*)r, (float*)d, false,
                               &sc));
  return PNS_OK;
}

int pns_vcycle(pns_ctx* ctx, int nu1, int nu2, double omega, const void* r, void* d) {
  if (ctx && ctx->prec == PNS_BF16)
    return fail(ctx, PNS_EUNSUPPORTED, "BF16 contexts have the action only");
  if (ctx && ctx->dim == 3 && ctx->nlev < 2)
    return fail(ctx, PNS_EUNSUPPORTED, "3D V-cycles need at least two levels");
  if (!check_ctx(ctx, true, true)) return ctx_code(ctx, true, true);
  if (nu1 < 0 || nu2 < 0 || !r || !d || r == d)
    return fail(ctx, PNS_EINVAL, "bad sweep counts or vectors");
  if (!ctx->has_coarse)
    return fail(ctx, PNS_EUNSUPPORTED, "coarsest level too large for the dense coarse solve");
  if (ctx->graph_mode)
    return ctx->es == 8 ? vcycle_graph<double>(ctx, nu1, nu2, omega, (const double*)r, (double*)d)
                        : vcycle_graph<float>(ctx, nu1, nu2, omega, (const float*)r, (float*)d);
  if (ctx->es == 8)
    PNS_HIP(ctx, vcycle_level<double>(ctx, 0, nu1, nu2, omega, (const double*)r, (double*)d));
  else
    PNS_HIP(ctx, vcycle_level<float>(ctx, 0, nu1, nu2, omega, (const float*)r, (float*)d));
  return PNS_OK;
}

int pns_level_apply(pns_ctx* ctx, int level, const void* x, void* y) {
  if (level == 0) return pns_cell_apply(ctx, x, y);
  if (!check_ctx(ctx, true, true)) return ctx_code(ctx, true, true);
  if (level < 0 || level >= ctx->nlev || !x || !y || x == y)
    return fail(ctx, PNS_EINVAL, "bad level or vectors");
  if (ctx->es == 8)
    PNS_HIP(ctx, apply_level<double>(ctx, level, (const double*)x, (double*)y));
  else
    PNS_HIP(ctx, apply_level<float>(ctx, level, (const float*)x, (float*)y));
  return PNS_OK;
}

int pns_restrict(pns_ctx* ctx, int level, const void* rf, void* rc) {
  if (!ctx) return PNS_EINVAL;
  if (level < 0 || level + 1 >= ctx->nlev || !rf || !rc)
    return fail(ctx, PNS_EINVAL, "bad level or vectors");
  const Grid& gf = ctx->lev[level].g;
  const Grid& gc = ctx->lev[level + 1].g;
  if (ctx->dim == 3 && ctx->es == 8)
    PNS_HIP(ctx, launch_restrict3<double>(ctx->lev[level].g3, ctx->lev[level + 1].g3,
                                          (const double*)rf, (double*)rc, ctx->stream));
  else if (ctx->dim == 3)
    PNS_HIP(ctx, launch_restrict3<float>(ctx->lev[level].g3, ctx->lev[level + 1].g3,
                                         (const float*)rf, (float*)rc, ctx->stream));
  else if (ctx->es == 8)
    PNS_HIP(ctx, launch_restrict<double>(gf, gc, (const double*)rf, (double*)rc, ctx->stream));
  else
    PNS_HIP(ctx, launch_restrict<float>(gf, gc, (const float*)rf, (float*)rc, ctx->stream));
  return PNS_OK;
}

int pns_prolongate_add(pns_ctx* ctx, int level, const void* dc, void* df) {
  if (!ctx) return PNS_EINVAL;
  if (level < 0 || level + 1 >= ctx->nlev || !dc || !df)
    return fail(ctx, PNS_EINVAL, "bad level or vectors");
  const Grid& gf = ctx->lev[level].g;
  const Grid& gc = ctx->lev[level + 1].g;
  if (ctx->dim == 3 && ctx->es == 8)
    PNS_HIP(ctx, launch_prolong_add3<double>(ctx->lev[level].g3, ctx->lev[level + 1].g3,
                                             (const double*)dc, (double*)df, ctx->stream));
  else if (ctx->dim == 3)
    PNS_HIP(ctx, launch_prolong_add3<float>(ctx->lev[level].g3, ctx->lev[level + 1].g3,
                                            (const float*)dc, (float*)df, ctx->stream));
  else if (ctx->es == 8)
    PNS_HIP(ctx, launch_prolong_add<double>(gf, gc, (const double*)dc, (double*)df, ctx->stream));
  else
    PNS_HIP(ctx, launch_prolong_add<float>(gf, gc, (const float*)dc, (float*)df, ctx->stream));
  return PNS_OK;
}

}  // extern "C"
