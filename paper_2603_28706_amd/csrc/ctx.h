// Internal: the context behind the opaque pns_ctx handle, shared by the C-ABI
// entry points (api.hip) and the slab solve (solve.hip).
#pragma once

#include <string>
#include <vector>

#include "pns_internal.h"

namespace pns {

struct Level {
  Grid g;                 // sizes (both dimensions); the quadrilateral mesh in 2D
  Grid3 g3{};             // the hexahedral mesh of the level (3D contexts)
  double* E64 = nullptr;  // Galerkin element matrices (FP64), levels >= 1 (and 0 if coarsest)
  void* E = nullptr;      // same, transposed per cell, in the context precision
  void* inv = nullptr;    // patch inverses, column-major, context precision (level 0
                          // with surrogate patches: complex 21x21 time-diagonal form)
  void* res = nullptr;    // defect
  void* r = nullptr;      // level right-hand side (levels >= 1)
  void* d = nullptr;      // level correction (levels >= 1)
  double* S = nullptr;    // 2D CIP face matrices of the level operator (3x3 per face
                          // and Radau node; level 0: at u_k, scaled by tau w_mu)
};

constexpr size_t kAlign = 256;
constexpr int64_t kMaxCoarse = 40000;  // dense coarsest inverse limit

inline int fail_msg(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

// Model of the kernels from the ABI description; PNS_OK or PNS_EINVAL with a message.
int make_model(const pns_model* md, Model* m, std::string* err);

}  // namespace pns

struct pns_ctx {
  int dim = 2;         // 3: hexahedra
  pns::Grid3 g3{};     // the 3D mesh (dim == 3)
  pns_mesh mesh{};
  pns_discretization disc{};
  int prec = PNS_FP64;
  size_t es = 8;
  int nlev = 1;
  hipStream_t stream = nullptr;
  std::vector<pns::Level> lev;
  pns::Model model{};
  bool has_state = false, has_smoother = false;
  std::string err;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // level-0 data
  void* uk = nullptr;
  double* uk64 = nullptr;
  double* urep = nullptr;
  double* Es0 = nullptr;
  double* Es1 = nullptr;
  double* Esr = nullptr;
  uint16_t* masks = nullptr;
  int* status = nullptr;
  // coarsest level (dense inverse when it is small enough)
  double* Adense = nullptr;
  float* Adense32 = nullptr;  // FP32 copy of the coarsest inverse (FP32 contexts)
  double* gjwork = nullptr;
  int* gjpiv = nullptr;
  int64_t pin[2] = {-1, -1};
  bool has_coarse = false;
  int apply_mode = PNS_APPLY_RECOMPUTE;
  int patch_kind = PNS_PATCH_SURROGATE;  // finest-level patch matrices
  void* tcache = nullptr;  // per-point tangent coefficients of level 0
  double* edge2 = nullptr;  // 2D action: per-tile partial sums on shared tile edges
  double* cipG = nullptr;   // 2D CIP: per-face weighted jumps
  double* Sr = nullptr;     // 2D CIP face matrices at t_rep (time-diagonal patches)
  void* E3 = nullptr;      // 3D: per-cell results of the action (170 per cell)
  void* slot2 = nullptr;   // 2D: per-patch results of the coarse-level sweeps and actions
  // 3D FP64 residual: state copy, left-trace term, per-cell slots of the action
  double* r3u = nullptr;
  double* r3b = nullptr;
  double* r3slot = nullptr;
  // patch-sweep variant per level (chosen by timing at pns_vanka_setup) and the
  // measured time of every variant of that level's form
  int sweep_var[16] = {};
  float sweep_ms[16][16] = {};
  // volume-force vector added to every slab residual (pns_set_load), or NULL
  const double* load = nullptr;
  // Dirichlet lifting per Radau node (pns_set_dirichlet, caller-owned), or NULL;
  // its boundary tables (2D): for the state's model (action, smoother) and for
  // the model of the last residual evaluation
  const double* lift = nullptr;
  double* ltab = nullptr;
  double* ltab_r = nullptr;
  // 2D action and residual in a fixed summation order (pns_set_reproducible)
  bool ordered = false;
  // pns_solve's Jacobian action with x and u_k stored in BF16 (3D FP32
  // contexts, pns_set_jacobian_precision)
  bool jac_bf16 = false;
  // V-cycles replayed from a captured HIP graph (pns_set_vcycle_graph)
  bool graph_mode = false;
  void* gr = nullptr;  // level-0 right-hand side and correction read / written by the graph
  void* gd = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t vgraph = nullptr;
  int g_nu1 = -1, g_nu2 = -1;
  double g_omega = 0.0;
  void drop_graph() {
    if (vgraph) (void)hipGraphExecDestroy(vgraph);
    vgraph = nullptr;
  }
  ~pns_ctx() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

#define PNS_HIP(ctx, call)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return pns::fail_msg((ctx) ? &(ctx)->err : nullptr, PNS_EHIP,                         \
                           std::string("HIP error: ") + hipGetErrorString(e_) + " at " + #call); \
  } while (0)
