"""Thin ctypes binding of libpnsmg.so (include/pnsmg.h).

Argument marshalling only: every step of the smoothing step runs in the HIP
kernels of the library.  PyTorch provides the device memory (the workspace
and the vectors) and the stream.  If the library is missing this module
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpnsmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pnsmg.h")

(PNS_OK, PNS_EINVAL, PNS_EWORKSPACE, PNS_EHIP, PNS_ESTATE, PNS_ESINGULAR, PNS_EUNSUPPORTED,
 PNS_ENOTCONV, PNS_ENONFINITE) = (0, -1, -2, -3, -4, -5, -6, -7, -8)
PICARD, EXACT_NEWTON, MODIFIED_NEWTON = 0, 1, 2
FP64, FP32, BF16 = 0, 1, 2
APPLY_RECOMPUTE, APPLY_CACHED = 0, 1
PATCH_SURROGATE, PATCH_EXACT = 0, 1


class PnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pnsmg error {code}: {msg}")
        self.code = code


class pns_mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class pns_discretization(ctypes.Structure):
    _fields_ = [("k_space", ctypes.c_int), ("k_time", ctypes.c_int),
                ("t0", ctypes.c_double), ("tau", ctypes.c_double)]


class pns_model(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("delta", ctypes.c_double), ("nu", ctypes.c_double),
                ("nu_inf", ctypes.c_double), ("gamma1", ctypes.c_double),
                ("gamma2", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("convection", ctypes.c_int), ("nitsche_q_sign", ctypes.c_int),
                ("lin", ctypes.c_int), ("gamma_cip", ctypes.c_double)]


class pns_solve_params(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("max_krylov", ctypes.c_int),
                ("restart", ctypes.c_int), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("eta0", ctypes.c_double), ("eta_max", ctypes.c_double), ("rho", ctypes.c_double),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double)]


class pns_solve_info(ctypes.Structure):
    _fields_ = [("newton_iterations", ctypes.c_int), ("krylov_iterations", ctypes.c_int),
                ("smoother_setups", ctypes.c_int), ("backtracks", ctypes.c_int),
                ("residual_initial", ctypes.c_double), ("residual_final", ctypes.c_double)]


class pns_request(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int * 2), ("lo", ctypes.c_double * 2),
                ("hi", ctypes.c_double * 2), ("tau", ctypes.c_double),
                ("n_levels", ctypes.c_int), ("precision", ctypes.c_int),
                ("patch_kind", ctypes.c_int), ("model", pns_model),
                ("params", pns_solve_params), ("v_prev_host", ctypes.POINTER(ctypes.c_double)),
                ("U_host", ctypes.POINTER(ctypes.c_double)), ("vcycle_graph", ctypes.c_int)]


class pns_result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("info", pns_solve_info),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("footprint", ctypes.c_size_t)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2

SOLVE_DEFAULTS = dict(max_newton=30, max_krylov=200, restart=30, rtol=1e-8, atol=0.0, eta0=0.1,
                      eta_max=0.5, rho=0.5, nu1=2, nu2=2, omega=0.1)

_lib = None
_vp = ctypes.c_void_p


def header_symbols(path: str = HEADER):
    """Every function the public header declares."""
    txt = open(path).read()
    return sorted(set(re.findall(r"\b(pns_[a-z_0-9]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP extension {LIB_PATH} is missing: build it with "
                               "__graft_entry__.build() (hipcc for gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        i, pp = ctypes.c_int, ctypes.POINTER
        L.pns_ctx_create.argtypes = [pp(pns_mesh), pp(pns_discretization), i, i, _vp,
                                     pp(_vp)]
        L.pns_ctx_destroy.argtypes = [_vp]
        L.pns_ctx_destroy.restype = None
        L.pns_last_error.argtypes = [_vp]
        L.pns_last_error.restype = ctypes.c_char_p
        L.pns_level_sizes.argtypes = [_vp, i, pp(ctypes.c_int64)]
        L.pns_workspace_bytes.argtypes = [_vp]
        L.pns_workspace_bytes.restype = ctypes.c_size_t
        L.pns_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.pns_set_state.argtypes = [_vp, pp(pns_model), _vp]
        L.pns_cell_apply.argtypes = [_vp, _vp, _vp]
        L.pns_set_apply_mode.argtypes = [_vp, i]
        L.pns_set_patch_kind.argtypes = [_vp, i]
        L.pns_set_jacobian_precision.argtypes = [_vp, i]
        L.pns_cell_defect.argtypes = [_vp, _vp, _vp, _vp]
        L.pns_vanka_setup.argtypes = [_vp, _vp]
        L.pns_vanka_smooth.argtypes = [_vp, i, i, ctypes.c_double, _vp, _vp]
        L.pns_vanka_smooth_static.argtypes = [_vp, i, i, ctypes.c_double, _vp, _vp]
        L.pns_vcycle.argtypes = [_vp, i, i, ctypes.c_double, _vp, _vp]
        L.pns_set_vcycle_graph.argtypes = [_vp, i]
        L.pns_sweep_variant.argtypes = [_vp, i, pp(ctypes.c_int)]
        L.pns_sweep_variant_time.argtypes = [_vp, i, i, pp(ctypes.c_double)]
        L.pns_set_sweep_variant.argtypes = [_vp, i, i]
        L.pns_level_apply.argtypes = [_vp, i, _vp, _vp]
        L.pns_restrict.argtypes = [_vp, i, _vp, _vp]
        L.pns_prolongate_add.argtypes = [_vp, i, _vp, _vp]
        L.pns_residual.argtypes = [_vp, pp(pns_model), _vp, _vp, _vp]
        L.pns_load_vector.argtypes = [_vp, _vp, _vp]
        L.pns_set_load.argtypes = [_vp, _vp]
        L.pns_set_dirichlet.argtypes = [_vp, _vp]
        L.pns_set_reproducible.argtypes = [_vp, i]
        L.pns_solve_workspace_bytes.argtypes = [_vp, i]
        L.pns_solve_workspace_bytes.restype = ctypes.c_size_t
        L.pns_solve.argtypes = [_vp, pp(pns_model), _vp, _vp, pp(pns_solve_params), _vp,
                                ctypes.c_size_t, pp(pns_solve_info)]
        L.pns_march.argtypes = [_vp, pp(pns_model), _vp, i, _vp, pp(pns_solve_params), _vp,
                                ctypes.c_size_t, pp(pns_solve_info)]
        L.pns_request_footprint.argtypes = [pp(pns_request)]
        L.pns_request_footprint.restype = ctypes.c_size_t
        L.pns_server_create.argtypes = [i, _vp, ctypes.c_size_t, pp(_vp)]
        L.pns_solve_request.argtypes = [_vp, pp(pns_request), pp(ctypes.c_uint64)]
        L.pns_poll.argtypes = [_vp, ctypes.c_uint64, pp(pns_result)]
        L.pns_wait.argtypes = [_vp, ctypes.c_uint64, pp(pns_result)]
        L.pns_release.argtypes = [_vp, ctypes.c_uint64]
        L.pns_server_destroy.argtypes = [_vp]
        L.pns_server_destroy.restype = None
        for f in ("pns_server_create", "pns_solve_request", "pns_poll", "pns_wait",
                  "pns_release"):
            getattr(L, f).restype = ctypes.c_int
        for f in ("pns_ctx_create", "pns_level_sizes", "pns_bind_workspace", "pns_set_state",
                  "pns_set_apply_mode", "pns_set_patch_kind", "pns_set_jacobian_precision",
                  "pns_cell_apply", "pns_cell_defect", "pns_vanka_setup", "pns_vanka_smooth",
                  "pns_vanka_smooth_static",
                  "pns_vcycle", "pns_level_apply", "pns_restrict", "pns_prolongate_add",
                  "pns_residual", "pns_solve", "pns_load_vector", "pns_set_load"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One pns_ctx with its workspace (a torch uint8 tensor on the device)."""

    def __init__(self, n, n_levels=1, precision=FP64, tau=0.01, lo=None, hi=None,
                 device="cuda", stream=None, patch_kind=None):
        """n: cells per direction, 2 entries (quadrilaterals) or 3 (hexahedra:
        action, smoother and V-cycle); lo/hi default to the unit square or cube.
        patch_kind is selected before the workspace is sized (on hexahedra the
        exact kind needs about twice the level-0 smoother storage)."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        # element type of y, b, r, d; x of the action is BF16 in a BF16 context
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.in_dtype = torch.bfloat16 if precision == BF16 else self.dtype
        dim = len(n)
        lo = (0.0,) * dim if lo is None else lo
        hi = (1.0,) * dim if hi is None else hi
        m = pns_mesh()
        m.dim = dim
        m.n_cells[0], m.n_cells[1], m.n_cells[2] = int(n[0]), int(n[1]), int(n[2]) if dim == 3 else 1
        for k in range(dim):
            m.lo[k], m.hi[k] = float(lo[k]), float(hi[k])
        d = pns_discretization(2, 1, 0.0, float(tau))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        rc = lib().pns_ctx_create(ctypes.byref(m), ctypes.byref(d), int(n_levels), int(precision),
                                  _vp(self.stream.cuda_stream), ctypes.byref(h))
        if rc != PNS_OK:
            raise PnsError(rc, "pns_ctx_create rejected the configuration")
        self.h = h
        self.dim = dim
        self.n_levels = n_levels
        if patch_kind is not None:
            self._check(lib().pns_set_patch_kind(self.h, int(patch_kind)))
        nbytes = lib().pns_workspace_bytes(self.h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(lib().pns_bind_workspace(self.h, _vp(aligned), nbytes))
        self.workspace_bytes = nbytes

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pns_ctx_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != PNS_OK:
            raise PnsError(rc, lib().pns_last_error(self.h).decode())

    def sizes(self, level=0):
        out = (ctypes.c_int64 * 4)()
        self._check(lib().pns_level_sizes(self.h, level, out))
        return dict(nst=out[0], cells=out[1], nv=out[2], ns=out[3])

    def vector(self, level=0):
        return self.torch.zeros(self.sizes(level)["nst"], dtype=self.dtype, device=self.device)

    def _vec(self, t, level=0, dtype=None):
        assert t.dtype == (dtype or self.dtype) and t.is_contiguous() and t.device.type == "cuda"
        assert t.numel() == self.sizes(level)["nst"]
        return _ptr(t)

    def _f64(self, t, n):
        assert t.dtype == self.torch.float64 and t.is_contiguous() and t.device.type == "cuda"
        assert t.numel() == n
        return _ptr(t)

    # -------------------------------------------------------------- C-ABI
    def pns_set_state(self, model: dict, uk):
        md = model_struct(model)
        assert uk.dtype == self.torch.float64 and uk.is_contiguous()
        assert uk.numel() == 2 * self.sizes(0)["nv"]
        self._uk = uk
        self._check(lib().pns_set_state(self.h, ctypes.byref(md), _ptr(uk)))

    def pns_set_apply_mode(self, mode):
        self._check(lib().pns_set_apply_mode(self.h, int(mode)))

    def pns_set_patch_kind(self, kind):
        self._check(lib().pns_set_patch_kind(self.h, int(kind)))

    def pns_set_jacobian_precision(self, precision):
        self._check(lib().pns_set_jacobian_precision(self.h, int(precision)))

    def pns_cell_apply(self, x, y):
        self._check(lib().pns_cell_apply(self.h, self._vec(x, dtype=self.in_dtype), self._vec(y)))

    def pns_cell_defect(self, b, x, y):
        self._check(lib().pns_cell_defect(self.h, self._vec(b), self._vec(x, dtype=self.in_dtype),
                                          self._vec(y)))

    def pns_vanka_setup(self, node_masks=None):
        if node_masks is None:
            self._check(lib().pns_vanka_setup(self.h, None))
        else:
            m = np.ascontiguousarray(node_masks, dtype=np.uint16)
            assert m.size == self.sizes(0)["cells"]
            self._check(lib().pns_vanka_setup(self.h, m.ctypes.data_as(_vp)))

    def pns_vanka_smooth(self, level, n_sweeps, omega, r, d):
        self._check(lib().pns_vanka_smooth(self.h, level, n_sweeps, float(omega),
                                           self._vec(r, level), self._vec(d, level)))

    def pns_vanka_smooth_static(self, level, n_sweeps, omega, r, d):
        self._check(lib().pns_vanka_smooth_static(self.h, level, n_sweeps, float(omega),
                                                  self._vec(r, level), self._vec(d, level)))

    def pns_vcycle(self, nu1, nu2, omega, r, d):
        self._check(lib().pns_vcycle(self.h, nu1, nu2, float(omega), self._vec(r), self._vec(d)))

    def pns_sweep_variant(self, level=0):
        out = (ctypes.c_int * 5)()
        self._check(lib().pns_sweep_variant(self.h, level, out))
        return dict(variant=out[0], count=out[1], waves=out[2], unroll=out[3], rows=out[4])

    def pns_sweep_variant_time(self, level, variant):
        ms = ctypes.c_double()
        self._check(lib().pns_sweep_variant_time(self.h, level, variant, ctypes.byref(ms)))
        return ms.value

    def pns_set_sweep_variant(self, level, variant):
        self._check(lib().pns_set_sweep_variant(self.h, level, variant))

    def pns_set_vcycle_graph(self, enable):
        self._check(lib().pns_set_vcycle_graph(self.h, int(enable)))

    def pns_level_apply(self, level, x, y):
        self._check(lib().pns_level_apply(self.h, level, self._vec(x, level), self._vec(y, level)))

    def pns_restrict(self, level, rf, rc):
        self._check(lib().pns_restrict(self.h, level, self._vec(rf, level),
                                       self._vec(rc, level + 1)))

    def pns_prolongate_add(self, level, dc, df):
        self._check(lib().pns_prolongate_add(self.h, level, self._vec(dc, level + 1),
                                             self._vec(df, level)))

    def pns_residual(self, model: dict, U, vprev, R):
        sz = self.sizes(0)
        vp = None if vprev is None else self._f64(vprev, sz["nv"])
        self._check(lib().pns_residual(self.h, ctypes.byref(model_struct(model)),
                                       self._f64(U, sz["nst"]), vp, self._f64(R, sz["nst"])))

    def pns_load_vector(self, f_qp, F):
        """F (FP64, N_st) = the volume-force vector of f at the Gauss points
        (FP64 device tensor [2, cells, 3^d, d])."""
        sz = self.sizes(0)
        d = self.dim
        self._f64(f_qp, 2 * sz["cells"] * 3 ** d * d)
        self._check(lib().pns_load_vector(self.h, _ptr(f_qp), self._f64(F, sz["nst"])))

    def pns_set_load(self, F):
        """Add F (FP64 device tensor of N_st values, kept alive by the caller)
        to every slab residual; None clears it."""
        if F is None:
            self._load = None
            self._check(lib().pns_set_load(self.h, None))
            return
        self._load = F
        self._check(lib().pns_set_load(self.h, self._f64(F, self.sizes(0)["nst"])))

    def pns_set_reproducible(self, on):
        self._check(lib().pns_set_reproducible(self.h, int(on)))

    def pns_set_dirichlet(self, ghat):
        """Dirichlet data from a lifting: FP64 device tensor of 2 N_v values (the
        Q2 velocity field at each Radau node; kept alive by the caller); None:
        homogeneous data."""
        if ghat is None:
            self._lift = None
            self._check(lib().pns_set_dirichlet(self.h, None))
            return
        self._lift = ghat
        self._check(lib().pns_set_dirichlet(self.h, self._f64(ghat, 2 * self.sizes(0)["nv"])))

    def pns_solve_workspace_bytes(self, restart):
        return lib().pns_solve_workspace_bytes(self.h, int(restart))

    def pns_solve(self, model: dict, vprev, U, check=True, **params):
        """Newton-Krylov slab solve; U (FP64) is updated in place.  Returns
        (return code, info dict); raises on errors other than PNS_ENOTCONV and
        PNS_ENONFINITE unless check is False."""
        prm = dict(SOLVE_DEFAULTS, **params)
        ps = pns_solve_params(*(prm[f] for f, _ in pns_solve_params._fields_))
        nbytes = self.pns_solve_workspace_bytes(ps.restart)
        if nbytes == 0:
            raise PnsError(PNS_EINVAL, "invalid restart length")
        work = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        base = (work.data_ptr() + 255) // 256 * 256
        sz = self.sizes(0)
        vp = None if vprev is None else self._f64(vprev, sz["nv"])
        info = pns_solve_info()
        rc = lib().pns_solve(self.h, ctypes.byref(model_struct(model)), vp,
                             self._f64(U, sz["nst"]), ctypes.byref(ps), _vp(base), nbytes,
                             ctypes.byref(info))
        if check and rc not in (PNS_OK, PNS_ENOTCONV, PNS_ENONFINITE):
            self._check(rc)
        del work
        return rc, {f: getattr(info, f) for f, _ in pns_solve_info._fields_}

    def pns_march(self, model: dict, v, n_slabs, U, check=True, **params):
        """Time marching over n_slabs slabs: v (FP64, velocity) is advanced in
        place, U (FP64) holds the last slab's solution.  Returns (return code,
        info dict with the summed iteration counts)."""
        prm = dict(SOLVE_DEFAULTS, **params)
        ps = pns_solve_params(*(prm[f] for f, _ in pns_solve_params._fields_))
        nbytes = self.pns_solve_workspace_bytes(ps.restart)
        if nbytes == 0:
            raise PnsError(PNS_EINVAL, "invalid restart length")
        work = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        base = (work.data_ptr() + 255) // 256 * 256
        sz = self.sizes(0)
        info = pns_solve_info()
        rc = lib().pns_march(self.h, ctypes.byref(model_struct(model)), self._f64(v, sz["nv"]),
                             int(n_slabs), self._f64(U, sz["nst"]), ctypes.byref(ps), _vp(base),
                             nbytes, ctypes.byref(info))
        if check and rc not in (PNS_OK, PNS_ENOTCONV, PNS_ENONFINITE):
            self._check(rc)
        del work
        return rc, {f: getattr(info, f) for f, _ in pns_solve_info._fields_}


def model_struct(model: dict):
    return pns_model(
        float(model["p"]), float(model["delta"]), float(model.get("nu", 1.0)),
        float(model.get("nu_inf", 0.0)), float(model.get("gamma1", 40.0)),
        float(model.get("gamma2", 40.0)), float(model.get("sigma_max", 1.0)),
        int(model.get("convection", 1)), int(model.get("qsign", 1)),
        int(model.get("lin", MODIFIED_NEWTON)), float(model.get("gamma_cip", 0.0)))


def masks_to_bits(masks):
    """(cells, 9) 0/1 keep-masks -> one uint16 bit field per cell."""
    masks = np.asarray(masks)
    return (masks.astype(np.uint16) << np.arange(masks.shape[1], dtype=np.uint16)).sum(
        axis=1).astype(np.uint16)


def make_request(n, model: dict, vprev, U_out, levels, precision=FP64, tau=0.01,
                 patch_kind=PATCH_SURROGATE, lo=(0.0, 0.0), hi=(1.0, 1.0), vcycle_graph=0,
                 **params):
    """pns_request for an n[0] x n[1] slab solve; vprev and U_out are float64
    numpy arrays that must stay alive until the request is done."""
    assert vprev.dtype == np.float64 and vprev.flags.c_contiguous
    assert U_out.dtype == np.float64 and U_out.flags.c_contiguous
    prm = dict(SOLVE_DEFAULTS, **params)
    q = pns_request()
    q.n_cells[0], q.n_cells[1] = int(n[0]), int(n[1])
    q.lo[0], q.lo[1] = float(lo[0]), float(lo[1])
    q.hi[0], q.hi[1] = float(hi[0]), float(hi[1])
    q.tau = float(tau)
    q.n_levels = int(levels)
    q.precision = int(precision)
    q.patch_kind = int(patch_kind)
    q.model = model_struct(model)
    q.params = pns_solve_params(*(prm[f] for f, _ in pns_solve_params._fields_))
    q.v_prev_host = vprev.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    q.U_host = U_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    q.vcycle_graph = int(vcycle_graph)
    return q


def result_dict(r: pns_result):
    return dict(state=r.state, status=r.status, t_submit=r.t_submit, t_start=r.t_start,
                t_done=r.t_done, footprint=r.footprint,
                **{f: getattr(r.info, f) for f, _ in pns_solve_info._fields_})


class Server:
    """A pns_server over a device arena (a torch uint8 tensor)."""

    def __init__(self, slots, arena_bytes, device="cuda"):
        import torch

        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=device)
        base = (self.arena.data_ptr() + 255) // 256 * 256
        h = _vp()
        rc = lib().pns_server_create(int(slots), _vp(base), int(arena_bytes), ctypes.byref(h))
        if rc != PNS_OK:
            raise PnsError(rc, "pns_server_create failed")
        self.h = h
        self._keep = {}

    def footprint(self, req):
        return lib().pns_request_footprint(ctypes.byref(req))

    def submit(self, req, keep=()):
        t = ctypes.c_uint64()
        rc = lib().pns_solve_request(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc != PNS_OK:
            raise PnsError(rc, "pns_solve_request rejected the request")
        self._keep[t.value] = (req, keep)
        return t.value

    def poll(self, ticket):
        r = pns_result()
        if lib().pns_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(r)) != PNS_OK:
            raise PnsError(PNS_EINVAL, "unknown ticket")
        return result_dict(r)

    def wait(self, ticket):
        r = pns_result()
        if lib().pns_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(r)) != PNS_OK:
            raise PnsError(PNS_EINVAL, "unknown ticket")
        return result_dict(r)

    def release(self, ticket):
        rc = lib().pns_release(self.h, ctypes.c_uint64(ticket))
        if rc != PNS_OK:
            raise PnsError(rc, "pns_release: unknown ticket or request not done")
        self._keep.pop(ticket, None)

    def close(self):
        if getattr(self, "h", None):
            lib().pns_server_destroy(self.h)
            self.h = None

    def __del__(self):
        if _lib is not None:
            self.close()
