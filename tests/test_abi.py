"""Host-side checks of the C-ABI library (no GPU needed): the shared object
loads, exports every function include/pnsmg.h declares, and rejects invalid
configurations before touching a device."""
import ctypes
import os

import pytest

from paper_2603_28706_amd import pnsmg


def test_library_exports_every_header_symbol():
    L = pnsmg.lib()
    syms = pnsmg.header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s


def _create(n=(8, 8), levels=1, prec=pnsmg.FP64, tau=0.01, dim=None, k_space=2, k_time=1,
            hi=1.0):
    m = pnsmg.pns_mesh()
    m.dim = len(n) if dim is None else dim
    m.n_cells[0], m.n_cells[1], m.n_cells[2] = n[0], n[1], n[2] if len(n) == 3 else 1
    m.hi[0] = m.hi[1] = m.hi[2] = hi
    d = pnsmg.pns_discretization(k_space, k_time, 0.0, tau)
    h = ctypes.c_void_p()
    rc = pnsmg.lib().pns_ctx_create(ctypes.byref(m), ctypes.byref(d), levels, prec, None,
                                    ctypes.byref(h))
    return rc, h


def test_create_rejects_bad_configurations():
    assert _create(dim=1)[0] == pnsmg.PNS_EUNSUPPORTED
    assert _create(n=(4, 4, 4), dim=4)[0] == pnsmg.PNS_EUNSUPPORTED
    assert _create(n=(6, 4, 4), levels=3)[0] == pnsmg.PNS_EINVAL  # 6 not divisible by 4
    assert _create(n=(4, 4, 4), levels=11)[0] == pnsmg.PNS_EINVAL
    assert _create(n=(4, 4, 0))[0] == pnsmg.PNS_EINVAL
    assert _create(n=(4, 4, 4), hi=0.0)[0] == pnsmg.PNS_EINVAL
    assert _create(n=(4, 4, 4), k_time=2)[0] == pnsmg.PNS_EUNSUPPORTED
    assert _create(k_time=2)[0] == pnsmg.PNS_EUNSUPPORTED
    assert _create(tau=0.0)[0] == pnsmg.PNS_EINVAL
    assert _create(n=(6, 8), levels=3)[0] == pnsmg.PNS_EINVAL     # not divisible by 4
    assert _create(n=(4, 4), levels=4)[0] == pnsmg.PNS_EINVAL     # 4 not divisible by 8
    assert _create(prec=7)[0] == pnsmg.PNS_EINVAL
    rc, h = _create(n=(256, 256), levels=1)   # apply-only context: no dense coarse solve
    assert rc == pnsmg.PNS_OK
    assert pnsmg.lib().pns_workspace_bytes(h) < 4 * 2 ** 30
    pnsmg.lib().pns_ctx_destroy(h)


def test_workspace_query_and_state_errors_without_device():
    rc, h = _create(n=(16, 16), levels=3)
    assert rc == pnsmg.PNS_OK
    L = pnsmg.lib()
    nbytes = L.pns_workspace_bytes(h)
    assert nbytes > 0 and nbytes % 256 == 0
    out = (ctypes.c_int64 * 4)()
    assert L.pns_level_sizes(h, 0, out) == 0 and out[0] == 2 * (2 * 33 ** 2 + 3 * 256)
    assert L.pns_level_sizes(h, 2, out) == 0 and out[1] == 16
    assert L.pns_level_sizes(h, 3, out) == pnsmg.PNS_EINVAL
    # calls before a workspace is bound fail cleanly
    x = ctypes.c_void_p(1024)
    assert L.pns_cell_apply(h, x, ctypes.c_void_p(2048)) == pnsmg.PNS_EWORKSPACE
    assert L.pns_bind_workspace(h, ctypes.c_void_p(1000), nbytes) == pnsmg.PNS_EWORKSPACE
    assert L.pns_bind_workspace(h, ctypes.c_void_p(4096), 16) == pnsmg.PNS_EWORKSPACE
    assert b"workspace" in L.pns_last_error(h)
    L.pns_ctx_destroy(h)


def lift3(nx, ny, nz):
    """Bytes of one hexahedral Dirichlet-data table."""
    return 2 * (ny * nz + nx * nz + nx * ny) * 9 * 3 * 11 * 8


def test_3d_context_layout_and_rejections():
    """A hexahedral context: unknown counts of Q2^3 / P1disc x dG(1); the
    workspace holds the state, the per-cell results of the action and the
    finest-level smoother (midpoint state, FP64 cell matrices, complex 85 x 85
    patch inverses, defect) and the FP64 residual's buffers; the exact patch
    kind adds the second Radau node's cell matrices and doubles the inverse
    storage, and a bound workspace too small for it rejects the switch; a
    one-level V-cycle and truncated patches are rejected before any device
    work."""
    rc, h = _create(n=(32, 32, 32))
    assert rc == pnsmg.PNS_OK
    L = pnsmg.lib()
    out = (ctypes.c_int64 * 4)()
    assert L.pns_level_sizes(h, 0, out) == 0
    nv = 3 * 65 ** 3
    nst = 1909894
    assert (out[0], out[1], out[2], out[3]) == (nst, 32768, nv, nv + 4 * 32768)
    assert L.pns_level_sizes(h, 1, out) == pnsmg.PNS_EINVAL
    nbytes = L.pns_workspace_bytes(h)
    es = 8
    kE = 170 * 170
    # state, action slots, residual buffers, midpoint state, one set of
    # spatial cell matrices, defect, complex 85 x 85 patch inverses
    # (and two Dirichlet-data tables: 9 points x 3 time slots x 11 values per
    # boundary face)
    base = 2 * nv * (es + 8) + 32768 * 170 * es + 2 * nv * 8 + nst * 8 + 32768 * 170 * 8
    base += 2 * lift3(32, 32, 32)
    need = base + nv * 8 + 16 + 32768 * 85 * 85 * 8 + nst * es + 32768 * 2 * 85 * 85 * es
    assert need <= nbytes < need + 4096
    # exact patches: both Radau nodes' cell matrices, real 170 x 170 inverses
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_EXACT) == pnsmg.PNS_OK
    need_x = base + nv * 8 + 16 + 2 * 32768 * 85 * 85 * 8 + nst * es + 32768 * kE * es
    nbytes_x = L.pns_workspace_bytes(h)
    assert need_x <= nbytes_x < need_x + 4096
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_SURROGATE) == pnsmg.PNS_OK
    assert L.pns_workspace_bytes(h) == nbytes
    # binding does no device work: a surrogate-sized buffer refuses the switch
    fake = ctypes.c_void_p(1 << 40)
    assert L.pns_bind_workspace(h, fake, ctypes.c_size_t(nbytes)) == pnsmg.PNS_OK
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_EXACT) == pnsmg.PNS_EWORKSPACE
    assert b"too small" in L.pns_last_error(h)
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_SURROGATE) == pnsmg.PNS_OK
    assert L.pns_bind_workspace(h, fake, ctypes.c_size_t(nbytes_x)) == pnsmg.PNS_OK
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_EXACT) == pnsmg.PNS_OK
    assert L.pns_workspace_bytes(h) == nbytes_x
    L.pns_ctx_destroy(h)
    rc, h = _create(n=(32, 32, 32))
    assert rc == pnsmg.PNS_OK
    # FGMRES(30) vectors: 31 + 30 Krylov vectors and 6 work vectors of N_st FP64
    assert L.pns_solve_workspace_bytes(h, 30) >= (61 + 6) * nst * 8
    assert L.pns_set_apply_mode(h, pnsmg.APPLY_CACHED) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_set_apply_mode(h, pnsmg.APPLY_RECOMPUTE) == pnsmg.PNS_OK
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_EXACT) == pnsmg.PNS_OK
    assert L.pns_set_patch_kind(h, pnsmg.PATCH_SURROGATE) == pnsmg.PNS_OK
    v = ctypes.c_void_p(4096)
    w = ctypes.c_void_p(8192)
    assert L.pns_vanka_setup(h, None) == pnsmg.PNS_EWORKSPACE
    assert L.pns_vanka_smooth(h, 0, 1, ctypes.c_double(0.1), v, w) == pnsmg.PNS_EWORKSPACE
    assert L.pns_vcycle(h, 1, 1, ctypes.c_double(0.1), v, w) == pnsmg.PNS_EUNSUPPORTED
    model = pnsmg.model_struct(dict(p=1.3, delta=1e-3, nu=1.0, nu_inf=1e-4, gamma1=40.0,
                                    gamma2=40.0, sigma_max=1.0, convection=1, qsign=1, lin=2))
    assert L.pns_residual(h, ctypes.byref(model), v, None, w) == pnsmg.PNS_EWORKSPACE
    info = pnsmg.pns_solve_info()
    assert L.pns_solve(h, ctypes.byref(model), v, w, None, None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EWORKSPACE
    assert L.pns_cell_apply(h, v, w) == pnsmg.PNS_EWORKSPACE
    # graph mode may be switched on; the one-level V-cycle itself is refused
    assert L.pns_set_vcycle_graph(h, 1) == pnsmg.PNS_OK
    assert L.pns_vcycle(h, 1, 1, ctypes.c_double(0.1), v, w) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_set_vcycle_graph(h, 0) == pnsmg.PNS_OK
    L.pns_ctx_destroy(h)
    # three levels 8^3 -> 4^3 -> 2^3: the two vectors of graph-replayed
    # V-cycles, level-0 matrices of both Radau nodes, Galerkin matrices (FP64
    # and transposed copies), real inverses of level 1, the dense coarsest
    # inverse
    rc, h = _create(n=(8, 8, 8), levels=3)
    assert rc == pnsmg.PNS_OK
    sizes = []
    for lev in range(3):
        assert L.pns_level_sizes(h, lev, out) == 0
        sizes.append((out[0], out[1]))
    assert sizes == [(33574, 512), (4886, 64), (814, 8)]
    kE = 170 * 170
    need = (2 * 3 * 17 ** 3 * 16 + 512 * 170 * 8 + 3 * 17 ** 3 * 8 + 2 * 512 * 85 * 85 * 8 + 16
            + 2 * 3 * 17 ** 3 * 8 + 33574 * 8 + 512 * 170 * 8 + 2 * 33574 * 8
            + 33574 * 8 + 512 * 2 * 85 * 85 * 8
            + 4886 * 8 * 3 + 64 * kE * 16 + 64 * kE * 8
            + 814 * 8 * 3 + 8 * kE * 16
            + 814 * 814 * 8 + (3 * 128 * 814 + 4 * 13 + 8) * 8 + 814 * 4
            + 2 * lift3(8, 8, 8))
    assert need <= L.pns_workspace_bytes(h) < need + 8192
    L.pns_ctx_destroy(h)
    # BF16: hexahedral action only (state in BF16, action slots in FP32)
    rc, h = _create(n=(4, 2, 3), prec=pnsmg.BF16)
    assert rc == pnsmg.PNS_OK
    nn3, nc3 = 9 * 5 * 7, 24
    need = 2 * 3 * nn3 * (2 + 8) + nc3 * 170 * 4
    assert need <= L.pns_workspace_bytes(h) < need + 1024
    assert L.pns_vanka_setup(h, None) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_vanka_smooth(h, 0, 1, ctypes.c_double(0.1), v, w) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_vcycle(h, 1, 1, ctypes.c_double(0.1), v, w) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_residual(h, ctypes.byref(model), v, None, w) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_solve_workspace_bytes(h, 30) == 0
    assert L.pns_set_vcycle_graph(h, 1) == pnsmg.PNS_EUNSUPPORTED
    L.pns_ctx_destroy(h)
    assert _create(n=(4, 4, 4), levels=2, prec=pnsmg.BF16)[0] == pnsmg.PNS_EUNSUPPORTED
    assert _create(n=(8, 8), prec=pnsmg.BF16)[0] == pnsmg.PNS_EINVAL
    # FP32: inverses and defect in single precision
    rc, h = _create(n=(4, 2, 3), prec=pnsmg.FP32)
    assert rc == pnsmg.PNS_OK
    nn = 9 * 5 * 7
    nc = 24
    nst = 2 * (3 * nn + 4 * nc)
    need = (2 * 3 * nn * (4 + 8) + nc * 170 * 4 + 3 * nn * 8 + nc * 85 * 85 * 8 + 16
            + nc * 2 * 85 * 85 * 4 + nst * 4 + 2 * 3 * nn * 8 + nst * 8 + nc * 170 * 8
            + 2 * lift3(4, 2, 3))
    assert need <= L.pns_workspace_bytes(h) < need + 4096
    L.pns_ctx_destroy(h)


def test_sweep_variant_entry_points_reject_bad_arguments():
    L = pnsmg.lib()
    rc, h = _create((8, 8), 2)
    assert rc == pnsmg.PNS_OK
    out = (ctypes.c_int * 5)()
    assert L.pns_sweep_variant(h, 0, out) == pnsmg.PNS_OK
    assert out[0] == 0 and out[1] == 6            # complex level-0 patches: 6 variants
    assert L.pns_sweep_variant(h, 1, out) == pnsmg.PNS_OK and out[1] == 12
    assert L.pns_sweep_variant(h, 2, out) == pnsmg.PNS_EINVAL
    assert L.pns_set_sweep_variant(h, 0, 6) == pnsmg.PNS_EINVAL
    assert L.pns_set_sweep_variant(h, 1, 11) == pnsmg.PNS_OK
    assert L.pns_set_sweep_variant(h, -1, 0) == pnsmg.PNS_EINVAL
    ms = ctypes.c_double(-1.0)
    assert L.pns_sweep_variant_time(h, 1, 3, ctypes.byref(ms)) == pnsmg.PNS_OK and ms.value == 0.0
    assert L.pns_sweep_variant_time(h, 1, 12, ctypes.byref(ms)) == pnsmg.PNS_EINVAL
    L.pns_ctx_destroy(h)
    rc, h = _create((2, 2, 2))
    assert L.pns_sweep_variant(h, 0, out) == pnsmg.PNS_EINVAL
    L.pns_ctx_destroy(h)


def test_march_rejects_bad_arguments():
    L = pnsmg.lib()
    model = pnsmg.model_struct(dict(p=1.8, delta=1e-2, nu=0.1, nu_inf=1e-4))
    prm = pnsmg.pns_solve_params(*(pnsmg.SOLVE_DEFAULTS[f] for f, _ in
                                   pnsmg.pns_solve_params._fields_))
    info = pnsmg.pns_solve_info()
    assert L.pns_march(None, ctypes.byref(model), None, 1, None, ctypes.byref(prm), None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EINVAL
    rc, h = _create((8, 8), 2)
    v, U = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    assert L.pns_march(h, ctypes.byref(model), v, -1, U, ctypes.byref(prm), None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EINVAL
    assert L.pns_march(h, ctypes.byref(model), v, 1, v, ctypes.byref(prm), None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EINVAL
    assert L.pns_march(h, ctypes.byref(model), v, 1, U, ctypes.byref(prm), None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EWORKSPACE
    L.pns_ctx_destroy(h)
    rc, h = _create((2, 2, 2), 2)  # 3D: same checks, no workspace bound yet
    assert L.pns_march(h, ctypes.byref(model), v, 1, U, ctypes.byref(prm), None, 0,
                       ctypes.byref(info)) == pnsmg.PNS_EWORKSPACE
    L.pns_ctx_destroy(h)


def test_vcycle_graph_switch_rejects_bad_arguments():
    L = pnsmg.lib()
    assert L.pns_set_vcycle_graph(None, 1) == pnsmg.PNS_EINVAL
    rc, h = _create((8, 8), 2)
    assert rc == pnsmg.PNS_OK
    assert L.pns_set_vcycle_graph(h, 2) == pnsmg.PNS_EINVAL
    assert L.pns_set_vcycle_graph(h, 1) == pnsmg.PNS_OK
    assert L.pns_set_vcycle_graph(h, 0) == pnsmg.PNS_OK
    # without a workspace the V-cycle is rejected in either mode
    assert L.pns_set_vcycle_graph(h, 1) == pnsmg.PNS_OK
    assert L.pns_vcycle(h, 2, 2, ctypes.c_double(0.1), ctypes.c_void_p(4096),
                        ctypes.c_void_p(8192)) == pnsmg.PNS_EWORKSPACE
    L.pns_ctx_destroy(h)


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(pnsmg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pnsmg, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pnsmg.lib()


def test_solve_workspace_query_rejects_bad_arguments():
    L = pnsmg.lib()
    assert L.pns_solve_workspace_bytes(None, 30) == 0
    rc, h = _create((8, 8), 2)
    assert rc == pnsmg.PNS_OK
    try:
        assert L.pns_solve_workspace_bytes(h, 0) == 0
        assert L.pns_solve_workspace_bytes(h, 201) == 0
        a = L.pns_solve_workspace_bytes(h, 10)
        b = L.pns_solve_workspace_bytes(h, 20)
        nst = 2 * (2 * 17 * 17 + 3 * 64)
        # ten more Krylov and ten more preconditioned vectors of N_st doubles
        assert b - a >= 20 * nst * 8
    finally:
        L.pns_ctx_destroy(h)


def test_solve_and_residual_reject_calls_without_workspace():
    L = pnsmg.lib()
    rc, h = _create((8, 8), 2)
    assert rc == pnsmg.PNS_OK
    try:
        md = pnsmg.model_struct(dict(p=1.5, delta=1e-2))
        assert L.pns_residual(h, ctypes.byref(md), None, None, None) == pnsmg.PNS_EWORKSPACE
        prm = pnsmg.pns_solve_params(*(pnsmg.SOLVE_DEFAULTS[f] for f, _ in
                                       pnsmg.pns_solve_params._fields_))
        rc = L.pns_solve(h, ctypes.byref(md), None, None, ctypes.byref(prm), None, 0, None)
        assert rc == pnsmg.PNS_EWORKSPACE
    finally:
        L.pns_ctx_destroy(h)


def test_server_entry_points_reject_bad_arguments():
    import numpy as np

    L = pnsmg.lib()
    h = ctypes.c_void_p()
    assert L.pns_server_create(0, None, 0, ctypes.byref(h)) == pnsmg.PNS_EINVAL
    assert L.pns_server_create(17, ctypes.c_void_p(256), 1 << 20, ctypes.byref(h)) == pnsmg.PNS_EINVAL
    assert L.pns_server_create(1, ctypes.c_void_p(100), 1 << 20, ctypes.byref(h)) == pnsmg.PNS_EINVAL
    # request sizes are computed on the host: invalid requests have no footprint
    vp = np.zeros(2 * 17 * 17)
    U = np.zeros(2 * (2 * 17 * 17 + 3 * 64))
    good = pnsmg.make_request((8, 8), dict(p=1.5, delta=1e-2), vp, U, levels=2)
    assert L.pns_request_footprint(ctypes.byref(good)) > 0
    bad_p = pnsmg.make_request((8, 8), dict(p=2.5, delta=1e-2), vp, U, levels=2)
    assert L.pns_request_footprint(ctypes.byref(bad_p)) == 0
    bad_levels = pnsmg.make_request((8, 8), dict(p=1.5, delta=1e-2), vp, U, levels=5)
    assert L.pns_request_footprint(ctypes.byref(bad_levels)) == 0
    too_big_coarse = pnsmg.make_request((256, 256), dict(p=1.5, delta=1e-2), vp, U, levels=1)
    assert L.pns_request_footprint(ctypes.byref(too_big_coarse)) == 0


def test_jacobian_precision_selection_without_device():
    """BF16 Jacobian storage is offered on hexahedral FP32 contexts only; it
    enlarges the solve work buffer by its BF16 staging."""
    L = pnsmg.lib()
    rc, h = _create(n=(4, 4, 4), levels=2, prec=pnsmg.FP32)
    assert rc == pnsmg.PNS_OK
    before = L.pns_solve_workspace_bytes(h, 30)
    assert L.pns_set_jacobian_precision(h, 7) == pnsmg.PNS_EINVAL
    assert L.pns_set_jacobian_precision(h, pnsmg.FP64) == pnsmg.PNS_EUNSUPPORTED
    assert L.pns_set_jacobian_precision(h, pnsmg.BF16) == pnsmg.PNS_OK
    after = L.pns_solve_workspace_bytes(h, 30)
    assert after >= before + 2 * (2 * (3 * 9 ** 3 + 4 * 64)) + 4 * 3 * 9 ** 3
    assert L.pns_set_jacobian_precision(h, pnsmg.FP32) == pnsmg.PNS_OK
    assert L.pns_solve_workspace_bytes(h, 30) == before
    L.pns_ctx_destroy(h)
    for n, prec in (((8, 8), pnsmg.FP32), ((4, 4, 4), pnsmg.FP64)):
        rc, h = _create(n=n, levels=1, prec=prec)
        assert rc == pnsmg.PNS_OK
        assert L.pns_set_jacobian_precision(h, pnsmg.BF16) == pnsmg.PNS_EUNSUPPORTED
        L.pns_ctx_destroy(h)


def test_fp32_contexts_hold_an_fp32_copy_of_the_coarsest_inverse():
    """The dense coarsest inverse is formed in FP64; an FP32 context keeps an
    FP32 copy of it, which its V-cycles read (n^2 x 4 more bytes)."""
    L = pnsmg.lib()
    out = (ctypes.c_int64 * 4)()
    ws = {}
    for prec in (pnsmg.FP64, pnsmg.FP32):
        rc, h = _create(n=(32, 32), levels=2, prec=prec)
        assert rc == pnsmg.PNS_OK
        assert L.pns_level_sizes(h, 1, out) == 0
        n = out[0]
        ws[prec] = L.pns_workspace_bytes(h)
        L.pns_ctx_destroy(h)
    assert n == 2 * (2 * 33 ** 2 + 3 * 256)
    # every other buffer of the FP32 context is at most as large as in FP64
    assert ws[pnsmg.FP64] >= n * n * 8
    assert ws[pnsmg.FP32] >= n * n * 12 and ws[pnsmg.FP32] > ws[pnsmg.FP64]
