"""pns_vanka_smooth_static, the allocation-free variant of pns_vanka_smooth
(its defect, tile-edge partial sums and 3D result slots in the library's static
device array): the same Vanka steps as pns_vanka_smooth on the same context,
on two calls in a row with the second on a smaller mesh (the array keeps the
first call's contents), on level 0 and on a coarse level, quadrilaterals and
hexahedra, FP64 and FP32; and the size limit, rejected before any device work.

Both entry points run the same kernels; the 2D level-0 action sums the cells
of a tile with LDS atomics, so the FP64 results agree to rounding (bound
1e-13 relative), FP32 to 1e-5."""
import ctypes

import numpy as np
import pytest

# torch first: the library then runs on the HIP runtime torch has loaded
torch = pytest.importorskip("torch")

from paper_2603_28706_amd import inputs, pnsmg  # noqa: E402

MODEL = dict(p=1.5, delta=1e-2, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1, lin=pnsmg.MODIFIED_NEWTON)


def test_static_smooth_rejects_levels_beyond_the_scratch_limit():
    """1024^2 FP64 level 0 needs 185 MB of scratch (> 64 MiB): PNS_EINVAL
    before the workspace, state or smoother are looked at."""
    L = pnsmg.lib()
    m = pnsmg.pns_mesh()
    m.dim = 2
    m.n_cells[0], m.n_cells[1], m.n_cells[2] = 1024, 1024, 1
    m.hi[0] = m.hi[1] = m.hi[2] = 1.0
    d = pnsmg.pns_discretization(2, 1, 0.0, 0.01)
    h = ctypes.c_void_p()
    assert L.pns_ctx_create(ctypes.byref(m), ctypes.byref(d), 1, pnsmg.FP64, None,
                            ctypes.byref(h)) == pnsmg.PNS_OK
    rc = L.pns_vanka_smooth_static(h, 0, 1, 0.5, ctypes.c_void_p(1024), ctypes.c_void_p(2048))
    assert rc == pnsmg.PNS_EINVAL
    assert b"static scratch" in L.pns_last_error(h)
    # a level that fits passes the size check and stops at the missing workspace
    m.n_cells[0], m.n_cells[1] = 64, 64
    h2 = ctypes.c_void_p()
    assert L.pns_ctx_create(ctypes.byref(m), ctypes.byref(d), 1, pnsmg.FP64, None,
                            ctypes.byref(h2)) == pnsmg.PNS_OK
    rc = L.pns_vanka_smooth_static(h2, 0, 1, 0.5, ctypes.c_void_p(1024), ctypes.c_void_p(2048))
    assert rc == pnsmg.PNS_EWORKSPACE
    L.pns_ctx_destroy(h)
    L.pns_ctx_destroy(h2)


# (cells of the first call, cells of the second, smaller, call, levels, CIP weight)
CASES = [
    ((48, 40), (16, 8), 2, pnsmg.FP64, 0.0),
    ((48, 40), (16, 8), 2, pnsmg.FP32, 0.0),
    ((48, 40), (16, 8), 2, pnsmg.FP64, 0.5),
    ((4, 4, 4), (2, 2, 2), 2, pnsmg.FP64, 0.0),
    ((4, 4, 4), (2, 2, 2), 2, pnsmg.FP32, 0.0),
]


@pytest.mark.gpu
@pytest.mark.parametrize("big,small,levels,prec,cip", CASES)
def test_static_smooth_equals_workspace_smooth(big, small, levels, prec, cip):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    tol = 1e-13 if prec == pnsmg.FP64 else 1e-5
    omega = 0.15 if len(big) == 3 else 0.3
    for call, n in enumerate((big, small)):
        print(f"static smooth: call {call}, mesh {n}, precision {prec}", flush=True)
        ctx = pnsmg.Context(n, n_levels=levels, precision=prec, tau=0.01)
        nv = ctx.sizes(0)["nv"]
        uk = inputs.uniform(500 + call, 2 * nv)
        ctx.pns_set_state(dict(MODEL, gamma_cip=cip),
                          torch.tensor(uk, dtype=torch.float64, device="cuda"))
        ctx.pns_vanka_setup()
        # the coarsest 3D level holds the dense inverse (no patches)
        lv_list = [0] if len(n) == 3 else list(range(levels))
        for lv in lv_list:
            nst = ctx.sizes(lv)["nst"]
            r = torch.tensor(inputs.uniform(510 + lv, nst), dtype=ctx.dtype, device="cuda")
            d0 = torch.tensor(inputs.uniform(520 + lv, nst), dtype=ctx.dtype, device="cuda")
            d_ws = d0.clone()
            d_st = d0.clone()
            ctx.pns_vanka_smooth(lv, 2, omega, r, d_ws)
            ctx.pns_vanka_smooth_static(lv, 2, omega, r, d_st)
            torch.cuda.synchronize()
            a = d_ws.double().cpu().numpy()
            b = d_st.double().cpu().numpy()
            assert np.all(np.isfinite(b))
            err = np.linalg.norm(a - b) / np.linalg.norm(a)
            print(f"  level {lv}: rel diff {err:.2e} (bound {tol:.0e})", flush=True)
            assert err <= tol
        del ctx
