"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances: FP64 apply <= 1e-12 relative (2-norm, velocity and pressure rows
separately); FP32 apply <= 1e-5 relative.  Smoother, transfers and V-cycle
are linear maps evaluated with different rounding order on both sides; their
FP64 tolerance is derived per test from the conditioning of the patch and
coarse matrices solved: max(1e-12, kappa_eq * 1e-16) with kappa_eq the largest
condition number of those matrices after row and column equilibration
(tests/tolerances.py).  On the parity workloads kappa_eq stays below 1e4, so
the bound is 1e-12; the benchmark model (p = 1.2, delta = 1e-4) reaches
kappa_eq ~ 1e5.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_28706_amd import inputs
from tolerances import fp64_tol, hierarchy_kappa, kappa_eq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

CONFIG1 = dict(p=1.5, delta=1e-2, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
               convection=1, qsign=1)
KINDS = [pnsmg.PICARD, pnsmg.EXACT_NEWTON, pnsmg.MODIFIED_NEWTON]


def oracle_problem(n, model, lin, tau=0.01, hi=(1.0, 1.0)):
    return O.Problem(n=tuple(n), hi=(hi[0], hi[1], 1.0), tau=tau, p=model["p"],
                     delta=model["delta"], nu=model["nu"], nu_inf=model["nu_inf"],
                     gamma1=model["gamma1"], gamma2=model["gamma2"],
                     sigma_max=model["sigma_max"], convection=model["convection"],
                     qsign=model["qsign"], lin=lin)


def to_dev(a, dtype):
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def rel_blocks(got, ref, prob):
    """relative 2-norm errors of the velocity rows and of the pressure rows"""
    vel = np.concatenate([np.arange(m * prob.ns, m * prob.ns + prob.nv) for m in range(prob.nt)])
    pre = np.concatenate([np.arange(m * prob.ns + prob.nv, (m + 1) * prob.ns)
                          for m in range(prob.nt)])
    out = []
    for idx in (vel, pre):
        out.append(np.linalg.norm(got[idx] - ref[idx]) / np.linalg.norm(ref[idx]))
    return out


MODES = [pnsmg.APPLY_CACHED, pnsmg.APPLY_RECOMPUTE]


def gpu_apply(n, model, lin, uk, x, precision, tau=0.01, hi=(1.0, 1.0), defect_b=None,
              mode=pnsmg.APPLY_CACHED):
    ctx = pnsmg.Context(n, n_levels=1, precision=precision, tau=tau, hi=hi)
    dt = ctx.dtype
    ctx.pns_set_apply_mode(mode)
    ctx.pns_set_state(dict(model, lin=lin), to_dev(uk, torch.float64))
    xd = to_dev(x, dt)
    y = ctx.vector()
    if defect_b is None:
        ctx.pns_cell_apply(xd, y)
    else:
        ctx.pns_cell_defect(to_dev(defect_b, dt), xd, y)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("lin", KINDS)
def test_config1_apply_fp64(lin, mode):
    n = (8, 8)
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(101, prob.nt * prob.nv)
    x = inputs.uniform(102, prob.nst)
    ref = O.apply(prob, uk, x)
    got = gpu_apply(n, CONFIG1, lin, uk, x, pnsmg.FP64, mode=mode)
    ev, ep = rel_blocks(got, ref, prob)
    print(f"config1 lin={lin} mode={mode} fp64 rel err vel={ev:.2e} pres={ep:.2e}")
    assert ev <= 1e-12 and ep <= 1e-12


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("lin", KINDS)
def test_config1_apply_fp32(lin, mode):
    n = (8, 8)
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(101, prob.nt * prob.nv)
    x = inputs.uniform(102, prob.nst)
    ref = O.apply(prob, uk, x)
    got = gpu_apply(n, CONFIG1, lin, uk, x, pnsmg.FP32, mode=mode)
    ev, ep = rel_blocks(got, ref, prob)
    print(f"config1 lin={lin} mode={mode} fp32 rel err vel={ev:.2e} pres={ep:.2e}")
    assert ev <= 1e-5 and ep <= 1e-5


@pytest.mark.parametrize("n,hi", [((37, 20), (1.0, 1.0)), ((16, 31), (2.0, 0.5)), ((1, 1), (1.0, 1.0)),
                                  ((15, 15), (1.0, 1.0)), ((46, 3), (1.0, 1.0))])
def test_apply_ragged_tiles_fp64(n, hi):
    """Meshes spanning several 15x15 tiles with ragged tails, anisotropic cells,
    the single-cell mesh and exactly one tile."""
    model = dict(CONFIG1, p=1.3, delta=1e-3, nu_inf=1e-4)
    for lin in KINDS:
        prob = oracle_problem(n, model, lin, hi=hi)
        uk = inputs.uniform(7, prob.nt * prob.nv)
        x = inputs.uniform(8, prob.nst)
        ref = O.apply(prob, uk, x)
        for mode in MODES:
            got = gpu_apply(n, model, lin, uk, x, pnsmg.FP64, hi=hi, mode=mode)
            ev, ep = rel_blocks(got, ref, prob)
            assert ev <= 1e-12 and ep <= 1e-12, (n, lin, mode, ev, ep)


def test_apply_variants_fp64():
    """p-Stokes (no convection), literal pressure sign, Newtonian p = 2,
    sigma_max = 0 and huge, nu_inf = 0."""
    n = (9, 7)
    variants = [dict(convection=0), dict(qsign=-1), dict(p=2.0), dict(sigma_max=0.0),
                dict(sigma_max=1e300), dict(nu_inf=0.0, p=1.1, delta=1e-5),
                dict(p=1.05, delta=1e-9, amp=1e-6), dict(p=1.9, delta=0.5, amp=30.0)]
    for v in variants:
        amp = v.pop("amp", 1.0)
        model = dict(CONFIG1, **v)
        for lin in KINDS:
            prob = oracle_problem(n, model, lin)
            uk = amp * inputs.uniform(11, prob.nt * prob.nv)
            x = inputs.uniform(12, prob.nst)
            ref = O.apply(prob, uk, x)
            for mode in MODES:
                got = gpu_apply(n, model, lin, uk, x, pnsmg.FP64, mode=mode)
                ev, ep = rel_blocks(got, ref, prob)
                assert ev <= 1e-12 and ep <= 1e-12, (v, lin, mode, ev, ep)


def test_defect_mode_fp64():
    n = (12, 10)
    prob = oracle_problem(n, CONFIG1, pnsmg.MODIFIED_NEWTON)
    uk = inputs.uniform(21, prob.nt * prob.nv)
    x = inputs.uniform(22, prob.nst)
    b = inputs.uniform(23, prob.nst)
    ref = b - O.apply(prob, uk, x)
    got = gpu_apply(n, CONFIG1, pnsmg.MODIFIED_NEWTON, uk, x, pnsmg.FP64, defect_b=b)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_zero_state_and_zero_input():
    n = (6, 6)
    prob = oracle_problem(n, CONFIG1, pnsmg.EXACT_NEWTON)
    uk = np.zeros(prob.nt * prob.nv)
    x = np.zeros(prob.nst)
    got = gpu_apply(n, CONFIG1, pnsmg.EXACT_NEWTON, uk, x, pnsmg.FP64)
    assert np.all(got == 0.0)
    x = inputs.uniform(5, prob.nst)
    ref = O.apply(prob, uk, x)
    got = gpu_apply(n, CONFIG1, pnsmg.EXACT_NEWTON, uk, x, pnsmg.FP64)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_full_size_apply_sampled_rows():
    """256 x 256 (the apply benchmark size) with the sin-series state: sampled
    rows (corners, edges, tile seams, interior, pressure) against the oracle."""
    n = (256, 256)
    model = dict(p=1.2, delta=1e-4, nu=1.0, nu_inf=1e-4, gamma1=40.0, gamma2=40.0,
                 sigma_max=1.0, convection=1, qsign=1)
    prob = oracle_problem(n, model, pnsmg.MODIFIED_NEWTON)
    uk = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    x = inputs.uniform(202, prob.nst)
    for prec, tol, mode in ((pnsmg.FP64, 1e-12, pnsmg.APPLY_CACHED),
                            (pnsmg.FP64, 1e-12, pnsmg.APPLY_RECOMPUTE),
                            (pnsmg.FP32, 1e-5, pnsmg.APPLY_CACHED)):
        got = gpu_apply(n, model, pnsmg.MODIFIED_NEWTON, uk, x, prec, mode=mode)
        rng = np.random.default_rng(0)
        NX = 2 * n[0] + 1
        special_nodes = [0, NX - 1, NX * NX - 1, 30, 29, 31, 30 * NX + 30, 60 * NX + 61,
                         (NX // 2) * NX + NX // 2, 2 * NX + 500]
        rows = []
        for mu in range(2):
            for comp in range(2):
                rows += [mu * prob.ns + comp * prob.num_nodes + s for s in special_nodes]
            rows += list(mu * prob.ns + prob.nv + np.array([0, 1, 2, 3 * 255, 3 * 65535 + 2]))
        rows += list(rng.integers(0, prob.nst, 200))
        rows = np.array(sorted(set(int(r) for r in rows)))
        ref = O.apply_rows(prob, uk, x, rows)
        err = np.abs(got[rows] - ref)
        scale = np.abs(ref).max()
        print(f"256^2 sampled rows prec={prec}: max abs err {err.max():.3e} / max |y| {scale:.3e}")
        assert err.max() <= tol * scale


# ------------------------------------------------------------------ smoother

def make_ctx(n, levels, model, lin, uk, precision=pnsmg.FP64, masks=None,
             patch_kind=pnsmg.PATCH_SURROGATE):
    ctx = pnsmg.Context(n, n_levels=levels, precision=precision, tau=0.01)
    ctx.pns_set_state(dict(model, lin=lin), to_dev(uk, torch.float64))
    ctx.pns_set_patch_kind(patch_kind)
    ctx.pns_vanka_setup(None if masks is None else pnsmg.masks_to_bits(masks))
    return ctx


@pytest.mark.parametrize("lin", KINDS)
def test_config1_vanka_sweep_fp64(lin):
    n = (8, 8)
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(101, prob.nt * prob.nv)
    r = inputs.uniform(103, prob.nst)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    patches = O.all_patches(prob)
    pm = O.patch_matrices(O.assemble_surrogate(prob, uk), patches)
    ref = O.vanka_step(A, pm, patches, r, np.zeros(prob.nst), 0.5)
    tol = fp64_tol(kappa_eq(pm))
    ctx = make_ctx(n, 1, CONFIG1, lin, uk)
    d = ctx.vector()
    ctx.pns_vanka_smooth(0, 1, 0.5, to_dev(r, torch.float64), d)
    got = d.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"config1 vanka lin={lin}: rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol
    # a second sweep (exercises the defect path)
    ref2 = O.vanka_step(A, pm, patches, r, ref, 0.5)
    ctx.pns_vanka_smooth(0, 1, 0.5, to_dev(r, torch.float64), d)
    got2 = d.cpu().numpy()
    assert np.linalg.norm(got2 - ref2) <= tol * np.linalg.norm(ref2)


def test_vanka_sweep_fp32():
    n = (8, 8)
    lin = pnsmg.MODIFIED_NEWTON
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(101, prob.nt * prob.nv)
    r = inputs.uniform(103, prob.nst)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    patches = O.all_patches(prob)
    pm = O.patch_matrices(O.assemble_surrogate(prob, uk), patches)
    ref = O.vanka_step(A, pm, patches, r, np.zeros(prob.nst), 0.5)
    ref = O.vanka_step(A, pm, patches, r, ref, 0.5)
    ctx = make_ctx(n, 1, CONFIG1, lin, uk, precision=pnsmg.FP32)
    d = ctx.vector()
    ctx.pns_vanka_smooth(0, 2, 0.5, to_dev(r, torch.float32), d)
    got = d.double().cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"vanka fp32 rel err {err:.2e}")
    assert err <= 1e-4


def test_truncated_patches_fp64():
    n = (10, 8)
    lin = pnsmg.MODIFIED_NEWTON
    model = dict(CONFIG1, p=1.1, delta=1e-5, nu_inf=1e-4)
    prob = oracle_problem(n, model, lin)
    uk = inputs.sin_series_velocity(n, seed=401, t_nodes=[0.01 / 3, 0.01])
    masks = inputs.truncation_masks(n, seed=402)
    r = inputs.uniform(403, prob.nst)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    patches = O.all_patches(prob, masks)
    assert len({len(p) for p in patches}) > 1
    pm = O.patch_matrices(O.assemble_surrogate(prob, uk), patches)
    ref = O.vanka_step(A, pm, patches, r, np.zeros(prob.nst), 0.5)
    tol = fp64_tol(kappa_eq(pm))
    ctx = make_ctx(n, 1, model, lin, uk, masks=masks)
    d = ctx.vector()
    ctx.pns_vanka_smooth(0, 1, 0.5, to_dev(r, torch.float64), d)
    got = d.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"truncated patches rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol


def test_transfers_and_galerkin_operator():
    n = (12, 8)
    lin = pnsmg.EXACT_NEWTON
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(31, prob.nt * prob.nv)
    H = O.build_hierarchy(prob, uk, n_levels=3)
    ctx = make_ctx(n, 3, CONFIG1, lin, uk)
    for l in range(2):                    # ctx level l = oracle level 2 - l
        ol = 2 - l
        rf = inputs.uniform(40 + l, H.probs[ol].nst)
        dc = inputs.uniform(50 + l, H.probs[ol - 1].nst)
        rc = ctx.vector(l + 1)
        ctx.pns_restrict(l, to_dev(rf, torch.float64), rc)
        ref_rc = H.P[ol - 1].T @ rf
        assert np.abs(rc.cpu().numpy() - ref_rc).max() <= 1e-13 * np.abs(ref_rc).max()
        df = to_dev(rf, torch.float64)
        ctx.pns_prolongate_add(l, to_dev(dc, torch.float64), df)
        ref_df = rf + H.P[ol - 1] @ dc
        assert np.abs(df.cpu().numpy() - ref_df).max() <= 1e-13 * np.abs(ref_df).max()
    for l in (1, 2):
        ol = 2 - l
        x = inputs.uniform(60 + l, H.probs[ol].nst)
        y = ctx.vector(l)
        ctx.pns_level_apply(l, to_dev(x, torch.float64), y)
        ref = H.A[ol] @ x
        err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"galerkin level {l}: rel err {err:.2e}")
        assert err <= 1e-12


@pytest.mark.parametrize("n,levels,lin", [((16, 16), 3, pnsmg.MODIFIED_NEWTON),
                                          ((8, 12), 2, pnsmg.PICARD),
                                          ((8, 8), 1, pnsmg.EXACT_NEWTON),
                                          ((16, 16), 1, pnsmg.MODIFIED_NEWTON),
                                          ((32, 32), 2, pnsmg.MODIFIED_NEWTON)])
def test_vcycle_fp64(n, levels, lin):
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(71, prob.nt * prob.nv)
    r = inputs.uniform(72, prob.nst)
    H = O.build_hierarchy(prob, uk, n_levels=levels)
    ref = O.vcycle(H, r, nu1=2, nu2=2, omega=0.5)
    tol = fp64_tol(hierarchy_kappa(H))
    ctx = make_ctx(n, levels, CONFIG1, lin, uk)
    d = ctx.vector()
    ctx.pns_vcycle(2, 2, 0.5, to_dev(r, torch.float64), d)
    got = d.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"vcycle n={n} levels={levels} lin={lin}: rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol


def test_vcycle_fp32_close_to_fp64():
    n = (16, 16)
    lin = pnsmg.MODIFIED_NEWTON
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(81, prob.nt * prob.nv)
    r = inputs.uniform(82, prob.nst)
    H = O.build_hierarchy(prob, uk, n_levels=3)
    ref = O.vcycle(H, r, nu1=2, nu2=2, omega=0.5)
    ctx = make_ctx(n, 3, CONFIG1, lin, uk, precision=pnsmg.FP32)
    d = ctx.vector()
    ctx.pns_vcycle(2, 2, 0.5, to_dev(r, torch.float32), d)
    got = d.double().cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"vcycle fp32 rel err {err:.2e}")
    assert err <= 1e-4


@pytest.mark.parametrize("masked", [False, True])
def test_exact_fine_patches_vanka_fp64(masked):
    # exact patch matrices R_K A R_K^T on the finest level (both Radau nodes
    # with their own coefficients) against the oracle's patches of the
    # assembled slab operator
    n = (10, 8)
    lin = pnsmg.MODIFIED_NEWTON
    model = dict(CONFIG1, p=1.2, delta=1e-4, nu_inf=1e-4)
    prob = oracle_problem(n, model, lin)
    uk = inputs.sin_series_velocity(n, seed=411, t_nodes=[0.01 / 3, 0.01])
    masks = inputs.truncation_masks(n, seed=412) if masked else None
    r = inputs.uniform(413, prob.nst)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    patches = O.all_patches(prob, masks)
    pm = O.patch_matrices(A, patches)
    ref = O.vanka_step(A, pm, patches, r, np.zeros(prob.nst), 0.3)
    ref = O.vanka_step(A, pm, patches, r, ref, 0.3)
    tol = fp64_tol(kappa_eq(pm))
    ctx = make_ctx(n, 1, model, lin, uk, masks=masks, patch_kind=pnsmg.PATCH_EXACT)
    d = ctx.vector()
    ctx.pns_vanka_smooth(0, 2, 0.3, to_dev(r, torch.float64), d)
    got = d.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"exact fine patches masked={masked}: rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol


def test_exact_fine_patches_vcycle_fp64_and_fp32():
    n = (16, 16)
    lin = pnsmg.MODIFIED_NEWTON
    prob = oracle_problem(n, CONFIG1, lin)
    uk = inputs.uniform(91, prob.nt * prob.nv)
    r = inputs.uniform(92, prob.nst)
    H = O.build_hierarchy(prob, uk, n_levels=3, surrogate=False)
    ref = O.vcycle(H, r, nu1=2, nu2=2, omega=0.3)
    for precision, tol in ((pnsmg.FP64, fp64_tol(hierarchy_kappa(H))), (pnsmg.FP32, 1e-4)):
        ctx = make_ctx(n, 3, CONFIG1, lin, uk, precision=precision, patch_kind=pnsmg.PATCH_EXACT)
        d = ctx.vector()
        rr = to_dev(r, ctx.dtype)
        ctx.pns_vcycle(2, 2, 0.3, rr, d)
        got = d.double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"vcycle exact fine patches prec={precision}: rel err {err:.2e}")
        assert err <= tol


# ----------------------------------------------- the benchmarked V-cycle shape

BENCH_MODEL = dict(CONFIG1, p=1.2, delta=1e-4, nu_inf=1e-4)


@pytest.mark.parametrize("n,precisions", [((64, 64), (pnsmg.FP64, pnsmg.FP32)),
                                          ((128, 128), (pnsmg.FP64,))])
def test_vcycle_benchmark_model_four_levels(n, precisions):
    """The V-cycle as benchmarked at 256^2: four levels (here 64^2 -> 8^2 and
    128^2 -> 16^2), surrogate finest patches, 2 + 2 steps, omega = 0.1, the
    modified-Newton tangent at p = 1.2, delta = 1e-4, nu_inf = 1e-4 and the
    sin-series state of the 256^2 workload (seed 201), against the oracle's
    V-cycle (sparse Galerkin triple products, dense LU patch solves, dense LU
    coarsest solve).  FP64 bound from the conditioning (kappa_eq ~ 1e5 here);
    FP32 (coarsest solve in FP64) within kappa_eq times the FP32 unit
    roundoff."""
    lin = pnsmg.MODIFIED_NEWTON
    prob = oracle_problem(n, BENCH_MODEL, lin)
    uk = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    r = inputs.uniform(203, prob.nst)
    H = O.build_hierarchy(prob, uk, n_levels=4)
    ref = O.vcycle(H, r, nu1=2, nu2=2, omega=0.1)
    kappa = hierarchy_kappa(H)
    for precision in precisions:
        tol = fp64_tol(kappa) if precision == pnsmg.FP64 else max(1e-4, kappa * 2.0 ** -24)
        ctx = make_ctx(n, 4, BENCH_MODEL, lin, uk, precision=precision)
        d = ctx.vector()
        ctx.pns_vcycle(2, 2, 0.1, to_dev(r, ctx.dtype), d)
        got = d.double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"benchmark-model V-cycle n={n} prec={precision}: rel err {err:.2e} "
              f"(kappa_eq {kappa:.1e}, bound {tol:.1e})")
        assert err <= tol
        del ctx
