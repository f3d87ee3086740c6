"""GPU parity of the CIP stabilisation (Sec. 3.2, eq. scip-def) through the
C-ABI: the Jacobian action with the CIP term (weight lagged at u_k) and the
FP64 residual with the CIP term (weight at the state) against the oracle, on
meshes with several 16 x 8 tiles and ragged tails, anisotropic cells and a
single cell (no interior face), every linearisation and both tangent modes,
action and defect; the multigrid operators with the face term (level-0
surrogate and exact patches, Galerkin coarse operators, the dense coarsest
operator, whole V-cycles) against the oracle's, which takes patches and
Galerkin products of the assembled operator with CIP; and a slab solve with
CIP reaching the oracle's Newton solution.  Tolerances as without CIP: FP64
action 1e-12, FP32 1e-5 relative per block; smoother and V-cycle FP64 bounds
from the conditioning of the matrices solved."""
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

MODEL = dict(p=1.4, delta=1e-3, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1, gamma_cip=0.7)
KINDS = [pnsmg.PICARD, pnsmg.EXACT_NEWTON, pnsmg.MODIFIED_NEWTON]


def oprob(n, model, lin, hi=(1.0, 1.0), tau=0.01):
    return O.Problem(n=tuple(n), hi=(hi[0], hi[1], 1.0), tau=tau, p=model["p"],
                     delta=model["delta"], nu=model["nu"], nu_inf=model["nu_inf"],
                     gamma1=model["gamma1"], gamma2=model["gamma2"],
                     sigma_max=model["sigma_max"], convection=model["convection"],
                     qsign=model["qsign"], lin=lin, gamma_cip=model["gamma_cip"])


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def blocks(prob):
    vel = np.concatenate([np.arange(m * prob.ns, m * prob.ns + prob.nv) for m in range(prob.nt)])
    pre = np.concatenate([np.arange(m * prob.ns + prob.nv, (m + 1) * prob.ns)
                          for m in range(prob.nt)])
    return vel, pre


def rel(got, ref, idx):
    return np.linalg.norm(got[idx] - ref[idx]) / np.linalg.norm(ref[idx])


@pytest.mark.parametrize("n,hi", [((37, 20), (1.0, 1.0)), ((16, 31), (2.0, 0.5)),
                                  ((1, 1), (1.0, 1.0)), ((2, 1), (1.0, 1.0)), ((9, 7), (1.0, 1.0))])
def test_apply_with_cip_matches_the_oracle(n, hi):
    for lin in KINDS:
        prob = oprob(n, MODEL, lin, hi=hi)
        uk = inputs.uniform(901, prob.nt * prob.nv)
        x = inputs.uniform(902, prob.nst)
        b = inputs.uniform(903, prob.nst)
        ref = O.apply(prob, uk, x)
        for prec, tol in ((pnsmg.FP64, 1e-12), (pnsmg.FP32, 1e-5)):
            for mode in (pnsmg.APPLY_RECOMPUTE, pnsmg.APPLY_CACHED):
                ctx = pnsmg.Context(n, n_levels=1, precision=prec, tau=0.01, hi=hi)
                ctx.pns_set_apply_mode(mode)
                ctx.pns_set_state(dict(MODEL, lin=lin), dev(uk))
                y = ctx.vector()
                ctx.pns_cell_apply(dev(x, ctx.dtype), y)
                yd = ctx.vector()
                ctx.pns_cell_defect(dev(b, ctx.dtype), dev(x, ctx.dtype), yd)
                torch.cuda.synchronize()
                got = y.double().cpu().numpy()
                bq = np.asarray(b, dtype=np.float32).astype(np.float64) if prec == pnsmg.FP32 else b
                gotd = yd.double().cpu().numpy()
                for idx in blocks(prob):
                    assert rel(got, ref, idx) <= tol, (n, lin, prec, mode, rel(got, ref, idx))
                    assert rel(gotd, bq - ref, idx) <= tol, (n, lin, prec, mode)
    # the CIP part is a visible part of the action on these inputs
    if n[0] * n[1] > 1:
        prob = oprob(n, MODEL, pnsmg.MODIFIED_NEWTON, hi=hi)
        a = O.apply(prob, uk, x)
        a0 = O.apply(prob.with_(gamma_cip=0.0), uk, x)
        assert np.linalg.norm(a - a0) > 1e-4 * np.linalg.norm(a)


@pytest.mark.parametrize("n", [(6, 5), (17, 9)])
def test_residual_with_cip_matches_the_oracle(n):
    prob = oprob(n, MODEL, pnsmg.MODIFIED_NEWTON)
    U = inputs.uniform(911, prob.nst)
    vprev = inputs.uniform(912, prob.nv)
    ref = O.residual(prob, U, vprev)
    ctx = pnsmg.Context(n, n_levels=1, precision=pnsmg.FP64, tau=0.01)
    R = torch.zeros(prob.nst, dtype=torch.float64, device="cuda")
    ctx.pns_residual(MODEL, dev(U), dev(vprev), R)
    torch.cuda.synchronize()
    got = R.cpu().numpy()
    for idx in blocks(prob):
        assert rel(got, ref, idx) <= 1e-12


def make_ctx(n, levels, model, uk, precision=pnsmg.FP64, masks=None,
             patch_kind=pnsmg.PATCH_SURROGATE):
    ctx = pnsmg.Context(n, n_levels=levels, precision=precision, tau=0.01)
    ctx.pns_set_state(dict(model, lin=pnsmg.MODIFIED_NEWTON), dev(uk))
    ctx.pns_set_patch_kind(patch_kind)
    ctx.pns_vanka_setup(None if masks is None else pnsmg.masks_to_bits(masks))
    return ctx


# nu = 0.2: the face term is of the size of the viscous one on these meshes
SMOOTH_MODEL = dict(MODEL, p=1.5, delta=1e-2, nu=0.2, nu_inf=1e-3, gamma_cip=1.0)


@pytest.mark.parametrize("kind,masked", [(pnsmg.PATCH_SURROGATE, False),
                                         (pnsmg.PATCH_SURROGATE, True),
                                         (pnsmg.PATCH_EXACT, True)])
def test_vanka_with_cip_matches_the_oracle(kind, masked):
    n = (10, 8)
    prob = oprob(n, SMOOTH_MODEL, pnsmg.MODIFIED_NEWTON)
    uk = inputs.sin_series_velocity(n, seed=931, t_nodes=[0.01 / 3, 0.01])
    masks = inputs.truncation_masks(n, seed=932) if masked else None
    r = inputs.uniform(933, prob.nst)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    patches = O.all_patches(prob, masks)
    src = O.assemble_surrogate(prob, uk) if kind == pnsmg.PATCH_SURROGATE else A
    pm = O.patch_matrices(src, patches)
    ref = O.vanka_step(A, pm, patches, r, np.zeros(prob.nst), 0.3)
    ref = O.vanka_step(A, pm, patches, r, ref, 0.3)
    # the face term is a visible part of the patches
    pm0 = O.patch_matrices((O.assemble_surrogate(prob.with_(gamma_cip=0.0), uk)
                            if kind == pnsmg.PATCH_SURROGATE else
                            O.assemble_slab(prob.with_(gamma_cip=0.0), O.split_uk(prob, uk))),
                           patches)
    assert max(np.abs(a - b).max() / np.abs(a).max() for a, b in zip(pm, pm0)) > 1e-3
    tol = fp64_tol(kappa_eq(pm))
    for prec in (pnsmg.FP64, pnsmg.FP32):
        ctx = make_ctx(n, 1, SMOOTH_MODEL, uk, precision=prec, masks=masks, patch_kind=kind)
        d = ctx.vector()
        ctx.pns_vanka_smooth(0, 2, 0.3, dev(r, ctx.dtype), d)
        got = d.double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"vanka with CIP kind={kind} masked={masked} prec={prec}: rel err {err:.2e}")
        assert err <= (tol if prec == pnsmg.FP64 else 1e-4)


def test_galerkin_levels_with_cip_match_the_oracle():
    n = (12, 8)
    prob = oprob(n, SMOOTH_MODEL, pnsmg.MODIFIED_NEWTON)
    uk = inputs.sin_series_velocity(n, seed=941, t_nodes=[0.01 / 3, 0.01])
    H = O.build_hierarchy(prob, uk, n_levels=3)
    ctx = make_ctx(n, 3, SMOOTH_MODEL, uk)
    for l in (1, 2):
        ol = 2 - l
        x = inputs.uniform(942 + l, H.probs[ol].nst)
        y = ctx.vector(l)
        ctx.pns_level_apply(l, dev(x), y)
        ref = H.A[ol] @ x
        err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
        # without the face term the coarse operator is visibly different
        Hc = O.build_hierarchy(prob.with_(gamma_cip=0.0), uk, n_levels=3)
        gap = np.linalg.norm(Hc.A[ol] @ x - ref) / np.linalg.norm(ref)
        print(f"galerkin level {l} with CIP: rel err {err:.2e} (face term {gap:.1e})")
        assert err <= 1e-12
        assert gap > 1e-4


@pytest.mark.parametrize("n,levels,kind", [((16, 16), 3, pnsmg.PATCH_SURROGATE),
                                           ((8, 12), 2, pnsmg.PATCH_SURROGATE),
                                           ((8, 8), 1, pnsmg.PATCH_SURROGATE),
                                           ((16, 16), 3, pnsmg.PATCH_EXACT)])
def test_vcycle_with_cip_matches_the_oracle(n, levels, kind):
    prob = oprob(n, SMOOTH_MODEL, pnsmg.MODIFIED_NEWTON)
    uk = inputs.sin_series_velocity(n, seed=951, t_nodes=[0.01 / 3, 0.01])
    r = inputs.uniform(952, prob.nst)
    H = O.build_hierarchy(prob, uk, n_levels=levels, surrogate=kind == pnsmg.PATCH_SURROGATE)
    ref = O.vcycle(H, r, nu1=2, nu2=2, omega=0.3)
    tol = fp64_tol(hierarchy_kappa(H))
    for prec in (pnsmg.FP64, pnsmg.FP32):
        ctx = make_ctx(n, levels, SMOOTH_MODEL, uk, precision=prec, patch_kind=kind)
        d = ctx.vector()
        ctx.pns_vcycle(2, 2, 0.3, dev(r, ctx.dtype), d)
        got = d.double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"vcycle with CIP n={n} levels={levels} kind={kind} prec={prec}: rel err {err:.2e} "
              f"(bound {tol:.1e})")
        assert err <= (tol if prec == pnsmg.FP64 else 1e-4)


def test_solve_with_cip_reaches_the_oracle_solution():
    n = (12, 12)
    # nu = 0.2: the CIP term moves the solution by 2 % here (far above the
    # tolerance) and is of the size of the viscous term, so a preconditioner
    # without it diverges; the weight of the residual is the state, the
    # Jacobian's is lagged, so Newton converges linearly (15 steps in the oracle)
    model = SMOOTH_MODEL
    prob = oprob(n, model, pnsmg.MODIFIED_NEWTON)
    vprev = inputs.sin_series_velocity(n, seed=921, t_nodes=[0.0])
    ref = O.newton_solve(prob, vprev, rtol=1e-13)
    for prec in (pnsmg.FP64, pnsmg.FP32):
        ctx = pnsmg.Context(n, n_levels=2, precision=prec, tau=0.01)
        U = dev(O.state_from_velocity(prob, np.concatenate([vprev, vprev])))
        rc, info = ctx.pns_solve(dict(model, lin=pnsmg.MODIFIED_NEWTON), dev(vprev), U,
                                 rtol=1e-10, omega=0.2, max_newton=60)
        torch.cuda.synchronize()
        print(f"solve with CIP prec {prec}: {info}")
        assert rc == pnsmg.PNS_OK
        Ug = U.cpu().numpy()
        assert O.mass_norm(prob, O.residual(prob, Ug, vprev)) <= 1.05e-10 * ref.residual_norms[0]
        vel = blocks(prob)[0]
        assert rel(Ug, ref.U, vel) <= 1e-6


def test_cip_on_hexahedra_is_refused():
    ctx = pnsmg.Context((2, 2, 2), n_levels=1, precision=pnsmg.FP64)
    uk = torch.zeros(2 * ctx.sizes()["nv"], dtype=torch.float64, device="cuda")
    with pytest.raises(pnsmg.PnsError) as e:
        ctx.pns_set_state(dict(MODEL, lin=pnsmg.MODIFIED_NEWTON), uk)
    assert e.value.code == pnsmg.PNS_EUNSUPPORTED


def test_cip_makes_the_convection_dominated_solve_converge():
    """The regime in which additive cell-patch Vanka fails without
    stabilisation (p = 1.2, delta = 1e-4, nu = 1e-2, 128^2: cell Peclet ~ 10 in
    the high-strain regions): with CIP (gamma 1) in the operator and in the
    preconditioner the modified-Newton / FGMRES solve reaches 1e-8 (about 20
    Newton steps); without it the first linear solve already fails."""
    n = 128
    vprev = inputs.sin_series_velocity((n, n), seed=201, t_nodes=[0.0])
    levels = 5
    out = {}
    for g in (0.0, 1.0):
        model = dict(p=1.2, delta=1e-4, nu=1e-2, nu_inf=1e-4, gamma1=40.0, gamma2=40.0,
                     sigma_max=1e-2, convection=1, qsign=1, gamma_cip=g,
                     lin=pnsmg.MODIFIED_NEWTON)
        ctx = pnsmg.Context((n, n), n_levels=levels, precision=pnsmg.FP64, tau=0.01,
                            patch_kind=pnsmg.PATCH_EXACT)
        sz = ctx.sizes(0)
        U0 = np.zeros(sz["nst"])
        U0[:sz["nv"]] = vprev
        U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
        U = dev(U0)
        rc, info = ctx.pns_solve(model, dev(vprev), U, rtol=1e-8, omega=0.2, max_newton=60,
                                 max_krylov=150, check=False)
        torch.cuda.synchronize()
        print(f"128^2 convection-dominated solve, gamma_cip {g}: rc {rc} {info}")
        out[g] = (rc, info)
        del ctx
    assert out[0.0][0] == pnsmg.PNS_ENOTCONV
    assert out[1.0][0] == pnsmg.PNS_OK
    assert out[1.0][1]["residual_final"] <= 1e-8 * out[1.0][1]["residual_initial"]
