"""Fixed summation order of the quadrilateral action, defect and residual
(pns_set_reproducible): repeated calls on the same inputs are bitwise equal,
and the results still agree with the oracle within the usual bounds (FP64
1e-12, FP32 1e-5 per velocity / pressure block); a whole slab solve repeated
in the same process gives bitwise the same iterate.  Meshes with several
16 x 8 tiles, ragged tails and boundary faces on every side; every
linearisation, both tangent modes, with Dirichlet data and CIP."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_28706_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

MODEL = dict(p=1.4, delta=1e-3, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1)
KINDS = [pnsmg.PICARD, pnsmg.EXACT_NEWTON, pnsmg.MODIFIED_NEWTON]


def oprob(n, model, lin, lifting=None):
    return O.Problem(n=tuple(n), tau=0.01, p=model["p"], delta=model["delta"], nu=model["nu"],
                     nu_inf=model["nu_inf"], gamma1=model["gamma1"], gamma2=model["gamma2"],
                     sigma_max=model["sigma_max"], convection=model["convection"],
                     qsign=model["qsign"], lin=lin, gamma_cip=model.get("gamma_cip", 0.0),
                     lifting=lifting)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def blocks(prob):
    vel = np.concatenate([np.arange(m * prob.ns, m * prob.ns + prob.nv) for m in range(prob.nt)])
    pre = np.concatenate([np.arange(m * prob.ns + prob.nv, (m + 1) * prob.ns)
                          for m in range(prob.nt)])
    return vel, pre


def rel(got, ref, idx):
    return np.linalg.norm(got[idx] - ref[idx]) / np.linalg.norm(ref[idx])


@pytest.mark.parametrize("n", [(37, 20), (16, 9)])
def test_ordered_action_is_bitwise_repeatable_and_matches_the_oracle(n):
    nv = 2 * (2 * n[0] + 1) * (2 * n[1] + 1)
    lift = inputs.uniform(1101, 2 * nv)
    for lin in KINDS:
        prob = oprob(n, MODEL, lin, lift)
        uk = inputs.uniform(1102, prob.nt * prob.nv)
        x = inputs.uniform(1103, prob.nst)
        b = inputs.uniform(1104, prob.nst)
        ref = O.apply(prob, uk, x)
        for prec, tol in ((pnsmg.FP64, 1e-12), (pnsmg.FP32, 1e-5)):
            for mode in (pnsmg.APPLY_RECOMPUTE, pnsmg.APPLY_CACHED):
                ctx = pnsmg.Context(n, n_levels=1, precision=prec, tau=0.01)
                ctx.pns_set_apply_mode(mode)
                ctx.pns_set_reproducible(1)
                L = dev(lift)
                ctx.pns_set_dirichlet(L)
                ctx.pns_set_state(dict(MODEL, lin=lin), dev(uk))
                xd, bd = dev(x, ctx.dtype), dev(b, ctx.dtype)
                outs, defs = [], []
                for _ in range(8):
                    y = ctx.vector()
                    ctx.pns_cell_apply(xd, y)
                    yd = ctx.vector()
                    ctx.pns_cell_defect(bd, xd, yd)
                    outs.append(y)
                    defs.append(yd)
                torch.cuda.synchronize()
                for y in outs[1:]:
                    assert torch.equal(y, outs[0]), (n, lin, prec, mode)
                for yd in defs[1:]:
                    assert torch.equal(yd, defs[0]), (n, lin, prec, mode)
                got = outs[0].double().cpu().numpy()
                for idx in blocks(prob):
                    assert rel(got, ref, idx) <= tol, (n, lin, prec, mode, rel(got, ref, idx))


@pytest.mark.parametrize("cip", [0.0, 0.5])
def test_ordered_residual_is_bitwise_repeatable_and_matches_the_oracle(cip):
    n = (33, 17)
    model = dict(MODEL, gamma_cip=cip)
    nv = 2 * (2 * n[0] + 1) * (2 * n[1] + 1)
    lift = inputs.uniform(1111, 2 * nv)
    prob = oprob(n, model, pnsmg.MODIFIED_NEWTON, lift)
    U = inputs.uniform(1112, prob.nst)
    vprev = inputs.uniform(1113, prob.nv)
    ref = O.residual(prob, U, vprev)
    ctx = pnsmg.Context(n, n_levels=1, precision=pnsmg.FP64, tau=0.01)
    ctx.pns_set_reproducible(1)
    L = dev(lift)
    ctx.pns_set_dirichlet(L)
    Ud, vd = dev(U), dev(vprev)
    outs = []
    for _ in range(8):
        R = torch.zeros(prob.nst, dtype=torch.float64, device="cuda")
        ctx.pns_residual(model, Ud, vd, R)
        outs.append(R)
    torch.cuda.synchronize()
    for R in outs[1:]:
        assert torch.equal(R, outs[0])
    got = outs[0].cpu().numpy()
    for idx in blocks(prob):
        assert rel(got, ref, idx) <= 1e-12


@pytest.mark.parametrize("precision", [pnsmg.FP64, pnsmg.FP32])
def test_ordered_solve_is_bitwise_repeatable(precision):
    n = (16, 16)
    model = dict(MODEL, p=1.5, delta=1e-2, lin=pnsmg.MODIFIED_NEWTON)
    vprev = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.0])
    results = []
    for _ in range(2):
        ctx = pnsmg.Context(n, n_levels=3, precision=precision, tau=0.01)
        ctx.pns_set_reproducible(1)
        sz = ctx.sizes(0)
        U0 = np.zeros(sz["nst"])
        U0[:sz["nv"]] = vprev
        U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
        U = dev(U0)
        rc, info = ctx.pns_solve(model, dev(vprev), U, rtol=1e-10)
        torch.cuda.synchronize()
        print(f"ordered solve prec {precision}: rc {rc} {info}")
        assert rc == pnsmg.PNS_OK
        results.append((U.clone(), info))
        del ctx
    assert torch.equal(results[0][0], results[1][0])
    assert results[0][1] == results[1][1]


def test_reproducible_flag_rejects_other_values():
    ctx = pnsmg.Context((4, 4), n_levels=1, precision=pnsmg.FP64)
    with pytest.raises(pnsmg.PnsError) as e:
        ctx.pns_set_reproducible(2)
    assert e.value.code == pnsmg.PNS_EINVAL
