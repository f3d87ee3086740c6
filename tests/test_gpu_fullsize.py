"""GPU checks at the full sizes of the benchmarked configurations, in the
launch configuration bench.py times, on outputs the oracle can form one by
one or on properties that hold at any size.

* Batched Vanka, 512 x 512, boundary-truncated surrogate patches (p = 1.1,
  delta = 1e-5), FP32 as benchmarked and FP64: the right-hand side is nonzero
  only on unknowns that belong to a single patch (the centre node's
  velocities and the pressure coefficients of sampled cells at least two
  cells apart), so one additive step from d = 0 gives d = omega A_K^{-1} R_K r
  on each sampled patch and exact zeros elsewhere.  Each patch matrix is
  formed by the oracle from the neighbouring element matrices.  FP64: forward
  error within 1e-12 or the patch's condition bound; FP32: backward error
  ||A_K delta - r_K|| <= 4 n u ||A_K|| ||delta|| (the patches reach
  condition numbers ~1e6, where an FP32 forward bound says nothing).
* V-cycle, 256 x 256, 4 levels, as benchmarked: V is linear and V(0) = 0.
* Slab solve, 256 x 256 to 1e-8 as benchmarked: the oracle's residual of the
  returned iterate meets the stopping test, in FP64 and mixed precision.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_28706_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

BASE = dict(nu=1.0, gamma1=40.0, gamma2=40.0, sigma_max=1.0, convection=1, qsign=1,
            lin=pnsmg.MODIFIED_NEWTON)
VANKA_MODEL = dict(BASE, p=1.1, delta=1e-5, nu_inf=1e-4)
VCYCLE_MODEL = dict(BASE, p=1.2, delta=1e-4, nu_inf=1e-4)
SOLVE_MODEL = dict(BASE, p=1.8, delta=1e-2, nu=0.1, nu_inf=1e-4)
OMEGA = 0.1

# sampled cells of the 512^2 mesh: corners, edges, interior; pairwise at least
# two cells apart in x or y, so that their patches share no unknown
SAMPLED = [(0, 0), (511, 0), (0, 511), (511, 511), (0, 255), (255, 0), (511, 300), (300, 511),
           (128, 128), (256, 257), (400, 100), (5, 7), (2, 0), (509, 511), (1, 300)]


def exclusive_dofs(prob, cx, cy):
    """unknowns of cell (cx, cy) that no other patch contains: the centre
    node's velocities and the cell's pressure coefficients, both Radau nodes"""
    NX = 2 * prob.n[0] + 1
    centre = (2 * cy + 1) * NX + 2 * cx + 1
    cell = cy * prob.n[0] + cx
    out = []
    for mu in range(prob.nt):
        base = mu * prob.ns
        out += [base + c * prob.num_nodes + centre for c in range(2)]
        out += [base + prob.nv + 3 * cell + j for j in range(3)]
    return out


@pytest.mark.parametrize("precision", [pnsmg.FP32, pnsmg.FP64])
def test_batched_vanka_512_isolated_patches(precision):
    n = (512, 512)
    for i, a in enumerate(SAMPLED):
        for b in SAMPLED[i + 1:]:
            assert abs(a[0] - b[0]) >= 2 or abs(a[1] - b[1]) >= 2
    prob = O.Problem(n=n, tau=0.01, p=VANKA_MODEL["p"], delta=VANKA_MODEL["delta"],
                     nu=VANKA_MODEL["nu"], nu_inf=VANKA_MODEL["nu_inf"], lin=O.MODIFIED_NEWTON)
    uk = inputs.sin_series_velocity(n, seed=401, t_nodes=[0.01 / 3, 0.01])
    masks = inputs.truncation_masks(n, seed=402)
    ctx = pnsmg.Context(n, n_levels=1, precision=precision)
    ctx.pns_set_patch_kind(pnsmg.PATCH_SURROGATE)
    ctx.pns_set_state(VANKA_MODEL, torch.tensor(uk, device="cuda"))
    ctx.pns_vanka_setup(pnsmg.masks_to_bits(masks))
    vals = inputs.uniform(403, prob.nst)
    r = np.zeros(prob.nst)
    for cx, cy in SAMPLED:
        idx = exclusive_dofs(prob, cx, cy)
        r[idx] = vals[idx]
    rd = torch.tensor(r, dtype=ctx.dtype, device="cuda")
    d = ctx.vector()
    ctx.pns_vanka_smooth(0, 1, OMEGA, rd, d)
    torch.cuda.synchronize()
    dg = d.double().cpu().numpy()
    r_used = rd.double().cpu().numpy()   # the right-hand side as the GPU holds it
    ur = O.representative_velocity(prob, uk)
    covered = np.zeros(prob.nst, dtype=bool)
    u = 2.0 ** -53 if precision == pnsmg.FP64 else 2.0 ** -24
    for cx, cy in SAMPLED:
        cell = cy * n[0] + cx
        AK, idx = O.local_patch_matrix(prob, [ur, ur], cell, masks[cell])
        covered[idx] = True
        delta = dg[idx] / OMEGA
        rK = r_used[idx]
        nK = idx.size
        back = np.linalg.norm(AK @ delta - rK)
        bound = 4 * nK * u * np.linalg.norm(AK, 2) * np.linalg.norm(delta)
        z = np.linalg.solve(AK, rK)
        kappa = np.linalg.cond(AK)
        fwd = np.linalg.norm(delta - z) / np.linalg.norm(z)
        print(f"cell {(cx, cy)} n_K={nK} kappa={kappa:.1e}: backward {back:.2e} "
              f"(bound {bound:.2e}), forward {fwd:.2e}")
        assert back <= bound, (cx, cy, back, bound)
        if precision == pnsmg.FP64:
            assert fwd <= max(1e-12, 4 * nK * u * kappa), (cx, cy, fwd, kappa)
    assert np.all(dg[~covered] == 0.0)


def test_vcycle_256_is_linear():
    n = (256, 256)
    uk = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    for precision, tol in ((pnsmg.FP64, 1e-12), (pnsmg.FP32, 1e-5)):
        ctx = pnsmg.Context(n, n_levels=4, precision=precision)
        ctx.pns_set_state(VCYCLE_MODEL, torch.tensor(uk, device="cuda"))
        ctx.pns_vanka_setup(None)
        nst = ctx.sizes()["nst"]
        r1 = torch.tensor(inputs.uniform(203, nst), dtype=ctx.dtype, device="cuda")
        r2 = torch.tensor(inputs.uniform(204, nst), dtype=ctx.dtype, device="cuda")
        outs = []
        for r in (r1, r2, 2 * r1 - 3 * r2, torch.zeros_like(r1)):
            d = ctx.vector()
            ctx.pns_vcycle(2, 2, OMEGA, r, d)
            outs.append(d.double())
        torch.cuda.synchronize()
        comb = 2 * outs[0] - 3 * outs[1]
        err = float(torch.linalg.norm(outs[2] - comb) / torch.linalg.norm(comb))
        print(f"256^2 V-cycle prec={precision}: linearity {err:.2e}")
        assert err <= tol
        assert bool(torch.all(outs[3] == 0))


@pytest.mark.parametrize("precision", [pnsmg.FP64, pnsmg.FP32])
def test_solve_256_reaches_the_oracle_residual(precision):
    n = (256, 256)
    vprev = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.0])
    ctx = pnsmg.Context(n, n_levels=6, precision=precision)
    sz = ctx.sizes()
    U0 = np.zeros(sz["nst"])
    U0[:sz["nv"]] = vprev
    U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
    U = torch.tensor(U0, device="cuda")
    rc, info = ctx.pns_solve(SOLVE_MODEL, torch.tensor(vprev, device="cuda"), U)
    torch.cuda.synchronize()
    assert rc == pnsmg.PNS_OK, info
    prob = O.Problem(n=n, p=SOLVE_MODEL["p"], delta=SOLVE_MODEL["delta"], nu=SOLVE_MODEL["nu"],
                     nu_inf=SOLVE_MODEL["nu_inf"], lin=O.MODIFIED_NEWTON)
    M = O.slab_mass(prob)
    r0 = O.mass_norm(prob, O.residual(prob, U0, vprev), M)
    r1 = O.mass_norm(prob, O.residual(prob, U.cpu().numpy(), vprev), M)
    print(f"256^2 solve prec={precision}: {info}, oracle ||R||_M {r1:.3e} / {r0:.3e}")
    assert r1 <= 1.05e-8 * r0
