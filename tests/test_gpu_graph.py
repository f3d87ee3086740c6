"""GPU tests of graph-replayed V-cycles (pns_set_vcycle_graph) through the
C-ABI: every replay is compared with the eager V-cycle on the same input,
with eager work and synchronisations of the program between the replays;
the graph is recaptured when omega changes and dropped when the state
changes.  The same arithmetic runs in both forms, only the summation order
inside the action's tiles (LDS atomics) differs: 1e-12 relative in FP64,
1e-6 in FP32."""
import numpy as np
import pytest

from paper_2603_28706_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

MODEL = dict(p=1.8, delta=1e-2, nu=0.1, nu_inf=1e-4, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1, lin=pnsmg.MODIFIED_NEWTON)


def make(n, levels, precision, seed=501):
    ctx = pnsmg.Context(n, n_levels=levels, precision=precision)
    uk = inputs.sin_series_velocity(n, seed=seed, t_nodes=[0.01 / 3, 0.01])
    ctx.pns_set_state(MODEL, torch.tensor(uk, device="cuda"))
    ctx.pns_vanka_setup(None)
    return ctx


def rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


@pytest.mark.parametrize("precision,tol", [(pnsmg.FP64, 1e-12), (pnsmg.FP32, 1e-6)])
def test_graph_replays_equal_eager_vcycles(precision, tol):
    n = (64, 64)
    ctx = make(n, 3, precision)
    dt = ctx.dtype
    rs = [torch.tensor(inputs.uniform(510 + i, ctx.sizes()["nst"]), dtype=dt, device="cuda")
          for i in range(3)]
    eager = []
    for r in rs:
        d = ctx.vector()
        ctx.pns_vcycle(2, 2, 0.1, r, d)
        eager.append(d.clone())
    ctx.pns_set_vcycle_graph(1)
    x = ctx.vector()
    y = ctx.vector()
    for rep in range(6):
        r = rs[rep % 3]
        d = ctx.vector()
        ctx.pns_vcycle(2, 2, 0.1, r, d)
        # the program's own eager work between the replays
        ctx.pns_cell_apply(r, y)
        x.copy_(y * 0.5)
        torch.cuda.synchronize()
        err = rel(d, eager[rep % 3])
        print(f"replay {rep}: rel diff {err:.2e}")
        assert err <= tol, (rep, err)
    # another omega: recaptured, equal to the eager V-cycle with that omega
    ctx.pns_set_vcycle_graph(0)
    d_e = ctx.vector()
    ctx.pns_vcycle(1, 1, 0.05, rs[0], d_e)
    ctx.pns_set_vcycle_graph(1)
    for _ in range(2):
        d_g = ctx.vector()
        ctx.pns_vcycle(1, 1, 0.05, rs[0], d_g)
        torch.cuda.synchronize()
        assert rel(d_g, d_e) <= tol


def test_graph_is_dropped_with_the_state():
    n = (32, 32)
    ctx = make(n, 3, pnsmg.FP64)
    r = torch.tensor(inputs.uniform(520, ctx.sizes()["nst"]), device="cuda")
    ctx.pns_set_vcycle_graph(1)
    d0 = ctx.vector()
    ctx.pns_vcycle(2, 2, 0.1, r, d0)
    # a new linearisation state and smoother: the next V-cycle is of the new operator
    uk = inputs.sin_series_velocity(n, seed=521, t_nodes=[0.01 / 3, 0.01])
    ctx.pns_set_state(dict(MODEL, p=1.6), torch.tensor(uk, device="cuda"))
    ctx.pns_vanka_setup(None)
    d1 = ctx.vector()
    ctx.pns_vcycle(2, 2, 0.1, r, d1)
    ctx.pns_set_vcycle_graph(0)
    d_e = ctx.vector()
    ctx.pns_vcycle(2, 2, 0.1, r, d_e)
    torch.cuda.synchronize()
    assert rel(d1, d_e) <= 1e-12
    assert rel(d1, d0) > 1e-3


def test_solve_with_graph_vcycles_matches_eager_solve():
    n = (64, 64)
    out = {}
    for graph in (0, 1):
        ctx = pnsmg.Context(n, n_levels=3, precision=pnsmg.FP64)
        ctx.pns_set_vcycle_graph(graph)
        vprev = inputs.sin_series_velocity(n, seed=530, t_nodes=[0.0])
        sz = ctx.sizes()
        U0 = np.zeros(sz["nst"])
        U0[:sz["nv"]] = vprev
        U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
        U = torch.tensor(U0, device="cuda")
        rc, info = ctx.pns_solve(MODEL, torch.tensor(vprev, device="cuda"), U)
        torch.cuda.synchronize()
        assert rc == pnsmg.PNS_OK, info
        out[graph] = (info, U.cpu().numpy())
    assert out[0][0]["newton_iterations"] == out[1][0]["newton_iterations"]
    diff = np.linalg.norm(out[0][1] - out[1][1]) / np.linalg.norm(out[0][1])
    print("graph vs eager solve:", out[1][0], f"rel diff {diff:.2e}")
    assert diff <= 1e-9
