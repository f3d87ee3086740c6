"""GPU tests of the request server (continuous batching of independent slab
solves) through the C-ABI.

A served request starts from U = 0 and, if that attempt stops with
PNS_ENOTCONV, once more from the left trace.  Each served result is compared
with a direct pns_solve of the same request from the same initial guess and
with the same request served inside a mix: both reach the same stopping test
along the same iteration path, so they agree far below the solve tolerance
(the only difference is the summation order of LDS sums inside the Jacobian
action); 1e-9 relative is required.  The oracle's residual of a served result
must meet the stopping test.
"""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_28706_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

MODEL = dict(p=1.8, delta=1e-2, nu=0.1, nu_inf=1e-4, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1, lin=pnsmg.MODIFIED_NEWTON)


def nst(n):
    return 2 * (2 * (2 * n[0] + 1) * (2 * n[1] + 1) + 3 * n[0] * n[1])


def request(n, seed, levels, precision=pnsmg.FP64, model=MODEL, **params):
    vprev = inputs.sin_series_velocity(n, seed=seed, t_nodes=[0.0])
    U = np.zeros(nst(n))
    q = pnsmg.make_request(n, model, vprev, U, levels, precision=precision, **params)
    return q, vprev, U


def direct_solve(n, seed, levels, precision=pnsmg.FP64, model=MODEL, from_trace=False,
                 patch_kind=None, **params):
    vprev = inputs.sin_series_velocity(n, seed=seed, t_nodes=[0.0])
    ctx = pnsmg.Context(n, n_levels=levels, precision=precision, patch_kind=patch_kind)
    sz = ctx.sizes(0)
    U0 = np.zeros(sz["nst"])
    if from_trace:
        U0[:sz["nv"]] = vprev
        U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
    U = torch.tensor(U0, device="cuda")
    rc, info = ctx.pns_solve(model, torch.tensor(vprev, device="cuda"), U, **params)
    torch.cuda.synchronize()
    return rc, info, U.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_served_result_equals_direct_solve_and_oracle_residual():
    n = (16, 16)
    srv = pnsmg.Server(slots=2, arena_bytes=256 << 20)
    q, vprev, U = request(n, 211, 2)
    t = srv.submit(q, keep=(vprev, U))
    res = srv.wait(t)
    srv.close()
    print("served", res)
    assert res["state"] == pnsmg.REQ_DONE and res["status"] == pnsmg.PNS_OK
    rc, info, Ud = direct_solve(n, 211, 2)
    assert rc == pnsmg.PNS_OK
    assert res["newton_iterations"] == info["newton_iterations"]
    assert rel(U, Ud) <= 1e-9
    prob = O.Problem(n=n, p=MODEL["p"], delta=MODEL["delta"], nu=MODEL["nu"],
                     nu_inf=MODEL["nu_inf"], lin=O.MODIFIED_NEWTON)
    r0 = O.mass_norm(prob, O.residual(prob, np.zeros(prob.nst), vprev))
    r = O.mass_norm(prob, O.residual(prob, U, vprev))
    assert r <= 1.05 * 1e-8 * r0


def test_request_that_stalls_from_zero_is_solved_from_the_left_trace():
    """A low-p request whose solve from U = 0 needs more Newton steps than the
    limit, while the one from the left trace needs fewer: the server's second
    attempt returns the trace-started solve (same iterate), with the iteration
    counts of both attempts summed."""
    n, seed, levels = (32, 32), 503, 3
    model = dict(MODEL, p=1.2216916515341412, delta=0.007985874701397328,
                 nu_inf=0.0008305981091400222, nu=1.0)
    prm = dict(omega=0.2, rho=0.5, max_krylov=150)
    kind = pnsmg.PATCH_EXACT
    rc0, info0, _ = direct_solve(n, seed, levels, model=model, patch_kind=kind, max_newton=60, **prm)
    rct, infot, _ = direct_solve(n, seed, levels, model=model, from_trace=True, patch_kind=kind,
                                 max_newton=60, **prm)
    print("from zero", rc0, info0, "from the trace", rct, infot)
    assert rc0 == pnsmg.PNS_OK and rct == pnsmg.PNS_OK
    assert infot["newton_iterations"] < info0["newton_iterations"]
    limit = info0["newton_iterations"] - 1
    rcz, infoz, _ = direct_solve(n, seed, levels, model=model, patch_kind=kind,
                                 max_newton=limit, **prm)
    rct2, infot2, Ut = direct_solve(n, seed, levels, model=model, from_trace=True,
                                    patch_kind=kind, max_newton=limit, **prm)
    assert rcz == pnsmg.PNS_ENOTCONV and rct2 == pnsmg.PNS_OK
    srv = pnsmg.Server(slots=1, arena_bytes=256 << 20)
    q, vprev, U = request(n, seed, levels, model=model, patch_kind=kind, max_newton=limit, **prm)
    res = srv.wait(srv.submit(q, keep=(vprev, U)))
    srv.close()
    print("served", res)
    assert res["status"] == pnsmg.PNS_OK
    assert res["newton_iterations"] == infoz["newton_iterations"] + infot2["newton_iterations"]
    assert rel(U, Ut) <= 1e-9


def test_result_is_the_same_alone_and_in_a_mix():
    target = ((32, 32), 303, 3, pnsmg.FP32)
    srv = pnsmg.Server(slots=3, arena_bytes=1 << 30)
    q, vprev, U_alone = request(target[0], target[1], target[2], precision=target[3])
    srv.wait(srv.submit(q, keep=(vprev, U_alone)))
    # the same request among others of mixed sizes and precisions
    mix = [((16, 16), 301, 2, pnsmg.FP64), ((64, 64), 302, 4, pnsmg.FP64), target,
           ((32, 32), 304, 3, pnsmg.FP64), ((16, 16), 305, 2, pnsmg.FP32),
           ((64, 64), 306, 4, pnsmg.FP32)]
    tickets, outs = [], []
    for (n, seed, lv, prec) in mix:
        q, vp, U = request(n, seed, lv, precision=prec)
        tickets.append(srv.submit(q, keep=(vp, U)))
        outs.append(U)
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for r in results:
        assert r["status"] == pnsmg.PNS_OK, r
    err = rel(outs[2], U_alone)
    print(f"alone vs mix: rel diff {err:.2e}")
    assert err <= 1e-9
    # the slots ran concurrently: some running intervals overlap
    iv = sorted((r["t_start"], r["t_done"]) for r in results)
    assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))


def test_admission_respects_the_arena():
    reqs = [request((32, 32), 320 + i, 3) for i in range(5)]
    srv0 = pnsmg.Server(slots=1, arena_bytes=1 << 20)
    fp = srv0.footprint(reqs[0][0])
    srv0.close()
    assert fp > 0
    # room for two requests at a time although four slots are free
    arena = int(2.5 * fp)
    srv = pnsmg.Server(slots=4, arena_bytes=arena)
    tickets = [srv.submit(q, keep=(v, U)) for (q, v, U) in reqs]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    assert all(r["status"] == pnsmg.PNS_OK for r in results)
    events = sorted([(r["t_start"], r["footprint"]) for r in results] +
                    [(r["t_done"], -r["footprint"]) for r in results],
                    key=lambda e: (e[0], e[1]))
    held = 0
    for _, f in events:
        held += f
        assert held <= arena
    assert max(sum(1 for r in results if r["t_start"] <= t < r["t_done"])
               for t, _ in events) <= 2


def test_rejects_requests_larger_than_the_arena():
    srv = pnsmg.Server(slots=1, arena_bytes=1 << 20)
    q, vprev, U = request((32, 32), 330, 3)
    with pytest.raises(pnsmg.PnsError) as e:
        srv.submit(q, keep=(vprev, U))
    assert e.value.code == pnsmg.PNS_EWORKSPACE
    srv.close()


def test_graph_replayed_request_and_release():
    """A request whose V-cycles replay a captured HIP graph takes the same
    iterations and reaches the same iterate as the eager one; a finished
    ticket can be released once, after which it is unknown."""
    n = (32, 32)
    srv = pnsmg.Server(slots=2, arena_bytes=512 << 20)
    q0, v0, U0 = request(n, 341, 3)
    q1, v1, U1 = request(n, 341, 3, vcycle_graph=1)
    t0 = srv.submit(q0, keep=(v0, U0))
    t1 = srv.submit(q1, keep=(v1, U1))
    r0, r1 = srv.wait(t0), srv.wait(t1)
    assert r0["status"] == pnsmg.PNS_OK and r1["status"] == pnsmg.PNS_OK
    assert r0["newton_iterations"] == r1["newton_iterations"]
    assert r0["krylov_iterations"] == r1["krylov_iterations"]
    err = rel(U1, U0)
    print(f"graph-replayed request vs eager: rel diff {err:.2e}")
    assert err <= 1e-9
    srv.release(t0)
    with pytest.raises(pnsmg.PnsError) as e:
        srv.release(t0)
    assert e.value.code == pnsmg.PNS_EINVAL
    with pytest.raises(pnsmg.PnsError):
        srv.poll(t0)
    assert srv.poll(t1)["state"] == pnsmg.REQ_DONE
    srv.release(t1)
    srv.close()


def test_served_nonfinite_request_is_reported():
    n = (16, 16)
    srv = pnsmg.Server(slots=1, arena_bytes=256 << 20)
    q, vprev, U = request(n, 351, 2)
    vprev[5] = np.inf
    q = pnsmg.make_request(n, MODEL, vprev, U, 2)
    t = srv.submit(q, keep=(vprev, U))
    res = srv.wait(t)
    srv.close()
    assert res["state"] == pnsmg.REQ_DONE and res["status"] == pnsmg.PNS_ENONFINITE
