"""CPU pins of the oracle's slab solve: the block mass-weighted residual norm and
the Newton iteration on R_n(U) = 0 (Sec. 6, Sec. 6.2).  They check the oracle against
closed forms and against properties that any correct solver has, not against
itself."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_28706_amd import inputs

N = (8, 8)


def vprev_field(n=N, seed=201):
    return inputs.sin_series_velocity(n, seed=seed, t_nodes=[0.0])


def test_mass_norm_closed_forms():
    prob = O.Problem(n=(4, 3), hi=(2.0, 0.5, 1.0), tau=0.02)
    area = 2.0 * 0.5
    r = np.zeros(prob.nst)
    # constant velocity component 0 at both Radau nodes: tau (sum of weights) |Omega| c^2
    for m in range(prob.nt):
        r[m * prob.ns:m * prob.ns + prob.num_nodes] = 3.0
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * area * 9.0, rel=1e-13)
    # the same at one Radau node only: weighted by that node's Radau weight
    r[prob.ns:] = 0.0
    w0 = O.radau_right(1)[1][0]
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * w0 * area * 9.0, rel=1e-13)
    # constant pressure coefficient 1 on every cell, both nodes: tau |Omega|
    r = np.zeros(prob.nst)
    for m in range(prob.nt):
        r[m * prob.ns + prob.nv::3][:prob.num_cells] = 1.0
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * area, rel=1e-13)
    # the x-slope coefficient: int ((x - x_c)/h_x)^2 = |K| / 12 per cell
    r = np.zeros(prob.nst)
    r[prob.nv + 1:prob.ns:3] = 1.0
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * w0 * area / 12.0, rel=1e-13)


def test_mass_norm_of_a_quadratic_field_is_its_l2_norm():
    # u_0 = x (1 - x) y is represented exactly by Q2 nodal values; int_Omega u_0^2 = 1/90
    prob = O.Problem(n=(3, 5))
    x, y = inputs.node_coordinates(prob.n, prob.lo[:2], prob.hi[:2])
    u = x * (1 - x) * y
    r = np.zeros(prob.nst)
    r[:prob.num_nodes] = u
    w0 = O.radau_right(1)[1][0]
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * w0 / 90.0, rel=1e-12)


def test_mass_norm_closed_forms_3d():
    prob = O.Problem(n=(2, 3, 2), hi=(2.0, 0.5, 1.5), tau=0.02)
    vol = 2.0 * 0.5 * 1.5
    w0, w1 = O.radau_right(1)[1]
    nn = prob.num_nodes
    # constant velocity component 2 (value 3) at both Radau nodes
    r = np.zeros(prob.nst)
    for m in range(prob.nt):
        r[m * prob.ns + 2 * nn:m * prob.ns + 3 * nn] = 3.0
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * vol * 9.0, rel=1e-13)
    # the z-slope pressure coefficient at the second node: |K| / 12 per cell
    r = np.zeros(prob.nst)
    r[prob.ns + prob.nv + 3:2 * prob.ns:4] = 1.0
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * w1 * vol / 12.0, rel=1e-13)
    # u_1 = x y (1.5 - z) z is triquadratic, represented exactly:
    # int u^2 = (8/3) (1/24) (1.5^5 / 30) over [0,2] x [0,0.5] x [0,1.5]
    x, y, z = inputs.node_coordinates(prob.n, prob.lo, prob.hi)
    r = np.zeros(prob.nst)
    r[nn:2 * nn] = x * y * (1.5 - z) * z
    exact = (8.0 / 3.0) * (0.125 / 3.0) * (1.5 ** 5 / 30.0)
    assert O.mass_norm(prob, r) ** 2 == pytest.approx(prob.tau * w0 * exact, rel=1e-12)


def test_zero_data_gives_zero_solution_without_steps():
    prob = O.Problem(n=N)
    res = O.newton_solve(prob, np.zeros(prob.nv))
    assert res.residual_norms == [0.0] and res.steps == []
    assert not res.U.any()


def test_linear_problem_is_solved_in_one_step():
    # p = 2 without convection: the residual is affine in U and every
    # linearisation is its exact derivative
    for lin in (O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON):
        prob = O.Problem(n=N, p=2.0, convection=0, lin=lin)
        res = O.newton_solve(prob, vprev_field(), rtol=1e-12)
        assert len(res.steps) == 1 and res.steps[0] == 1.0
        assert res.residual_norms[-1] <= 1e-12 * res.residual_norms[0]


def test_exact_newton_converges_quadratically():
    # estimated order log(r_{k+1}/r_k) / log(r_k/r_{k-1}) near 2 above the
    # rounding floor; a Jacobian missing a term of the residual's derivative
    # would converge linearly (order 1), like the clipped tangent does
    orders = {}
    for lin in (O.EXACT_NEWTON, O.MODIFIED_NEWTON):
        prob = O.Problem(n=N, p=1.5, delta=1e-2, lin=lin)
        res = O.newton_solve(prob, vprev_field(), rtol=1e-15)
        r = np.asarray(res.residual_norms) / res.residual_norms[0]
        r = r[r > 1e-13]
        orders[lin] = [np.log(r[k + 1] / r[k]) / np.log(r[k] / r[k - 1])
                       for k in range(len(r) - 2, max(len(r) - 4, 0), -1)]
    assert min(orders[O.EXACT_NEWTON]) > 1.6
    assert max(orders[O.MODIFIED_NEWTON]) < 1.3


def test_all_linearisations_reach_the_same_solution():
    vp = vprev_field()
    sols = []
    for lin in (O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON):
        prob = O.Problem(n=N, p=1.5, delta=1e-2, lin=lin)
        res = O.newton_solve(prob, vp, rtol=1e-13)
        assert res.residual_norms[-1] <= 1e-13 * res.residual_norms[0]
        sols.append(res.U)
    scale = np.abs(sols[0]).max()
    for s in sols[1:]:
        # the pinned pressure coefficient makes even the pressures comparable
        assert np.abs(s - sols[0]).max() <= 1e-9 * scale


def test_kinetic_energy_decays_without_convection():
    # p-Stokes with homogeneous Dirichlet data and no forcing is dissipative:
    # the velocity at the end of the slab (right Radau node) carries less
    # kinetic energy than the left trace, and more so for stronger viscosity
    vp = vprev_field()
    prob0 = O.Problem(n=N)
    Mv = O.assemble_velocity_mass(prob0)
    e0 = vp @ (Mv[:prob0.nv, :prob0.nv] @ vp)
    ratios = []
    for nu in (0.1, 1.0):
        prob = O.Problem(n=N, p=1.5, nu=nu, convection=0)
        res = O.newton_solve(prob, vp, rtol=1e-12)
        u_end = res.U[prob.ns:prob.ns + prob.nv]
        ratios.append(u_end @ (Mv[:prob.nv, :prob.nv] @ u_end) / e0)
    assert 0.0 < ratios[1] < ratios[0] < 1.0


def test_solution_is_independent_of_the_initial_guess():
    prob = O.Problem(n=N, p=1.5, delta=1e-2)
    vp = vprev_field()
    a = O.newton_solve(prob, vp, rtol=1e-13)
    U0 = a.U + 1e-3 * inputs.uniform(7, prob.nst)
    U0[O.pressure_pin_indices(prob)] = 0.0
    b = O.newton_solve(prob, vp, U0=U0, rtol=1e-13)
    assert np.abs(a.U - b.U).max() <= 1e-9 * np.abs(a.U).max()
