"""Pins of the oracle's spatial forms, slab Jacobian and slab residual.

What fixes each expected value (never the oracle's own formula):
* DoF counts printed in the paper (262,144 cells -> 2,887,682 spatial DoF in
  Sec. 7.1; three P1disc coefficients per cell in the DFG table of Sec. 7.2);
* exact integrals (sympy) of polynomial fields the Q2/P1disc spaces contain:
  mass, divergence and boundary pairings;
* integration-by-parts identities of the weak form (Sec. 2, Sec. 3.2): a
  constant pressure is in the kernel of the momentum rows; with the symmetric
  reading of B^s the constant pressure test annihilates every velocity; a
  constant stress (linear velocity) makes the viscous volume term and its
  boundary flux cancel; a constant velocity makes the convective volume and
  boundary terms cancel, leaving only the inflow correction B^c;
* the exact-Newton Jacobian is the derivative of the residual (Sec. 4.1,
  eq. gateaux-def) with the inflow factor lagged (Sec. 4.3);
* Picard is the fixed-point form J_Pic(U) U = A_gamma(U) (Sec. 4.2);
* symmetry of the viscous block and coercivity of the viscous-Nitsche term for
  nu_inf > 0 (Cor. linearized-viscous-coercive);
* brute-force assembled J_n equals the element-by-element action.
"""
import numpy as np
import pytest
import sympy as S

from oracle import oracle as O
from paper_2603_28706_amd import inputs

X, Y = S.symbols("x y", real=True)


def nodal(prob, exprs):
    """Q2 nodal interpolant of a velocity field given by sympy expressions."""
    xs = inputs.node_coordinates(prob.n, prob.lo, prob.hi)
    out = []
    for e in exprs:
        f = S.lambdify((X, Y), e, "numpy")
        out.append(np.broadcast_to(np.asarray(f(xs[0], xs[1]), dtype=float), xs[0].shape))
    return np.concatenate(out)


def p1disc(prob, expr):
    """P1disc coefficients of a globally linear pressure: value at the cell centre
    and h_k times the slope."""
    f = S.lambdify((X, Y), expr, "numpy")
    gx = S.lambdify((X, Y), S.diff(expr, X), "numpy")
    gy = S.lambdify((X, Y), S.diff(expr, Y), "numpy")
    hx, hy = prob.h
    out = np.zeros(3 * prob.num_cells)
    for c in range(prob.num_cells):
        i, j = c % prob.n[0], c // prob.n[0]
        xc, yc = prob.lo[0] + (i + .5) * hx, prob.lo[1] + (j + .5) * hy
        out[3 * c:3 * c + 3] = [f(xc, yc), hx * gx(xc, yc), hy * gy(xc, yc)]
    return out


def spatial(prob, vel=None, pres=None):
    v = np.zeros(prob.ns)
    if vel is not None:
        v[:prob.nv] = vel
    if pres is not None:
        v[prob.nv:] = pres
    return v


def box_faces(prob):
    (x0, y0), (x1, y1) = prob.lo[:2], prob.hi[:2]
    # (parametrisation var, fixed substitution, range, normal)
    return [
        (Y, {X: x0}, (y0, y1), (-1, 0)), (Y, {X: x1}, (y0, y1), (1, 0)),
        (X, {Y: y0}, (x0, x1), (0, -1)), (X, {Y: y1}, (x0, x1), (0, 1)),
    ]


def bint(prob, fn):
    """sum over boundary faces of int fn(normal) ds (exact)."""
    tot = 0
    for var, sub, (a, b), n in box_faces(prob):
        tot += S.integrate(fn(n).subs(sub), (var, a, b))
    return tot


def vint(prob, e):
    return S.integrate(e, (X, prob.lo[0], prob.hi[0]), (Y, prob.lo[1], prob.hi[1]))


# ------------------------------------------------------------------- counts

def test_dof_counts_against_paper():
    # Sec. 7.1: 262,144 cells (512^2) carry 2,887,682 spatial unknowns
    assert O.Problem(n=(512, 512)).ns == 2_887_682
    # Sec. 7.2: P1disc has three coefficients per cell (304 cells -> 912)
    for cells, pdofs in [(304, 912), (1216, 3648), (4864, 14592), (19456, 58368)]:
        assert 3 * cells == pdofs
    assert O.Problem(n=(8, 8)).nst == 1540
    assert O.Problem(n=(256, 256)).nst == 1_445_892
    assert O.Problem(n=(32, 32, 32)).nst == 1_909_894


# ------------------------------------------------------------ exact integrals

def test_mass_matrix_exact_integral():
    prob = O.Problem(n=(3, 2), hi=(2.0, 1.0, 1.0))
    f = X ** 2 * Y + S.Rational(1, 2)
    g = Y ** 2 * X + X
    Mx = O.assemble_velocity_mass(prob)
    a = spatial(prob, nodal(prob, [f, 0 * X]))
    b = spatial(prob, nodal(prob, [g, 0 * X]))
    exact = float(vint(prob, f * g))
    assert abs(a @ (Mx @ b) - exact) < 1e-13 * abs(exact)


@pytest.mark.parametrize("qsign", [1, -1])
def test_pressure_velocity_blocks_exact(qsign):
    """continuity block: -(div u, q) + qsign <u.n, q>; momentum block:
    -(div w, pi) + <pi, w.n>; polynomial fields, exact integration."""
    prob = O.Problem(n=(3, 2), hi=(1.5, 1.0, 1.0), qsign=qsign, convection=0)
    u = [X ** 2 + X * Y, X * Y - Y ** 2 / 3]
    q = 1 + 2 * X - Y
    J = O.assemble_spatial(prob, np.zeros(prob.nv))
    uu = spatial(prob, vel=nodal(prob, u))
    qq = spatial(prob, pres=p1disc(prob, q))
    div = S.diff(u[0], X) + S.diff(u[1], Y)
    cont = -vint(prob, div * q) + qsign * bint(prob, lambda n: (u[0] * n[0] + u[1] * n[1]) * q)
    mom = -vint(prob, div * q) + bint(prob, lambda n: q * (u[0] * n[0] + u[1] * n[1]))
    assert abs(qq @ (J @ uu) - float(cont)) < 1e-12
    assert abs(uu @ (J @ qq) - float(mom)) < 1e-12


def test_newtonian_viscous_nitsche_form_exact():
    """p = 2 (eta = nu_inf + nu everywhere, eta_D the same) and no convection:
    the velocity block is
    (eta Dx, Dw) - <eta Dx n, w> - eta_D <x, Dw n> + g1 eta_D/h <x,w> + g2/h <x.n, w.n>."""
    prob = O.Problem(n=(2, 2), p=2.0, nu=0.7, nu_inf=0.2, delta=0.3, convection=0,
                     gamma1=5.0, gamma2=3.0, lin=O.EXACT_NEWTON)
    eta = 0.9
    h = prob.h[0]
    xf = [X ** 2 * Y, X - Y ** 2]
    wf = [Y * X + 1, X ** 2 - X * Y]
    rng = np.random.default_rng(0)
    uk = rng.uniform(-1, 1, prob.nv)  # irrelevant for p = 2
    J = O.assemble_spatial(prob, uk)

    def Dfix(f):
        G = [[S.diff(f[i], v) for v in (X, Y)] for i in range(2)]
        return [[(G[i][j] + G[j][i]) / 2 for j in range(2)] for i in range(2)]

    Dx, Dw = Dfix(xf), Dfix(wf)
    vol = vint(prob, eta * sum(Dx[i][j] * Dw[i][j] for i in range(2) for j in range(2)))

    def bterm(n):
        Dxn = [Dx[i][0] * n[0] + Dx[i][1] * n[1] for i in range(2)]
        Dwn = [Dw[i][0] * n[0] + Dw[i][1] * n[1] for i in range(2)]
        xw = xf[0] * wf[0] + xf[1] * wf[1]
        xn = xf[0] * n[0] + xf[1] * n[1]
        wn = wf[0] * n[0] + wf[1] * n[1]
        return (-eta * (Dxn[0] * wf[0] + Dxn[1] * wf[1]) - eta * (Dwn[0] * xf[0] + Dwn[1] * xf[1])
                + prob.gamma1 * eta / h * xw + prob.gamma2 / h * xn * wn)

    exact = float(vol + bint(prob, bterm))
    a = spatial(prob, vel=nodal(prob, xf))
    b = spatial(prob, vel=nodal(prob, wf))
    assert abs(b @ (J @ a) - exact) < 1e-12 * max(1.0, abs(exact))


def test_newton_convection_exact_for_linear_state():
    """Newton convection with a linear state u and Q2 fields, exact integration:
    -(x (x) u + u (x) x, grad w) + <(x.n) u + (u.n) x, w> - <(u.n)^- x, w>."""
    base = O.Problem(n=(2, 2), p=2.0, nu=1.0, nu_inf=0.0, delta=1.0, gamma1=0.0, gamma2=0.0,
                     lin=O.EXACT_NEWTON)
    u = [1 + X - Y / 2, S.Rational(1, 2) - X + Y / 3]
    xf = [X * Y, Y ** 2 - X]
    wf = [X ** 2, X * Y + 1]
    uk = nodal(base, u)
    Jc = O.assemble_spatial(base, uk) - O.assemble_spatial(base.with_(convection=0), uk)
    G = [[S.diff(wf[i], v) for v in (X, Y)] for i in range(2)]
    vol = -vint(base, sum((xf[i] * u[j] + u[i] * xf[j]) * G[i][j]
                          for i in range(2) for j in range(2)))

    def bterm(n):
        un = u[0] * n[0] + u[1] * n[1]
        xn = xf[0] * n[0] + xf[1] * n[1]
        uw = u[0] * wf[0] + u[1] * wf[1]
        xw = xf[0] * wf[0] + xf[1] * wf[1]
        neg = (S.Abs(un) - un) / 2
        return xn * uw + un * xw - neg * xw

    # (u.n)^- is piecewise: integrate each face numerically-exactly via sympy piecewise
    exact = float(vol + bint(base, bterm))
    a = spatial(base, vel=nodal(base, xf))
    b = spatial(base, vel=nodal(base, wf))
    # (u.n)^- is not polynomial where u.n changes sign on a face: allow quadrature error there
    assert abs(b @ (Jc @ a) - exact) < 2e-3 * max(1.0, abs(exact))


def test_penalty_terms_constant_fields_closed_form():
    """u_k = 0, no convection, constant x = c and w = e: only the penalty terms
    survive: g1 eta_D/h |Gamma| c.e + g2/h sum_faces |F| (c.n)(e.n)."""
    prob = O.Problem(n=(4, 4), p=1.4, delta=0.05, nu=1.3, nu_inf=0.01, convection=0,
                     gamma1=7.0, gamma2=11.0)
    J = O.assemble_spatial(prob, np.zeros(prob.nv))
    c, e = np.array([0.3, -1.2]), np.array([2.0, 0.7])
    nn = prob.num_nodes
    a = spatial(prob, vel=np.concatenate([np.full(nn, c[0]), np.full(nn, c[1])]))
    b = spatial(prob, vel=np.concatenate([np.full(nn, e[0]), np.full(nn, e[1])]))
    etaD = 0.01 + 1.3 * 0.05 ** (1.4 - 2)
    h = 0.25
    exact = 7.0 * etaD / h * 4.0 * (c @ e) + 11.0 / h * (2 * c[0] * e[0] + 2 * c[1] * e[1])
    assert abs(b @ (J @ a) - exact) < 1e-12 * abs(exact)


# ---------------------------------------------------- identities (residual)

def time_constant_state(prob, vel, pres):
    U = np.zeros(prob.nst)
    for m in range(prob.nt):
        U[m * prob.ns:m * prob.ns + prob.nv] = vel
        U[m * prob.ns + prob.nv:(m + 1) * prob.ns] = pres
    return U


def test_time_residual_vanishes_for_constant_state():
    prob = O.Problem(n=(3, 3), convection=0)
    rng = np.random.default_rng(1)
    v = rng.uniform(-1, 1, prob.nv)
    U = time_constant_state(prob, v, np.zeros(3 * prob.num_cells))
    R_with = O.residual(prob, U, vprev=v)
    R_tau0 = O.residual(prob.with_(tau=1e-300), U, vprev=v)   # spatial part scaled away
    assert np.abs(R_tau0).max() < 1e-14
    # and with a different left trace the jump term is -m_t (x) M_x (v - vprev)
    vp = rng.uniform(-1, 1, prob.nv)
    Mx = O.assemble_velocity_mass(prob)
    Rj = O.residual(prob.with_(tau=1e-300), U, vprev=vp)
    _, _, _, m = O.time_matrices(1)
    for mu in range(2):
        expect = -m[mu] * (Mx @ spatial(prob, vel=v - vp))
        assert np.allclose(Rj[mu * prob.ns:(mu + 1) * prob.ns], expect, atol=1e-14)
    assert np.isfinite(R_with).all()


@pytest.mark.parametrize("lin", [O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON])
def test_constant_pressure_kernel_and_left_kernel(lin):
    prob = O.Problem(n=(4, 3), lin=lin)
    rng = np.random.default_rng(2)
    uk = rng.uniform(-1, 1, prob.nt * prob.nv)
    Jn = O.assemble_slab(prob, O.split_uk(prob, uk))
    for mu in range(prob.nt):
        e = np.zeros(prob.nst)
        e[mu * prob.ns + prob.nv::3][:prob.num_cells] = 1.0   # constant coefficient of every cell
        e[(mu + 1) * prob.ns:] = 0.0
        scale = abs(Jn).max()
        assert np.abs(Jn @ e).max() < 1e-13 * scale
        assert np.abs(Jn.T @ e).max() < 1e-13 * scale
    # literal "+q I" breaks the left kernel
    Jl = O.assemble_slab(prob.with_(qsign=-1), O.split_uk(prob, uk))
    e = np.zeros(prob.nst)
    e[prob.nv:prob.ns:3] = 1.0
    assert np.abs(Jl.T @ e).max() > 1e-3


def test_constant_stress_cancels_viscous_flux():
    """u linear => S(Du) constant => (S, Dw) - <S n, w> = 0 for every w.
    With no convection, zero pressure and a time-constant state, the momentum
    residual reduces to the Nitsche terms, which are integrated exactly here."""
    prob = O.Problem(n=(3, 3), p=1.3, delta=1e-3, nu=1.0, nu_inf=1e-3, convection=0,
                     gamma1=9.0, gamma2=4.0)
    u = [2 * X - Y, X + Y / 2 + 1]          # D u constant, |Du| ~ 2
    vel = nodal(prob, u)
    U = time_constant_state(prob, vel, np.zeros(3 * prob.num_cells))
    R = O.residual(prob, U, vprev=vel)
    etaD = 1e-3 + 1.0 * 1e-3 ** (1.3 - 2)
    h = prob.h[0]
    w_exprs = [[X * Y + 1, Y ** 2], [X ** 2 - Y, X * Y * Y]]
    for wf in w_exprs:
        Dw = [[(S.diff(wf[i], vv) + S.diff(wf[j], v)) / 2 for j, vv in enumerate((X, Y))]
              for i, v in enumerate((X, Y))]

        def bterm(n):
            Dwn = [Dw[i][0] * n[0] + Dw[i][1] * n[1] for i in range(2)]
            uw = u[0] * wf[0] + u[1] * wf[1]
            un = u[0] * n[0] + u[1] * n[1]
            wn = wf[0] * n[0] + wf[1] * n[1]
            return (-etaD * (Dwn[0] * u[0] + Dwn[1] * u[1]) + prob.gamma1 * etaD / h * uw
                    + prob.gamma2 / h * un * wn)

        nitsche = float(bint(prob, bterm))
        w = spatial(prob, vel=nodal(prob, wf))
        got = sum(w @ R[m * prob.ns:(m + 1) * prob.ns] / (-prob.tau * wm)
                  for m, wm in enumerate([0.75, 0.25])) / 2
        assert abs(got - nitsche) < 1e-10 * max(1.0, abs(nitsche)), (got, nitsche)


def test_constant_velocity_leaves_only_inflow_correction():
    """c(u)(w) = -(u (x) u, grad w) + <(u.n) u, w> vanishes for constant u; the
    remaining convective residual is -<(u.n)^- u, w>; for w = e constant that is
    -sum_faces |F| (u.n)^- (u.e)."""
    prob = O.Problem(n=(3, 3), p=1.7, convection=1)
    uc = np.array([0.8, -0.3])
    nn = prob.num_nodes
    vel = np.concatenate([np.full(nn, uc[0]), np.full(nn, uc[1])])
    U = time_constant_state(prob, vel, np.zeros(3 * prob.num_cells))
    Rc = O.residual(prob, U, vprev=vel) - O.residual(prob.with_(convection=0), U, vprev=vel)
    # inflow: left face (n=(-1,0), u.n=-0.8 -> 0.8) and top face (n=(0,1), u.n=-0.3 -> 0.3)
    for e in (np.array([1.0, 0.0]), np.array([0.0, 1.0]), np.array([0.4, 2.0])):
        w = spatial(prob, vel=np.concatenate([np.full(nn, e[0]), np.full(nn, e[1])]))
        expect = -(0.8 + 0.3) * (uc @ e)
        for m, wm in enumerate([0.75, 0.25]):
            got = w @ Rc[m * prob.ns:(m + 1) * prob.ns] / (-prob.tau * wm)
            assert abs(got - expect) < 1e-12, (got, expect)


# --------------------------------------------------- linearisations vs residual

@pytest.mark.parametrize("conv", [0, 1])
def test_exact_newton_is_derivative_of_residual(conv):
    prob = O.Problem(n=(3, 3), p=1.5, delta=1e-2, nu_inf=1e-3, convection=conv,
                     lin=O.EXACT_NEWTON)
    rng = np.random.default_rng(4)
    U = rng.uniform(-1, 1, prob.nst)
    dU = rng.uniform(-1, 1, prob.nst)
    vprev = rng.uniform(-1, 1, prob.nv)
    uk = np.concatenate([U[m * prob.ns:m * prob.ns + prob.nv] for m in range(prob.nt)])
    Jd = O.apply(prob, uk, dU)
    eps = 1e-6
    fd = -(O.residual(prob, U + eps * dU, vprev, ulag=uk)
           - O.residual(prob, U - eps * dU, vprev, ulag=uk)) / (2 * eps)
    assert np.linalg.norm(Jd - fd) <= 1e-7 * np.linalg.norm(Jd)


def test_picard_fixed_point_form():
    prob = O.Problem(n=(3, 2), p=1.3, delta=1e-3, lin=O.PICARD)
    rng = np.random.default_rng(5)
    U = rng.uniform(-1, 1, prob.nst)
    uk = np.concatenate([U[m * prob.ns:m * prob.ns + prob.nv] for m in range(prob.nt)])
    assert np.allclose(O.apply(prob, uk, U), -O.residual(prob, U), rtol=0, atol=1e-12)


def test_modified_newton_limits_globally():
    base = O.Problem(n=(3, 3), p=1.2, delta=1e-3, convection=0)
    rng = np.random.default_rng(6)
    uk = rng.uniform(-1, 1, base.nt * base.nv)
    x = rng.uniform(-1, 1, base.nst)
    y_inf = O.apply(base.with_(lin=O.MODIFIED_NEWTON, sigma_max=1e300), uk, x)
    y_ex = O.apply(base.with_(lin=O.EXACT_NEWTON), uk, x)
    y_0 = O.apply(base.with_(lin=O.MODIFIED_NEWTON, sigma_max=0.0), uk, x)
    y_pic = O.apply(base.with_(lin=O.PICARD), uk, x)
    assert np.allclose(y_inf, y_ex, rtol=0, atol=1e-13 * np.abs(y_ex).max())
    assert np.allclose(y_0, y_pic, rtol=0, atol=1e-13 * np.abs(y_pic).max())
    # with convection on, sigma_max = 0 keeps the Newton convection
    c = base.with_(convection=1)
    d0 = O.apply(c.with_(lin=O.MODIFIED_NEWTON, sigma_max=0.0), uk, x) - y_0
    dex = O.apply(c.with_(lin=O.EXACT_NEWTON), uk, x) - y_ex
    assert np.allclose(d0, dex, rtol=0, atol=1e-13 * np.abs(y_ex).max())


# ---------------------------------------------------- structure of J_n

@pytest.mark.parametrize("lin", [O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON])
def test_interior_element_matrix_symmetric_without_convection(lin):
    prob = O.Problem(n=(3, 3), convection=0, lin=lin, p=1.3, delta=1e-3)
    rng = np.random.default_rng(7)
    E = O.element_matrices(prob, rng.uniform(-1, 1, prob.nv))
    Ec = E[4]   # the interior cell
    assert np.allclose(Ec, Ec.T, atol=1e-13 * np.abs(Ec).max())


def test_full_spatial_block_symmetric_at_zero_state():
    prob = O.Problem(n=(3, 3), convection=0, p=1.3, delta=1e-3)
    J = O.assemble_spatial(prob, np.zeros(prob.nv)).toarray()
    assert np.allclose(J, J.T, atol=1e-13 * np.abs(J).max())


def test_kronecker_structure():
    prob = O.Problem(n=(3, 2))
    rng = np.random.default_rng(8)
    uk = rng.uniform(-1, 1, prob.nt * prob.nv)
    Jn = O.assemble_slab(prob, O.split_uk(prob, uk)).toarray()
    Mx = O.assemble_velocity_mass(prob).toarray()
    _, _, K, _ = O.time_matrices(1)
    ns, nv = prob.ns, prob.nv
    for i in range(2):
        for j in range(2):
            if i != j:
                blk = Jn[i * ns:(i + 1) * ns, j * ns:(j + 1) * ns]
                assert np.allclose(blk[:nv, :nv], K[i, j] * Mx[:nv, :nv], atol=1e-15)
                assert np.abs(blk[nv:, :]).max() == 0 and np.abs(blk[:, nv:]).max() == 0
    # pressure-pressure block is zero
    for i in range(2):
        assert np.abs(Jn[i * ns + nv:(i + 1) * ns, i * ns + nv:(i + 1) * ns]).max() == 0


def test_assembled_equals_matrix_free():
    prob = O.Problem(n=(4, 3), p=1.2, delta=1e-4, nu_inf=1e-4)
    rng = np.random.default_rng(9)
    uk = rng.uniform(-1, 1, prob.nt * prob.nv)
    x = rng.uniform(-1, 1, prob.nst)
    for lin in (O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON):
        pr = prob.with_(lin=lin)
        y = O.apply(pr, uk, x)
        Jn = O.assemble_slab(pr, O.split_uk(pr, uk))
        assert np.abs(Jn @ x - y).max() <= 1e-14 * np.abs(y).max()


@pytest.mark.parametrize("lin", [O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON])
def test_viscous_nitsche_coercive_for_positive_nu_inf(lin):
    """Velocity block without convection and pressure (the form a*_m of
    eq. am-def): for nu_inf > 0 its symmetric part is positive definite once
    gamma1 exceeds a threshold that grows with the ratio of the frozen boundary
    viscosity to the tangent's lower bound (Cor. linearized-viscous-coercive);
    the penalty is PSD so positivity persists for larger gamma1; without penalty
    the form is indefinite.  For a mild state (tangent close to eta_D) the
    configured gamma1 = 40 suffices."""
    prob = O.Problem(n=(4, 4), p=1.3, delta=1e-2, nu=1.0, nu_inf=1e-2, convection=0, lin=lin)
    rng = np.random.default_rng(10)
    u = rng.uniform(-1, 1, prob.nv)
    nv = prob.nv

    def lam_min(pr, state):
        A = O.assemble_spatial(pr, state).toarray()[:nv, :nv]
        return np.linalg.eigvalsh(0.5 * (A + A.T))[0]

    gammas = [0.0, 10.0, 40.0, 160.0, 640.0, 2560.0]
    lams = [lam_min(prob.with_(gamma1=g, gamma2=g), u) for g in gammas]
    assert lams[0] < 0
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(lams, lams[1:]))
    assert lams[-1] > 0
    assert lam_min(prob, 1e-3 * u) > 0
