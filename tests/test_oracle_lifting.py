"""Pins of the oracle's inhomogeneous Dirichlet data (Sec. 3.2, eq. def-b-gam;
eq. disc-residual).  The lifting ghat_D is a Q2 velocity field per Radau node,
g_D its trace; the Nitsche terms B^s and B^r are frozen at G = D ghat_D and the
residual carries B_gamma(g_D, w) on its right-hand side.

What fixes each expected value (never the oracle's own formula):
* exact integrals (sympy) of the boundary terms for polynomial fields, with the
  stress derivative DS(G) obtained by symbolic differentiation of the stress
  law of eq. (constitutive-law) (not the tangent formula the oracle uses): the
  change of the spatial Jacobian when the lifting is switched on, and the
  right-hand side B_gamma(g_D, .) with inflow, symmetry and penalty parts;
* consistency (Sec. 3.2, "Consistency and adjoint consistency"): a velocity
  linear in space and time and a linear pressure lie in the discrete space, so
  with g_D their trace and f from the strong form eq. (pns-strong) the slab
  residual vanishes, in 2D and 3D, for p != 2;
* the exact-Newton Jacobian is the derivative of the residual with the lifting
  present (the frozen coefficients make B^s and B^r linear in U)."""
import numpy as np
import pytest
import sympy as S

from oracle import oracle as O
from paper_2603_28706_amd import inputs

X, Y, Z, T, EPS = S.symbols("x y z t eps", real=True)


def nodal(prob, exprs, t=None):
    xs = inputs.node_coordinates(prob.n, prob.lo, prob.hi)
    syms = (X, Y, Z)[:prob.dim]
    out = []
    for e in exprs:
        e = e.subs(T, t) if t is not None else e
        f = S.lambdify(syms, e, "numpy")
        out.append(np.broadcast_to(np.asarray(f(*xs[:prob.dim]), dtype=float), xs[0].shape))
    return np.concatenate(out)


def box_faces_2d(prob):
    (x0, y0), (x1, y1) = prob.lo[:2], prob.hi[:2]
    return [(Y, {X: x0}, (y0, y1), (-1, 0)), (Y, {X: x1}, (y0, y1), (1, 0)),
            (X, {Y: y0}, (x0, x1), (0, -1)), (X, {Y: y1}, (x0, x1), (0, 1))]


def bint(prob, fn):
    tot = 0
    for var, sub, (a, b), n in box_faces_2d(prob):
        tot += S.integrate(S.expand(fn(n).subs(sub)), (var, a, b))
    return tot


def symgrad(f, syms):
    d = len(f)
    G = [[S.diff(f[i], syms[j]) for j in range(d)] for i in range(d)]
    return [[(G[i][j] + G[j][i]) / 2 for j in range(d)] for i in range(d)]


def stress(prob, A):
    """S(A) = (nu_inf + nu (delta^2 + |A|^2)^((p-2)/2)) A, eq. (constitutive-law)."""
    d = len(A)
    a2 = sum(A[i][j] ** 2 for i in range(d) for j in range(d))
    p = S.nsimplify(prob.p)
    eta = S.nsimplify(prob.nu_inf) + S.nsimplify(prob.nu) * (S.nsimplify(prob.delta) ** 2
                                                             + a2) ** ((p - 2) / 2)
    return [[eta * A[i][j] for j in range(d)] for i in range(d)], eta


def dstress(prob, G, B):
    """DS(G)(B) by differentiating eps -> S(G + eps B) at eps = 0 (G constant)."""
    d = len(G)
    Sg, _ = stress(prob, [[G[i][j] + EPS * B[i][j] for j in range(d)] for i in range(d)])
    return [[S.diff(Sg[i][j], EPS).subs(EPS, 0) for j in range(d)] for i in range(d)]


def spatial(prob, vel):
    v = np.zeros(prob.ns)
    v[:prob.nv] = vel
    return v


# a lifting linear in space: G = D ghat constant, [[0.8, 0.1], [0.1, 0.6]]
G_LIFT = [S.Rational(2, 5) + S.Rational(4, 5) * X - S.Rational(3, 10) * Y,
          -S.Rational(1, 5) + S.Rational(1, 2) * X + S.Rational(3, 5) * Y]


def test_frozen_coefficients_follow_the_lifting_gradient():
    """J(lifting) - J(0), velocity block, between polynomial Q2 fields x, w:
    -<x, (DS(G) - DS(0))(Dw) n> + gamma1 (eta(G) - eta(0)) / h <x, w>."""
    prob = O.Problem(n=(2, 2), p=1.4, delta=0.3, nu=0.7, nu_inf=0.2, convection=0,
                     gamma1=5.0, gamma2=3.0, lin=O.EXACT_NEWTON)
    g = nodal(prob, G_LIFT)
    lifted = prob.with_(lifting=np.concatenate([g, g]))
    uk = np.zeros(prob.nv)
    dJ = (O.assemble_spatial(lifted, uk, g) - O.assemble_spatial(prob, uk)).toarray()
    G = symgrad(G_LIFT, (X, Y))
    zero = [[0, 0], [0, 0]]
    h = prob.h[0]
    xf = [X ** 2 * Y + 1, X - Y ** 2]
    wf = [Y * X + X, X ** 2 - X * Y + Y]
    Dw = symgrad(wf, (X, Y))
    dSg, dS0 = dstress(prob, G, Dw), dstress(prob, zero, Dw)
    _, etaG = stress(prob, G)
    _, eta0 = stress(prob, zero)

    def bterm(n):
        dn = [sum((dSg[i][j] - dS0[i][j]) * n[j] for j in range(2)) for i in range(2)]
        xw = xf[0] * wf[0] + xf[1] * wf[1]
        return -(dn[0] * xf[0] + dn[1] * xf[1]) + prob.gamma1 * (etaG - eta0) / h * xw

    exact = float(bint(prob, bterm))
    a = spatial(prob, nodal(prob, xf))
    b = spatial(prob, nodal(prob, wf))
    got = b @ (dJ @ a)
    assert abs(exact) > 1e-2
    assert abs(got - exact) < 1e-12 * max(1.0, abs(exact)), (got, exact)


@pytest.mark.parametrize("qsign", [1, -1])
def test_right_hand_side_is_b_gamma_of_the_data(qsign):
    """R(U = 0) with the lifting minus R(U = 0) without it is tau w_mu B_gamma(g_D, w):
    -<(g.n)^- g, w> - <g, DS(G)(Dw) n> + qsign <g.n, q> + gamma1 eta(G)/h <g, w>
    + gamma2/h <g.n, w.n>, the lifting different at the two Radau nodes."""
    prob = O.Problem(n=(2, 3), hi=(1.0, 1.5, 1.0), p=1.6, delta=0.2, nu=0.9, nu_inf=0.05,
                     convection=1, gamma1=4.0, gamma2=6.0, qsign=qsign)
    # g.n keeps one sign on every face: inflow on the left and bottom faces only
    lifts = [[S.Rational(3, 2) + S.Rational(3, 10) * X - S.Rational(1, 5) * Y,
              S.Rational(6, 5) + S.Rational(1, 4) * X + S.Rational(1, 10) * Y],
             [S.Rational(1, 1) + S.Rational(1, 2) * X + S.Rational(1, 5) * Y,
              S.Rational(4, 5) - S.Rational(1, 5) * X + S.Rational(3, 10) * Y]]
    lift = np.concatenate([nodal(prob, gl) for gl in lifts])
    lifted = prob.with_(lifting=lift)
    R = O.residual(lifted, np.zeros(prob.nst)) - O.residual(prob, np.zeros(prob.nst))
    h = prob.h
    wf = [X * Y + 1, X ** 2 - Y]
    qf = 1 + 2 * X - Y
    Dw = symgrad(wf, (X, Y))
    b = spatial(prob, nodal(prob, wf))
    # P1disc coefficients of the linear pressure test: value at the centre, h_k slope
    qv = np.zeros(prob.ns)
    for c in range(prob.num_cells):
        i, j = c % prob.n[0], c // prob.n[0]
        xc, yc = (i + .5) * h[0], (j + .5) * h[1]
        qv[prob.nv + 3 * c:prob.nv + 3 * c + 3] = [1 + 2 * xc - yc, 2 * h[0], -h[1]]
    for mu, wmu in enumerate((0.75, 0.25)):
        gl = lifts[mu]
        G = symgrad(gl, (X, Y))
        DSw = dstress(prob, G, Dw)
        _, etaG = stress(prob, G)

        def bterm(n):
            hF = h[0] if n[0] != 0 else h[1]
            gn = gl[0] * n[0] + gl[1] * n[1]
            wn = wf[0] * n[0] + wf[1] * n[1]
            gw = gl[0] * wf[0] + gl[1] * wf[1]
            neg = (S.Abs(gn) - gn) / 2
            dn = [DSw[i][0] * n[0] + DSw[i][1] * n[1] for i in range(2)]
            return (-neg * gw - (dn[0] * gl[0] + dn[1] * gl[1]) + prob.gamma1 * etaG / hF * gw
                    + prob.gamma2 / hF * gn * wn)

        def qterm(n):
            return qsign * (gl[0] * n[0] + gl[1] * n[1]) * qf

        Rm = R[mu * prob.ns:(mu + 1) * prob.ns]
        exact_v = float(bint(prob, bterm))
        exact_q = float(bint(prob, qterm))
        got_v = b @ Rm / (prob.tau * wmu)
        got_q = qv @ Rm / (prob.tau * wmu)
        assert abs(got_v - exact_v) < 1e-11 * max(1.0, abs(exact_v)), (mu, got_v, exact_v)
        assert abs(got_q - exact_q) < 1e-11 * max(1.0, abs(exact_q)), (mu, got_q, exact_q)


def linear_solution(dim):
    """u linear in space and time and divergence free, pi linear in space."""
    syms = (X, Y, Z)[:dim]
    if dim == 2:
        u = [(1 + T) * (S.Rational(3, 10) + S.Rational(1, 5) * X + S.Rational(1, 2) * Y),
             (1 + T) * (-S.Rational(1, 5) + S.Rational(2, 5) * X - S.Rational(1, 5) * Y)]
        pi = S.Rational(7, 10) * X - S.Rational(2, 5) * Y
    else:
        u = [(1 + T) * (S.Rational(3, 10) + S.Rational(1, 5) * X + S.Rational(1, 2) * Y
                        - S.Rational(1, 10) * Z),
             (1 + T) * (-S.Rational(1, 5) + S.Rational(2, 5) * X - S.Rational(1, 2) * Y
                        + S.Rational(1, 5) * Z),
             (1 + T) * (S.Rational(1, 10) - S.Rational(3, 10) * X + S.Rational(1, 4) * Y
                        + S.Rational(3, 10) * Z)]
        pi = S.Rational(7, 10) * X - S.Rational(2, 5) * Y + S.Rational(1, 5) * Z
    assert S.simplify(sum(S.diff(u[i], syms[i]) for i in range(dim))) == 0
    return u, pi, syms


def strong_force(prob, u, pi, syms):
    """f = d_t u + div(u (x) u) - div S(Du) + grad pi (Du constant in space, so
    div S(Du) = 0)."""
    d = len(u)
    return [S.diff(u[i], T) + sum(S.diff(u[i] * u[j], syms[j]) for j in range(d))
            + S.diff(pi, syms[i]) for i in range(d)]


@pytest.mark.parametrize("dim,p", [(2, 1.4), (2, 1.8), (3, 1.5)])
def test_linear_solution_with_its_trace_as_data_has_zero_residual(dim, p):
    n = (3, 2) if dim == 2 else (2, 2, 2)
    prob = O.Problem(n=n, p=p, delta=0.1, nu=0.8, nu_inf=0.05, convection=1, tau=0.1,
                     gamma1=10.0, gamma2=10.0)
    u, pi, syms = linear_solution(dim)
    t0 = 0.3
    tn = O.radau_times(prob, t0)
    vels = [nodal(prob, u, t=float(t)) for t in tn]
    lift = np.concatenate(vels)
    lifted = prob.with_(lifting=lift)
    U = np.zeros(prob.nst)
    h = prob.h
    for m in range(prob.nt):
        U[m * prob.ns:m * prob.ns + prob.nv] = vels[m]
        for c in range(prob.num_cells):
            idx = []
            r = c
            for k in range(dim):
                idx.append(r % n[k])
                r //= n[k]
            ctr = {syms[k]: (idx[k] + 0.5) * h[k] for k in range(dim)}
            coef = [float(pi.subs(ctr))] + [float(S.diff(pi, syms[k])) * h[k] for k in range(dim)]
            base = m * prob.ns + prob.nv + (dim + 1) * c
            U[base:base + dim + 1] = coef
    vprev = nodal(prob, u, t=t0)
    f = strong_force(prob, u, pi, syms)
    qp = O.quadrature_points(prob)
    fq = np.zeros((prob.nt, prob.num_cells, 3 ** dim, dim))
    for m, t in enumerate(tn):
        for k in range(dim):
            fk = S.lambdify(syms, f[k].subs(T, float(t)), "numpy")
            fq[m, :, :, k] = np.broadcast_to(fk(*[qp[..., j] for j in range(dim)]),
                                             fq[m, :, :, k].shape)
    load = O.load_vector(prob, fq)
    R = O.residual(lifted, U, vprev=vprev, load=load)
    # the same state without the data is far from a solution
    R0 = O.residual(prob, U, vprev=vprev, load=load)
    assert np.abs(R).max() <= 1e-12 * np.abs(R0).max(), (np.abs(R).max(), np.abs(R0).max())


@pytest.mark.parametrize("conv", [0, 1])
def test_exact_newton_is_derivative_of_residual_with_lifting(conv):
    prob = O.Problem(n=(3, 3), p=1.5, delta=1e-2, nu_inf=1e-3, convection=conv,
                     lin=O.EXACT_NEWTON)
    rng = np.random.default_rng(14)
    lifted = prob.with_(lifting=rng.uniform(-1, 1, prob.nt * prob.nv))
    U = rng.uniform(-1, 1, prob.nst)
    dU = rng.uniform(-1, 1, prob.nst)
    vprev = rng.uniform(-1, 1, prob.nv)
    uk = np.concatenate([U[m * prob.ns:m * prob.ns + prob.nv] for m in range(prob.nt)])
    Jd = O.apply(lifted, uk, dU)
    eps = 1e-6
    fd = -(O.residual(lifted, U + eps * dU, vprev, ulag=uk)
           - O.residual(lifted, U - eps * dU, vprev, ulag=uk)) / (2 * eps)
    assert np.linalg.norm(Jd - fd) <= 1e-7 * np.linalg.norm(Jd)
    # and the lifting changes the Jacobian
    assert np.linalg.norm(Jd - O.apply(prob, uk, dU)) > 1e-6 * np.linalg.norm(Jd)
