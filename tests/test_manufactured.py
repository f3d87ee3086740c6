"""Pins of the manufactured-solution data of the convergence test (Sec. 7.1,
eq. conv-test): the exact velocity is divergence free and vanishes on the
boundary and at t = 0; the symbolic force f satisfies eq. (pns-strong) when
every derivative is replaced by central differences of the closed forms (an
independent numerical route, catching a dropped term or sign in the symbolic
derivation); the gradient matches differences of the velocity; the error
quadrature of `slab_errors` integrates a known field exactly; and the oracle's
load vector F = tau w (f, phi) equals tau w M_x I(f) for f in Q2 (the 3-point
Gauss rule integrates Q2 x Q2 exactly), with zero pressure rows."""
import numpy as np
import pytest

import manufactured as mf
from oracle import oracle as O


def fd(fun, x, y, t, k, h=1e-5):
    e = [0.0, 0.0, 0.0]
    e[k] = h
    return (fun(x + e[0], y + e[1], t + e[2]) - fun(x - e[0], y - e[1], t - e[2])) / (2 * h)


def test_exact_solution_properties():
    rng = np.random.default_rng(3)
    x, y, t = rng.random(50), rng.random(50), rng.random()
    div = fd(lambda a, b, c: mf.exact_velocity(a, b, c)[..., 0], x, y, t, 0) + \
        fd(lambda a, b, c: mf.exact_velocity(a, b, c)[..., 1], x, y, t, 1)
    assert np.abs(div).max() < 1e-8
    s = np.linspace(0, 1, 11)
    for bx, by in ((s, 0 * s), (s, 0 * s + 1), (0 * s, s), (0 * s + 1, s)):
        assert np.abs(mf.exact_velocity(bx, by, 0.7)).max() < 1e-15
    assert np.abs(mf.exact_velocity(x, y, 0.0)).max() == 0.0
    G = mf.exact_gradient(x, y, t)
    for i in range(2):
        for j in range(2):
            g = fd(lambda a, b, c: mf.exact_velocity(a, b, c)[..., i], x, y, t, j)
            assert np.abs(G[..., i, j] - g).max() < 1e-8


@pytest.mark.parametrize("p,delta,nu,nu_inf", [(1.5, 1e-2, 1e-2, 1e-5), (1.25, 1e-1, 1e-2, 0.0),
                                               (2.0, 1e-3, 0.1, 0.0)])
def test_forcing_satisfies_the_strong_form(p, delta, nu, nu_inf):
    """d_t u + div(u (x) u) - div S(Du) + grad pi - f = 0 by central
    differences (nested for the stress divergence) of the closed forms; the
    regularisation keeps S smooth for these delta."""
    rng = np.random.default_rng(5)
    x, y, t = 0.1 + 0.8 * rng.random(20), 0.1 + 0.8 * rng.random(20), 0.3 + 0.5 * rng.random()
    vel = mf.exact_velocity

    def grad_fd(a, b, c, h=1e-6):
        return np.stack([np.stack([fd(lambda aa, bb, cc: vel(aa, bb, cc)[..., i], a, b, c, j, h)
                                   for j in range(2)], -1) for i in range(2)], -2)

    def stress(a, b, c):
        G = grad_fd(a, b, c)
        D = 0.5 * (G + np.swapaxes(G, -1, -2))
        a2 = np.sum(D * D, axis=(-2, -1))
        return (nu_inf + nu * (delta ** 2 + a2) ** ((p - 2) / 2))[..., None, None] * D

    got = mf.forcing(p, delta, nu, nu_inf, x, y, t)
    for i in range(2):
        r = fd(lambda a, b, c: vel(a, b, c)[..., i], x, y, t, 2)
        for j in range(2):
            r = r + fd(lambda a, b, c: vel(a, b, c)[..., i] * vel(a, b, c)[..., j], x, y, t, j)
            r = r - fd(lambda a, b, c: stress(a, b, c)[..., i, j], x, y, t, j, h=1e-4)
        r = r + fd(mf.exact_pressure, x, y, t, i)
        scale = np.abs(got[..., i]).max()
        assert np.abs(r - got[..., i]).max() <= 1e-5 * max(scale, 1.0), (i, np.abs(r - got[..., i]).max())


def test_slab_error_quadrature_is_exact_for_a_polynomial_field():
    """With u_h = 0 and p = 2 (Phi = identity) the natural-distance error of a
    slab is ||D u||^2 of the exact solution; compare with a much finer rule."""
    n = 4
    U0 = np.zeros(2 * (2 * n + 1) ** 2)
    e4, d4 = mf.slab_errors(n, U0, U0, 0.2, 0.1, 2.0, 0.0, nq=4)
    e8, d8 = mf.slab_errors(n, U0, U0, 0.2, 0.1, 2.0, 0.0, nq=8)
    assert d4 == 0.0 and d8 == 0.0
    assert e4 == pytest.approx(e8, rel=1e-4)


def test_dg1_interpolation_of_a_linear_in_time_q2_field_has_zero_error():
    """A field that is Q2 in space and linear in time is represented exactly by
    its values at the Radau nodes: the discrete gradient of slab_errors equals
    the nodal field's gradient at every time (checked through div of a known
    Q2 field: u = (x^2, -2 x y) has div 0)."""
    n = 3
    NX = 2 * n + 1
    g = np.linspace(0, 1, NX)
    xx, yy = np.meshgrid(g, g, indexing="xy")
    u = np.concatenate([(xx ** 2).ravel(), (-2 * xx * yy).ravel()])
    _, d = mf.slab_errors(n, u, 2 * u, 0.0, 0.5, 2.0, 0.0)
    assert d < 1e-28


@pytest.mark.parametrize("n", [(3, 2), (4, 4)])
def test_load_vector_equals_mass_times_interpolant_for_q2_forces(n):
    prob = O.Problem(n=n, tau=0.05)
    qp = O.quadrature_points(prob)
    rng = np.random.default_rng(7)
    c = rng.standard_normal((2, 2, 9))      # biquadratic coefficients per (mu, comp)

    def fq2(mu, comp, x, y):
        k = c[mu, comp]
        return sum(k[3 * j + i] * x ** i * y ** j for i in range(3) for j in range(3))

    f_qp = np.zeros((2, prob.num_cells, 9, 2))
    for mu in range(2):
        for comp in range(2):
            f_qp[mu, :, :, comp] = fq2(mu, comp, qp[..., 0], qp[..., 1])
    F = O.load_vector(prob, f_qp)
    NX, NY = 2 * n[0] + 1, 2 * n[1] + 1
    gx, gy = np.meshgrid(np.linspace(0, 1, NX), np.linspace(0, 1, NY), indexing="xy")
    M = O.assemble_velocity_mass(prob).tocsr()
    _, w = O.radau_right(1)
    for mu in range(2):
        interp = np.zeros(prob.ns)
        for comp in range(2):
            interp[comp * prob.num_nodes:(comp + 1) * prob.num_nodes] = fq2(mu, comp, gx, gy).ravel()
        want = prob.tau * w[mu] * (M @ interp)
        got = F[mu * prob.ns:(mu + 1) * prob.ns]
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
        assert np.all(got[prob.nv:] == 0.0)
