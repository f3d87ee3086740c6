"""Pins of the oracle's temporal matrices and pointwise constitutive tangents.

Each check is fixed by mathematics or by a statement of the paper, not by
re-typing the oracle's formula:
* right Gauss-Radau rule: textbook nodes, exactness on P_2k and failure on
  P_{2k+1} (Remark "Gauss-Radau quadrature", Sec. 5.2);
* M_t equals the diagonal of the Radau weights (Sec. 5.2);
* K_t + K_t^T = e_last e_last^T + m_t m_t^T (integration by parts) and
  K_t 1 = m_t (partition of unity);
* the stress law is the gradient of its convex potential;
* the exact tangent is the derivative of S (eq. pns-dstress), checked by
  central differences;
* spectrum of the rank-one tangents (App. B, Lemma rankone-tangent;
  eqs. exact-par-eig, ell-exact, local-cond-clip);
* limits of the clipped tangent (s = 1 gives exact Newton, s = 0 Picard) and
  the Newtonian case p = 2 where all three coincide.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def test_radau_k1_nodes_weights():
    nodes, w = O.radau_right(1)
    assert np.allclose(nodes, [1.0 / 3.0, 1.0], atol=1e-15)
    assert np.allclose(w, [0.75, 0.25], atol=1e-15)


def test_radau_k2_textbook_nodes():
    # right Radau, 3 points on [0,1]: (4 -+ sqrt 6)/10 and 1
    nodes, w = O.radau_right(2)
    s6 = np.sqrt(6.0)
    assert np.allclose(nodes, [(4 - s6) / 10, (4 + s6) / 10, 1.0], atol=1e-14)
    assert np.allclose(w, [(16 - s6) / 36, (16 + s6) / 36, 1.0 / 9.0], atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_radau_exactness_degree(k):
    nodes, w = O.radau_right(k)
    for q in range(2 * k + 1):
        assert abs(np.sum(w * nodes ** q) - 1.0 / (q + 1)) < 1e-13
    q = 2 * k + 1
    assert abs(np.sum(w * nodes ** q) - 1.0 / (q + 1)) > 1e-6


def test_radau_k1_fails_on_cubic_by_known_amount():
    nodes, w = O.radau_right(1)
    assert abs(np.sum(w * nodes ** 3) - 5.0 / 18.0) < 1e-15  # exact value is 1/4


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_time_matrices_identities(k):
    nodes, M, K, m = O.time_matrices(k)
    _, w = O.radau_right(k)
    assert np.allclose(M, np.diag(w), atol=1e-14)
    e = np.zeros(k + 1)
    e[-1] = 1.0
    assert np.allclose(K + K.T, np.outer(e, e) + np.outer(m, m), atol=1e-13)
    assert np.allclose(K @ np.ones(k + 1), m, atol=1e-13)
    assert abs(np.sum(K) - 1.0) < 1e-13


def test_time_matrices_k0_backward_euler():
    _, M, K, m = O.time_matrices(0)
    assert np.allclose(M, [[1.0]]) and np.allclose(K, [[1.0]]) and np.allclose(m, [1.0])


def test_time_matrices_k1_values():
    _, M, K, m = O.time_matrices(1)
    assert np.allclose(K, [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-14)
    assert np.allclose(m, [1.5, -0.5], atol=1e-14)
    # eigenvalues of M^{-1} K are 2 +- sqrt(2) i
    ev = np.sort_complex(np.linalg.eigvals(np.linalg.solve(M, K)))
    assert np.allclose(ev, [2 - np.sqrt(2) * 1j, 2 + np.sqrt(2) * 1j], atol=1e-12)


def test_midpoint_weights():
    nodes, _ = O.radau_right(1)
    assert np.allclose([O.lagrange(nodes, m, np.array([0.5]))[0] for m in range(2)], [0.75, 0.25])


# ------------------------------------------------------------------ tangents

def rand_sym(rng, d, scale=1.0):
    A = rng.normal(size=(d, d)) * scale
    return 0.5 * (A + A.T)


PARAMS = [
    dict(p=1.5, delta=1e-2, nu=1.0, nu_inf=1e-3),
    dict(p=1.2, delta=1e-4, nu=1.0, nu_inf=1e-4),
    dict(p=1.1, delta=1e-5, nu=0.7, nu_inf=0.0),
    dict(p=1.9, delta=0.3, nu=2.0, nu_inf=0.5),
]


def potential(pr, A):
    a2 = np.sum(A * A)
    return 0.5 * pr["nu_inf"] * a2 + pr["nu"] / pr["p"] * (pr["delta"] ** 2 + a2) ** (pr["p"] / 2)


@pytest.mark.parametrize("pr", PARAMS)
@pytest.mark.parametrize("d", [2, 3])
def test_stress_is_gradient_of_potential(pr, d):
    rng = np.random.default_rng(1)
    prob = O.Problem(n=(1,) * d, **pr)
    for _ in range(5):
        A = rand_sym(rng, d)
        S = O.stress(prob, A)
        G = np.zeros_like(A)
        eps = 1e-6
        for i, j in itertools.product(range(d), range(d)):
            E = np.zeros_like(A)
            E[i, j] = 1.0
            G[i, j] = (potential(pr, A + eps * E) - potential(pr, A - eps * E)) / (2 * eps)
        assert np.linalg.norm(S - G) <= 1e-7 * np.linalg.norm(S)


@pytest.mark.parametrize("pr", PARAMS)
@pytest.mark.parametrize("d", [2, 3])
def test_exact_tangent_is_derivative_of_stress(pr, d):
    rng = np.random.default_rng(2)
    prob = O.Problem(n=(1,) * d, **pr)
    for scale in (1e-3, 1.0, 30.0):
        A = rand_sym(rng, d, scale)
        B = rand_sym(rng, d)
        T = O.tangent(prob, O.EXACT_NEWTON, A, B)
        eps = 1e-5 * scale
        fd = (O.stress(prob, A + eps * B) - O.stress(prob, A - eps * B)) / (2 * eps)
        assert np.linalg.norm(T - fd) <= 1e-7 * np.linalg.norm(T)


def sym_basis(d):
    out = []
    for i in range(d):
        E = np.zeros((d, d))
        E[i, i] = 1.0
        out.append(E)
    for i in range(d):
        for j in range(i + 1, d):
            E = np.zeros((d, d))
            E[i, j] = E[j, i] = np.sqrt(0.5)
            out.append(E)
    return out


def tangent_matrix(prob, kind, A):
    basis = sym_basis(A.shape[0])
    return np.array([[np.sum(O.tangent(prob, kind, A, Bj) * Bi) for Bj in basis] for Bi in basis])


@pytest.mark.parametrize("pr", PARAMS)
@pytest.mark.parametrize("d", [2, 3])
def test_exact_tangent_spectrum_and_bounds(pr, d):
    rng = np.random.default_rng(3)
    prob = O.Problem(n=(1,) * d, **pr)
    p, delta, nu, nuinf = pr["p"], pr["delta"], pr["nu"], pr["nu_inf"]
    for scale in (1e-2, 1.0, 10.0):
        A = rand_sym(rng, d, scale)
        r2 = np.sum(A * A)
        D2 = delta ** 2 + r2
        mu = nu * D2 ** ((p - 2) / 2)
        eta = nuinf + mu
        lam_par = nuinf + mu * (delta ** 2 + (p - 1) * r2) / D2        # eq. (exact-par-eig)
        Tm = tangent_matrix(prob, O.EXACT_NEWTON, A)
        assert np.allclose(Tm, Tm.T, atol=1e-12 * np.abs(Tm).max())
        ev = np.sort(np.linalg.eigvalsh(Tm))
        n = len(ev)
        expect = np.sort([eta] * (n - 1) + [lam_par])
        assert np.allclose(ev, expect, rtol=1e-10, atol=0)
        lo, hi = nuinf + (p - 1) * mu, nuinf + mu                       # eq. (ell-exact)
        assert ev[0] >= lo * (1 - 1e-12) and ev[-1] <= hi * (1 + 1e-12)


@pytest.mark.parametrize("pr", PARAMS)
def test_clipped_tangent_limits_and_spectrum(pr):
    rng = np.random.default_rng(4)
    d = 2
    base = O.Problem(n=(1, 1), **pr)
    for _ in range(4):
        A = rand_sym(rng, d, 3.0)
        B = rand_sym(rng, d)
        big = base.with_(sigma_max=1e300)
        zero = base.with_(sigma_max=0.0)
        assert np.allclose(O.tangent(big, O.MODIFIED_NEWTON, A, B),
                           O.tangent(big, O.EXACT_NEWTON, A, B), rtol=1e-14, atol=0)
        assert np.allclose(O.tangent(zero, O.MODIFIED_NEWTON, A, B),
                           O.tangent(zero, O.PICARD, A, B), rtol=1e-14, atol=0)
        # intermediate clip: parallel eigenvalue eta + s theta |sigma|^2, eq. (local-tangent-clip)
        p, delta, nu, nuinf = pr["p"], pr["delta"], pr["nu"], pr["nu_inf"]
        r2 = np.sum(A * A)
        D2 = delta ** 2 + r2
        mu = nu * D2 ** ((p - 2) / 2)
        sig = mu * np.sqrt(r2)
        smax = 0.3 * sig
        s = smax / sig
        pm = base.with_(sigma_max=smax)
        ev = np.sort(np.linalg.eigvalsh(tangent_matrix(pm, O.MODIFIED_NEWTON, A)))
        eta = nuinf + mu
        theta = (p - 2) / (mu * D2)
        lam_par = eta + s * theta * sig ** 2
        assert np.allclose(ev, np.sort([eta, eta, lam_par]), rtol=1e-10)
        # for |A| >> delta the smallest eigenvalue is nu_inf + (1 - s(2-p)) mu, eq. (local-cond-clip)
        if delta ** 2 < 1e-6 * r2:
            assert abs(lam_par - (nuinf + (1 - s * (2 - p)) * mu)) <= 1e-5 * eta


def test_clipped_tangent_zero_state():
    prob = O.Problem(n=(1, 1), p=1.3, delta=1e-3, nu=1.0, nu_inf=1e-3, sigma_max=1.0)
    A = np.zeros((2, 2))
    B = np.array([[0.3, -0.2], [-0.2, 0.7]])
    eta0 = 1e-3 + 1e-3 ** (1.3 - 2)
    for kind in (O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON):
        assert np.allclose(O.tangent(prob, kind, A, B), eta0 * B, rtol=1e-14)


@pytest.mark.parametrize("d", [2, 3])
def test_newtonian_case_all_tangents_coincide(d):
    rng = np.random.default_rng(5)
    prob = O.Problem(n=(1,) * d, p=2.0, delta=0.1, nu=0.8, nu_inf=0.3, sigma_max=0.5)
    for _ in range(3):
        A = rand_sym(rng, d, 5.0)
        B = rand_sym(rng, d)
        for kind in (O.PICARD, O.EXACT_NEWTON, O.MODIFIED_NEWTON):
            assert np.allclose(O.tangent(prob, kind, A, B), 1.1 * B, rtol=1e-14)
