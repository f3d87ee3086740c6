"""Pins of the oracle's CIP stabilisation, eq. (scip-def) in Sec. 3.2:
s_CIP(u^; x, v) = sum over interior faces of gamma h_F^2 int_F |u^ . n_F|
[grad x n_F] . [grad v n_F] ds, with the weight lagged at u_k in the Jacobian
of every linearisation (eq. Amu-decomp) and at the state itself in the
residual.

* Sec. 5.2 states the lagged form is symmetric positive semidefinite (an L2(F)
  inner product of identical jumps with a nonnegative weight): checked on the
  assembled matrix, 2D and 3D.
* It vanishes on fields whose gradient is continuous across the faces (global
  biquadratic polynomials are in Q2 and C^1).
* Exact integrals of a field with a kink: u_1 = |x - 1/2| on 2 x 1 cells (jump
  of d_x u_1 = -2 across the face x = 1/2, h_F = 1/2, face length 1) gives
  s(u^; u, u) = gamma (1/2)^2 4 int_F |u^ . n| ds = gamma for u^ = (+-1, 0), and
  gamma / 2 for u^ = (y, 0); likewise across y = 1/2 and in 3D.
* The exact-Newton Jacobian with CIP is the derivative of the residual with
  the CIP weight (and the inflow factor) frozen at u_k.
* The Picard fixed-point identity J_Pic(U) U = -R(U) holds with CIP on.
"""
import numpy as np
import pytest

from oracle import oracle as O


def nodal(prob, f):
    """Nodal values (x fastest) of f(x, y[, z]) on the Q2 nodes."""
    g = [np.linspace(prob.lo[k], prob.hi[k], 2 * prob.n[k] + 1) for k in range(prob.dim)]
    mesh = np.meshgrid(*g, indexing="ij")
    return np.transpose(f(*mesh), tuple(range(prob.dim))[::-1]).ravel()


def velocity(prob, comps):
    return np.concatenate([nodal(prob, c) for c in comps])


def spatial_vec(prob, vel):
    v = np.zeros(prob.ns)
    v[:prob.nv] = vel
    return v


@pytest.mark.parametrize("n", [(3, 3), (4, 2), (2, 2, 2)])
def test_lagged_cip_is_symmetric_positive_semidefinite(n):
    prob = O.Problem(n=n, gamma_cip=1.3)
    rng = np.random.default_rng(11)
    uw = rng.uniform(-1, 1, prob.nv)
    S = O.cip_matrix(prob, uw).toarray()
    assert np.abs(S - S.T).max() <= 1e-14 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-12 * ev.max()
    assert ev.max() > 0.0


@pytest.mark.parametrize("n", [(3, 2), (2, 2, 2)])
def test_cip_vanishes_on_fields_with_continuous_gradient(n):
    prob = O.Problem(n=n, gamma_cip=2.0)
    rng = np.random.default_rng(12)
    uw = rng.uniform(-1, 1, prob.nv)
    S = O.cip_matrix(prob, uw)
    if prob.dim == 2:
        f1 = lambda x, y: 0.3 + x - 2 * y + x * x * y - 0.7 * x * y * y + x * x * y * y
        f2 = lambda x, y: -x * x + 3 * x * y + y * y * x
        v = spatial_vec(prob, velocity(prob, [f1, f2]))
    else:
        f = lambda x, y, z: x * x * y * z - y * y + 2 * x * z * z
        v = spatial_vec(prob, velocity(prob, [f, f, f]))
    assert np.abs(S @ v).max() <= 1e-13 * np.abs(S).max() * np.abs(v).max()


@pytest.mark.parametrize("weight,expect", [((1.0, 0.0), 1.0), ((-1.0, 0.0), 1.0),
                                           ("y", 0.5), ((0.0, 1.0), 0.0)])
def test_cip_of_a_kink_across_a_vertical_face(weight, expect):
    gamma = 0.8
    prob = O.Problem(n=(2, 1), gamma_cip=gamma)
    u = spatial_vec(prob, velocity(prob, [lambda x, y: np.abs(x - 0.5), lambda x, y: 0 * x]))
    if weight == "y":
        uw = velocity(prob, [lambda x, y: y, lambda x, y: 0 * x])
    else:
        uw = velocity(prob, [lambda x, y: 0 * x + weight[0], lambda x, y: 0 * x + weight[1]])
    S = O.cip_matrix(prob, uw)
    assert u @ (S @ u) == pytest.approx(gamma * expect, rel=1e-13, abs=1e-15)


def test_cip_of_a_kink_across_a_horizontal_face_and_in_3d():
    gamma = 1.7
    prob = O.Problem(n=(1, 2), gamma_cip=gamma)
    u = spatial_vec(prob, velocity(prob, [lambda x, y: 0 * x, lambda x, y: np.abs(y - 0.5)]))
    uw = velocity(prob, [lambda x, y: 0 * x, lambda x, y: 0 * x + 2.0])
    assert u @ (O.cip_matrix(prob, uw) @ u) == pytest.approx(gamma * 2.0, rel=1e-13)
    p3 = O.Problem(n=(2, 1, 1), gamma_cip=gamma)
    zero = lambda x, y, z: 0 * x
    u3 = spatial_vec(p3, velocity(p3, [lambda x, y, z: np.abs(x - 0.5), zero, zero]))
    uw3 = velocity(p3, [lambda x, y, z: 0 * x + 1.0, zero, zero])
    assert u3 @ (O.cip_matrix(p3, uw3) @ u3) == pytest.approx(gamma, rel=1e-13)


@pytest.mark.parametrize("conv", [0, 1])
def test_exact_newton_with_cip_is_derivative_of_residual(conv):
    prob = O.Problem(n=(3, 3), p=1.5, delta=1e-2, nu_inf=1e-3, convection=conv,
                     lin=O.EXACT_NEWTON, gamma_cip=0.5)
    rng = np.random.default_rng(13)
    U = rng.uniform(-1, 1, prob.nst)
    dU = rng.uniform(-1, 1, prob.nst)
    vprev = rng.uniform(-1, 1, prob.nv)
    uk = np.concatenate([U[m * prob.ns:m * prob.ns + prob.nv] for m in range(prob.nt)])
    Jd = O.apply(prob, uk, dU)
    eps = 1e-6
    fd = -(O.residual(prob, U + eps * dU, vprev, ulag=uk)
           - O.residual(prob, U - eps * dU, vprev, ulag=uk)) / (2 * eps)
    assert np.linalg.norm(Jd - fd) <= 1e-7 * np.linalg.norm(Jd)
    # the CIP part is not negligible in this check
    J0 = O.apply(prob.with_(gamma_cip=0.0), uk, dU)
    assert np.linalg.norm(Jd - J0) > 1e-3 * np.linalg.norm(Jd)


def test_picard_fixed_point_form_with_cip():
    prob = O.Problem(n=(3, 2), p=1.3, delta=1e-3, lin=O.PICARD, gamma_cip=1.0)
    rng = np.random.default_rng(14)
    U = rng.uniform(-1, 1, prob.nst)
    uk = np.concatenate([U[m * prob.ns:m * prob.ns + prob.nv] for m in range(prob.nt)])
    assert np.allclose(O.apply(prob, uk, U), -O.residual(prob, U), rtol=0, atol=1e-12)
