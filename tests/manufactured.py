"""Manufactured solution of the convergence test (Sec. 7.1, eq. conv-test):
on [0,1]^2 x [0,1]

    u(x, t)  = sin t (sin^2(pi x) sin(pi y) cos(pi y), -sin(pi x) cos(pi x) sin^2(pi y)),
    pi(x, t) = sin t sin(pi x) cos(pi x) sin(pi y) cos(pi y),

divergence free, zero on the boundary and at t = 0, with the volume force
f = d_t u + div(u (x) u) - div S(D u) + grad pi of eq. (pns-strong) for the
stress law of eq. (constitutive-law), S(D) = (nu_inf + nu (delta^2 +
|D|^2)^((p-2)/2)) D.  f is derived symbolically (sympy) from these
definitions and evaluated with numpy; it is problem data handed to both the
GPU solve and the oracle.  The error measures of Table tab:conv-pns: the
space-time L2 norms of Phi_delta(D u) - Phi_delta(D u_h), eq. (nat-dist),
Phi_delta(A) = (delta^2 + |A|^2)^((p-2)/4) A, and of div u_h, evaluated here
from the discrete slab solutions (Q2 velocity, dG(1) in time on the right
Radau nodes 1/3, 1) with Gauss rules of 4 points per direction in space and in
time on every cell and slab.
"""
import functools

import numpy as np
import sympy as s

X, Y, T = s.symbols("x y t", real=True)
_PI = s.pi
U_EXACT = (s.sin(T) * s.sin(_PI * X) ** 2 * s.sin(_PI * Y) * s.cos(_PI * Y),
           -s.sin(T) * s.sin(_PI * X) * s.cos(_PI * X) * s.sin(_PI * Y) ** 2)
P_EXACT = s.sin(T) * s.sin(_PI * X) * s.cos(_PI * X) * s.sin(_PI * Y) * s.cos(_PI * Y)


def _grad(u):
    return s.Matrix([[s.diff(u[i], v) for v in (X, Y)] for i in range(2)])


@functools.lru_cache(maxsize=None)
def _forcing_funcs(p, delta, nu, nu_inf):
    u = s.Matrix(U_EXACT)
    G = _grad(u)
    D = (G + G.T) / 2
    a2 = sum(D[i, j] ** 2 for i in range(2) for j in range(2))
    eta = nu_inf + nu * (delta ** 2 + a2) ** ((s.Float(p, 30) - 2) / 2)
    S = eta * D
    f = []
    for i in range(2):
        fi = s.diff(u[i], T)
        fi += sum(s.diff(u[i] * u[j], (X, Y)[j]) for j in range(2))
        fi -= sum(s.diff(S[i, j], (X, Y)[j]) for j in range(2))
        fi += s.diff(P_EXACT, (X, Y)[i])
        f.append(fi)
    fx = s.lambdify((X, Y, T), f[0], "numpy")
    fy = s.lambdify((X, Y, T), f[1], "numpy")
    grad = s.lambdify((X, Y, T), [G[0, 0], G[0, 1], G[1, 0], G[1, 1]], "numpy")
    return fx, fy, grad


def forcing(p, delta, nu, nu_inf, x, y, t):
    """f(x, y, t) of eq. (pns-strong) for the exact solution: array [..., 2]."""
    fx, fy, _ = _forcing_funcs(float(p), float(delta), float(nu), float(nu_inf))
    x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
    return np.stack([np.broadcast_to(fx(x, y, t), x.shape),
                     np.broadcast_to(fy(x, y, t), x.shape)], axis=-1)


def exact_pressure(x, y, t):
    return np.sin(t) * np.sin(np.pi * x) * np.cos(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * y)


def exact_velocity(x, y, t):
    su = np.sin(t)
    return np.stack([su * np.sin(np.pi * x) ** 2 * np.sin(np.pi * y) * np.cos(np.pi * y),
                     -su * np.sin(np.pi * x) * np.cos(np.pi * x) * np.sin(np.pi * y) ** 2],
                    axis=-1)


def exact_gradient(x, y, t):
    """grad u, [..., 2, 2] with [i][j] = d u_i / d x_j."""
    _, _, g = _forcing_funcs(1.5, 1e-2, 1.0, 0.0)   # the gradient does not depend on the law
    x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
    vals = [np.broadcast_to(v, x.shape) for v in g(x, y, t)]
    return np.stack(vals, axis=-1).reshape(x.shape + (2, 2))


def gauss_points(n):
    """Gauss-Legendre rule with n points on [0, 1]."""
    gx, gw = np.polynomial.legendre.leggauss(n)
    return 0.5 * (gx + 1.0), 0.5 * gw


def forcing_at_quadrature(p, delta, nu, nu_inf, qpts, times):
    """f at the cell Gauss points (qpts [cells, 9, 2]) for each Radau time:
    [len(times), cells, 9, 2]."""
    return np.stack([forcing(p, delta, nu, nu_inf, qpts[..., 0], qpts[..., 1], t)
                     for t in times])


def _q2(s_, a):
    return [2.0 * (s_ - 0.5) * (s_ - 1.0), -4.0 * s_ * (s_ - 1.0), 2.0 * s_ * (s_ - 0.5)][a]


def _dq2(s_, a):
    return [4.0 * s_ - 3.0, -8.0 * s_ + 4.0, 4.0 * s_ - 1.0][a]


def velocity_gradient_at(n, vel, xi):
    """Gradients of the Q2 velocity field `vel` (2 (2n+1)^2 nodal values,
    component 0 then 1, nodes lexicographic) at the reference points xi
    [m, 2] of every cell of the n x n mesh of the unit square: [cells, m, 2, 2]."""
    h = 1.0 / n
    NX = 2 * n + 1
    nn = NX * NX
    cy, cx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cx, cy = cx.ravel(), cy.ravel()
    out = np.zeros((n * n, xi.shape[0], 2, 2))
    for ay in range(3):
        for ax in range(3):
            node = (2 * cy + ay) * NX + (2 * cx + ax)
            dx = _dq2(xi[:, 0], ax) * _q2(xi[:, 1], ay) / h
            dy = _q2(xi[:, 0], ax) * _dq2(xi[:, 1], ay) / h
            for c in range(2):
                v = vel[c * nn + node][:, None]
                out[:, :, c, 0] += v * dx[None, :]
                out[:, :, c, 1] += v * dy[None, :]
    return out


def phi_delta(A, p, delta):
    a2 = np.sum(A * A, axis=(-2, -1))
    return ((delta ** 2 + a2) ** ((p - 2.0) / 4.0))[..., None, None] * A


def slab_errors(n, U1, U2, t0, tau, p, delta, nq=4):
    """Squared space-time L2 errors of one slab: (||Phi(Du) - Phi(Du_h)||^2,
    ||div u_h||^2) over (t0, t0 + tau) x [0,1]^2, u_h(t) the dG(1)
    interpolation of the velocities U1, U2 at the Radau nodes 1/3, 1."""
    g, w = gauss_points(nq)
    xi = np.stack(np.meshgrid(g, g, indexing="xy"), axis=-1).reshape(-1, 2)
    wq = np.outer(w, w).ravel()
    h = 1.0 / n
    G1 = velocity_gradient_at(n, U1, xi)
    G2 = velocity_gradient_at(n, U2, xi)
    cy, cx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    px = (cx.ravel()[:, None] + xi[None, :, 0]) * h
    py = (cy.ravel()[:, None] + xi[None, :, 1]) * h
    e_phi = 0.0
    e_div = 0.0
    for tt, wt in zip(*gauss_points(nq)):
        l1 = 1.5 * (1.0 - tt)          # Lagrange basis of the Radau nodes 1/3, 1 at tt
        l2 = 1.5 * tt - 0.5
        Gh = l1 * G1 + l2 * G2
        Dh = 0.5 * (Gh + np.swapaxes(Gh, -1, -2))
        Ge = exact_gradient(px, py, t0 + tau * tt)
        De = 0.5 * (Ge + np.swapaxes(Ge, -1, -2))
        diff = phi_delta(De, p, delta) - phi_delta(Dh, p, delta)
        e_phi += wt * tau * h * h * np.sum(wq[None, :] * np.sum(diff ** 2, axis=(-2, -1)))
        div = Gh[..., 0, 0] + Gh[..., 1, 1]
        e_div += wt * tau * h * h * np.sum(wq[None, :] * div ** 2)
    return e_phi, e_div
