"""Pins of the oracle's Vanka smoother, surrogate patches, transfers and V-cycle.

Fixed by mathematics and by statements of the paper (Sec. 6.3, App. C):
* the nested prolongation reproduces every coarse Q2 velocity and P1disc
  pressure field exactly on the fine mesh;
* Galerkin coarse operators of the Newtonian Stokes operator without penalty
  equal the coarse re-discretisation (nested conforming spaces, exact
  quadrature), and P^T M_f P = M_c for the temporal mass part;
* the surrogate patch equals the exact patch when the state is constant in
  time; for a state varying with amplitude s across the slab the difference is
  first order in s (Lemma patch-surrogate (a)) and the spectrum of
  A_K^{-1} A~_K lies in the disc |z-1| <= ||A_K^{-1} E|| (part (b));
* the additive Vanka step is the explicit Schwarz operator
  d + omega sum_K R_K^T A_K^{-1} R_K (r - A d) (eq. stmg-vanka-update) written
  with 0/1 restriction matrices and dense inverses;
* a two-level V-cycle equals its closed-form error-propagation composition.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_2603_28706_amd import inputs


def q2_field(prob, f):
    xs = inputs.node_coordinates(prob.n, prob.lo, prob.hi)
    return f(*xs)


def test_prolongation_reproduces_coarse_fields():
    coarse = O.Problem(n=(2, 3), hi=(1.0, 1.5, 1.0))
    fine = O.Problem(n=(4, 6), hi=(1.0, 1.5, 1.0))
    Ps = O.prolongation_spatial(coarse, fine)
    # a field that is biquadratic on each coarse cell: a global biquadratic
    f0 = lambda x, y: 1 + x * y - 2 * x ** 2 * y ** 2 + y ** 2
    f1 = lambda x, y: x ** 2 - 3 * y + x * y ** 2
    vc = np.concatenate([q2_field(coarse, f0), q2_field(coarse, f1)])
    vf = np.concatenate([q2_field(fine, f0), q2_field(fine, f1)])
    pc = np.zeros(3 * coarse.num_cells)
    for c in range(coarse.num_cells):
        i, j = c % 2, c // 2
        xc, yc = (i + .5) * .5, (j + .5) * .5
        q = lambda x, y: 0.3 + c - 2 * x + 5 * y   # piecewise linear, discontinuous
        pc[3 * c:3 * c + 3] = [q(xc, yc), -2 * .5, 5 * .5]
    pf = np.zeros(3 * fine.num_cells)
    for c in range(fine.num_cells):
        i, j = c % 4, c // 4
        cc = (i // 2) + 2 * (j // 2)
        xc, yc = (i + .5) * .25, (j + .5) * .25
        q = lambda x, y: 0.3 + cc - 2 * x + 5 * y
        pf[3 * c:3 * c + 3] = [q(xc, yc), -2 * .25, 5 * .25]
    got = Ps @ np.concatenate([vc, pc])
    assert np.allclose(got, np.concatenate([vf, pf]), atol=1e-13)


def test_galerkin_equals_rediscretisation_for_newtonian_stokes():
    kw = dict(p=2.0, nu=0.6, nu_inf=0.1, delta=0.5, convection=0, gamma1=0.0, gamma2=0.0)
    coarse = O.Problem(n=(2, 2), **kw)
    fine = O.Problem(n=(4, 4), **kw)
    rng = np.random.default_rng(0)
    Af = O.assemble_slab(fine, [rng.uniform(-1, 1, fine.nv)] * 2)
    Ac = O.assemble_slab(coarse, [rng.uniform(-1, 1, coarse.nv)] * 2)
    P = O.prolongation(coarse, fine)
    G = (P.T @ Af @ P).toarray()
    assert np.abs(G - Ac.toarray()).max() < 1e-12 * np.abs(Ac).max()
    Mf = O.assemble_velocity_mass(fine)
    Mc = O.assemble_velocity_mass(coarse)
    Ps = O.prolongation_spatial(coarse, fine)
    assert np.abs((Ps.T @ Mf @ Ps - Mc).toarray()).max() < 1e-15


def test_surrogate_equals_exact_for_time_constant_state():
    prob = O.Problem(n=(3, 3), p=1.3, delta=1e-3)
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, prob.nv)
    uk = np.concatenate([u, u])
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    As = O.assemble_surrogate(prob, uk)
    assert abs(A - As).max() < 1e-13 * abs(A).max()


def test_surrogate_perturbation_first_order_and_spectrum():
    prob = O.Problem(n=(3, 3), p=1.4, delta=1e-2, tau=0.05)
    rng = np.random.default_rng(2)
    u0 = rng.uniform(-1, 1, prob.nv)
    g = rng.uniform(-1, 1, prob.nv)
    nodes, _ = O.radau_right(1)
    K = 4
    idx = O.cell_patch(prob, K)
    norms = []
    for s in (1e-2, 5e-3, 2.5e-3):
        uk = np.concatenate([u0 + s * t * g for t in nodes])
        AK = O.assemble_slab(prob, O.split_uk(prob, uk)).tocsr()[idx][:, idx].toarray()
        AsK = O.assemble_surrogate(prob, uk).tocsr()[idx][:, idx].toarray()
        E = AsK - AK
        norms.append(np.linalg.norm(E, 2))
        F = np.linalg.solve(AK, E)
        eps = np.linalg.norm(F, 2)
        lam = np.linalg.eigvals(np.linalg.solve(AK, AsK))
        assert np.all(np.abs(lam - 1) <= eps * (1 + 1e-8))
    r1, r2 = norms[0] / norms[1], norms[1] / norms[2]
    assert abs(r1 - 2) < 0.05 and abs(r2 - 2) < 0.05


def test_patch_contains_neighbour_contributions():
    """R_K A R_K^T: the diagonal entry of an interior cell's corner node sums the
    four cells sharing that node."""
    prob = O.Problem(n=(3, 3))
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, prob.nv)
    E = O.element_matrices(prob, u)
    ld = O.local_dofs(prob)
    J = O.assemble_spatial(prob, u).tocsr()
    g = ld[4, 0]                 # local node 0 (lower-left corner) of the centre cell
    cells = [c for c in range(9) if g in ld[c, :9]]
    assert len(cells) == 4
    tot = sum(E[c][list(ld[c]).index(g), list(ld[c]).index(g)] for c in cells)
    assert abs(J[g, g] - tot) < 1e-13 * abs(tot)


def test_vanka_step_is_explicit_schwarz_operator():
    prob = O.Problem(n=(3, 2), p=1.5, delta=1e-2)
    rng = np.random.default_rng(4)
    uk = rng.uniform(-1, 1, prob.nt * prob.nv)
    A = O.assemble_slab(prob, O.split_uk(prob, uk)).toarray()
    patches = O.all_patches(prob)
    r = rng.uniform(-1, 1, prob.nst)
    d = rng.uniform(-1, 1, prob.nst)
    omega = 0.7
    B = np.zeros_like(A)
    for idx in patches:
        R = sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)),
                          shape=(len(idx), prob.nst)).toarray()
        B += R.T @ np.linalg.inv(R @ A @ R.T) @ R
    expect = d + omega * B @ (r - A @ d)
    got = O.vanka_step(sp.csr_matrix(A), O.patch_matrices(sp.csr_matrix(A), patches), patches,
                       r, d, omega)
    assert np.allclose(got, expect, rtol=0, atol=1e-10 * np.abs(expect).max())
    # a solution is a fixed point
    x = rng.uniform(-1, 1, prob.nst)
    got = O.vanka_step(sp.csr_matrix(A), O.patch_matrices(sp.csr_matrix(A), patches), patches,
                       A @ x, x, omega)
    assert np.allclose(got, x, atol=1e-12)


def test_truncated_patches_sizes():
    masks = inputs.truncation_masks((6, 6), seed=7)
    prob = O.Problem(n=(6, 6))
    patches = O.all_patches(prob, masks)
    sizes = sorted({len(p) for p in patches})
    assert set(sizes) <= {30, 34, 38, 42} and 42 in sizes and len(sizes) > 1


def test_two_level_vcycle_matches_closed_form():
    fine = O.Problem(n=(4, 4), p=1.5, delta=1e-2)
    rng = np.random.default_rng(5)
    uk = rng.uniform(-1, 1, fine.nt * fine.nv)
    H = O.build_hierarchy(fine, uk, n_levels=2)
    A = H.A[1].toarray()
    n = A.shape[0]
    omega, nu1, nu2 = 0.5, 2, 1
    B = np.zeros_like(A)
    for AK, idx in zip(H.patch_mats[1], H.patches[1]):
        B[np.ix_(idx, idx)] += np.linalg.inv(AK)
    P = H.P[0].toarray()
    nc = P.shape[1]
    Ac = H.A[0].toarray()
    for i in H.pin:
        Ac[i, :] = 0
        Ac[:, i] = 0
        Ac[i, i] = 1
    Cinv = np.linalg.inv(Ac)
    Z = np.eye(nc)
    Z[H.pin, H.pin] = 0
    C = Cinv @ Z
    S = np.eye(n) - omega * B @ A
    pre = sum(np.linalg.matrix_power(S, i) for i in range(nu1)) @ (omega * B)
    post = sum(np.linalg.matrix_power(S, i) for i in range(nu2)) @ (omega * B)
    # d_pre = pre r; d = d_pre + P C P^T (r - A d_pre); d = S^nu2 d + post r
    V = pre + P @ C @ P.T @ (np.eye(n) - A @ pre)
    V = np.linalg.matrix_power(S, nu2) @ V + post
    r = rng.uniform(-1, 1, n)
    got = O.vcycle(H, r, nu1=nu1, nu2=nu2, omega=omega)
    assert np.allclose(got, V @ r, rtol=0, atol=1e-9 * np.abs(V @ r).max())


def test_coarse_solve_with_pinned_pressure():
    prob = O.Problem(n=(2, 2), p=1.5, delta=1e-2)
    rng = np.random.default_rng(6)
    uk = rng.uniform(-1, 1, prob.nt * prob.nv)
    H = O.build_hierarchy(prob, uk, n_levels=1)
    x = rng.uniform(-1, 1, prob.nst)
    x[H.pin] = 0.0
    r = H.A[0] @ x
    d = O.coarse_solve(H, r)
    assert np.abs(H.A[0] @ d - r).max() < 1e-10 * np.abs(r).max()


@pytest.mark.parametrize("n", [(4, 3), (2, 2, 2)])
def test_local_patch_matrix_equals_restriction_of_the_assembled_operator(n):
    """Patches formed from the neighbouring element matrices only are the
    restriction R_K A R_K^T of the globally assembled slab operator (exact
    and surrogate states, full and truncated patches)."""
    prob = O.Problem(n=n, p=1.3, delta=1e-3, lin=O.MODIFIED_NEWTON)
    uk = inputs.uniform(61, prob.nt * prob.nv)
    masks = inputs.truncation_masks(n, seed=62)
    A = O.assemble_slab(prob, O.split_uk(prob, uk))
    ur = O.representative_velocity(prob, uk)
    As = O.assemble_surrogate(prob, uk)
    for cell in range(prob.num_cells):
        for mask in (None, masks[cell]):
            for Ag, blocks in ((A, O.split_uk(prob, uk)), (As, [ur] * prob.nt)):
                AK, idx = O.local_patch_matrix(prob, blocks, cell, mask)
                ref = Ag.tocsr()[idx][:, idx].toarray()
                assert np.abs(AK - ref).max() <= 1e-14 * np.abs(ref).max(), (cell, mask)


def test_prolongation_reproduces_coarse_fields_3d():
    """3D nested interpolation: a global triquadratic velocity field and a
    piecewise-linear (per coarse cell, discontinuous) pressure are reproduced
    exactly on the refined mesh."""
    coarse = O.Problem(n=(2, 1, 2), hi=(1.0, 0.5, 2.0))
    fine = O.Problem(n=(4, 2, 4), hi=(1.0, 0.5, 2.0))
    Ps = O.prolongation_spatial(coarse, fine)
    fs = [lambda x, y, z: 1 + x * y * z - 2 * x ** 2 * y ** 2 * z ** 2 + z ** 2,
          lambda x, y, z: x ** 2 - 3 * y + x * y ** 2 * z,
          lambda x, y, z: y * z ** 2 - x ** 2 * z + 0.5]
    vc = np.concatenate([q2_field(coarse, f) for f in fs])
    vf = np.concatenate([q2_field(fine, f) for f in fs])

    def pressure(prob, parent):
        h = prob.h
        out = np.zeros(4 * prob.num_cells)
        for c in range(prob.num_cells):
            i, j, k = c % prob.n[0], (c // prob.n[0]) % prob.n[1], c // (prob.n[0] * prob.n[1])
            ctr = [(i + .5) * h[0], (j + .5) * h[1], (k + .5) * h[2]]
            pc = parent(i, j, k)
            q = lambda x, y, z: 0.3 + pc - 2 * x + 5 * y - 1.5 * z
            out[4 * c:4 * c + 4] = [q(*ctr), -2 * h[0], 5 * h[1], -1.5 * h[2]]
        return out

    pcoarse = pressure(coarse, lambda i, j, k: i + 2 * j + 3 * k)
    pfine = pressure(fine, lambda i, j, k: i // 2 + 2 * (j // 2) + 3 * (k // 2))
    got = Ps @ np.concatenate([vc, pcoarse])
    assert np.allclose(got, np.concatenate([vf, pfine]), atol=1e-13)


def test_two_level_vcycle_matches_closed_form_3d():
    """The recursive 3D V-cycle (2^3 -> 1^3) equals the explicit composition
    of smoother, restriction, pinned coarse inverse and prolongation."""
    fine = O.Problem(n=(2, 2, 2), p=1.5, delta=1e-2)
    rng = np.random.default_rng(7)
    uk = rng.uniform(-1, 1, fine.nt * fine.nv)
    H = O.build_hierarchy(fine, uk, n_levels=2)
    A = H.A[1].toarray()
    n = A.shape[0]
    omega, nu1, nu2 = 0.5, 1, 2
    B = np.zeros_like(A)
    for AK, idx in zip(H.patch_mats[1], H.patches[1]):
        B[np.ix_(idx, idx)] += np.linalg.inv(AK)
    P = H.P[0].toarray()
    nc = P.shape[1]
    Ac = H.A[0].toarray()
    for i in H.pin:
        Ac[i, :] = 0
        Ac[:, i] = 0
        Ac[i, i] = 1
    Z = np.eye(nc)
    Z[H.pin, H.pin] = 0
    C = np.linalg.inv(Ac) @ Z
    S = np.eye(n) - omega * B @ A
    pre = sum(np.linalg.matrix_power(S, i) for i in range(nu1)) @ (omega * B)
    post = sum(np.linalg.matrix_power(S, i) for i in range(nu2)) @ (omega * B)
    V = pre + P @ C @ P.T @ (np.eye(n) - A @ pre)
    V = np.linalg.matrix_power(S, nu2) @ V + post
    r = rng.uniform(-1, 1, n)
    got = O.vcycle(H, r, nu1=nu1, nu2=nu2, omega=omega)
    assert np.allclose(got, V @ r, rtol=0, atol=1e-9 * np.abs(V @ r).max())
