"""Plain FP64 CPU oracle for the space-time (p,delta)-Navier-Stokes smoothing step.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package,
and it shares no code with the HIP path.  The element-level arithmetic is plain
C in ``pns_oracle.c`` (per-cell quadrature loops, no sum factorisation); this
module adds the global pieces with numpy / scipy library primitives:

* right Gauss-Radau nodes and the temporal matrices M_t, K_t, m_t
  (Sec. 3.1 "Gauss-Radau temporal nodes", Sec. 5.2 definitions of M_t, K_t, m_t);
* assembled spatial blocks J_mu and the slab Jacobian J_n,
  eq. (slab-underint-jac);
* Vanka cell patches, the exact patch matrices R_K A R_K^T and the finest-level
  surrogate patches with coefficients frozen at the slab midpoint,
  eq. (surrogate-diag) (Sec. 6.3);
* one additive Vanka smoothing step, eq. (stmg-vanka-update);
* the nested Q2 / P1disc prolongation, Galerkin coarse operators
  A_l = P^T A_{l+1} P (Sec. 6.3 "Hierarchy and coarse operators") and the
  V-cycle with a dense LU on the coarsest level;
* the block mass-weighted residual norm and a plain Newton iteration on the
  slab residual with direct (sparse LU) linear solves and Armijo backtracking
  (Sec. 6.1 "Krylov solver and preconditioning", Sec. 6.2 "Globalization and
  stopping criteria"), which defines the solution a slab solve has to reach.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field as dcfield

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

PICARD, EXACT_NEWTON, MODIFIED_NEWTON = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "pns_oracle.c")


def build(verbose: bool = False) -> str:
    """Compile the C part of the oracle (plain gcc, -O2, no fast-math)."""
    import subprocess

    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", SRC_PATH, "-o", LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _CProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("nt", ctypes.c_int), ("kt", ctypes.c_double * 16),
        ("wt", ctypes.c_double * 4), ("mt", ctypes.c_double * 4),
        ("tau", ctypes.c_double),
        ("p", ctypes.c_double), ("delta", ctypes.c_double),
        ("nu", ctypes.c_double), ("nu_inf", ctypes.c_double),
        ("gamma1", ctypes.c_double), ("gamma2", ctypes.c_double),
        ("sigma_max", ctypes.c_double),
        ("convection", ctypes.c_int), ("qsign", ctypes.c_int), ("lin", ctypes.c_int),
        ("gamma_cip", ctypes.c_double),
        ("ghat", ctypes.c_void_p), ("gnode", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_CProblem)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        for name, args in [
            ("orc_num_nodes", [P]), ("orc_num_cells", [P]),
            ("orc_spatial_size", [P]), ("orc_local_size", [P]),
        ]:
            getattr(L, name).argtypes = args
            getattr(L, name).restype = ctypes.c_int
        L.orc_stress.argtypes = [P, dp, dp]
        L.orc_tangent.argtypes = [P, ctypes.c_int, dp, dp, dp]
        L.orc_local_dofs.argtypes = [P, ctypes.c_int, ip]
        L.orc_element_matrix.argtypes = [P, ctypes.c_int, dp, dp]
        L.orc_element_mass.argtypes = [P, ctypes.c_int, dp]
        L.orc_all_element_matrices.argtypes = [P, dp, dp]
        L.orc_apply.argtypes = [P, dp, dp, dp]
        L.orc_apply_threads.argtypes = [P, dp, dp, dp, ctypes.c_int]
        L.orc_element_form.argtypes = [P, ctypes.c_int, dp, dp, dp, dp]
        L.orc_element_lift.argtypes = [P, ctypes.c_int, dp]
        L.orc_residual.argtypes = [P, dp, dp, dp, dp]
        L.orc_load.argtypes = [P, dp, dp]
        L.orc_cip_count.argtypes = [P]
        L.orc_cip_count.restype = ctypes.c_int
        L.orc_cip_face.argtypes = [P, dp, ctypes.c_int, ip, dp]
        L.orc_cip_face.restype = None
        for f in ("orc_stress", "orc_tangent", "orc_local_dofs", "orc_element_matrix",
                  "orc_element_mass", "orc_all_element_matrices", "orc_apply",
                  "orc_apply_threads", "orc_element_form", "orc_element_lift", "orc_residual",
                  "orc_load"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ time

def radau_right(k: int):
    """Right-sided (k+1)-point Gauss-Radau rule on [0,1] (Sec. 3.1): the nodes are
    the roots of P_{k+1} - P_k on [-1,1] (which include +1), mapped to [0,1];
    weights integrate the nodal Lagrange basis exactly."""
    from numpy.polynomial import legendre as L

    if k == 0:
        return np.array([1.0]), np.array([1.0])
    c = np.zeros(k + 2)
    c[k + 1] = 1.0
    c[k] = -1.0
    r = np.sort(np.real(L.legroots(c)))
    nodes = 0.5 * (r + 1.0)
    nodes[-1] = 1.0
    gx, gw = L.leggauss(k + 2)
    gx = 0.5 * (gx + 1.0)
    gw = 0.5 * gw
    w = np.array([np.sum(gw * lagrange(nodes, i, gx)) for i in range(k + 1)])
    return nodes, w


def lagrange(nodes, i, t):
    t = np.asarray(t, dtype=np.float64)
    v = np.ones_like(t)
    for j, tj in enumerate(nodes):
        if j != i:
            v = v * (t - tj) / (nodes[i] - tj)
    return v


def lagrange_der(nodes, i, t):
    t = np.asarray(t, dtype=np.float64)
    tot = np.zeros_like(t)
    for m, tm in enumerate(nodes):
        if m == i:
            continue
        v = np.ones_like(t) / (nodes[i] - tm)
        for j, tj in enumerate(nodes):
            if j != i and j != m:
                v = v * (t - tj) / (nodes[i] - tj)
        tot = tot + v
    return tot


def time_matrices(k: int):
    """Reference M_t, K_t, m_t of Sec. 5.2:
    (M_t)_ij = int xi_j xi_i, (K_t)_ij = int xi_j' xi_i + xi_j(0) xi_i(0),
    (m_t)_i = xi_i(0), with xi the Radau Lagrange basis.  Integrals by a
    Gauss-Legendre rule exact for the polynomial degree involved."""
    from numpy.polynomial import legendre as L

    nodes, _ = radau_right(k)
    n = k + 1
    gx, gw = L.leggauss(k + 2)
    gx = 0.5 * (gx + 1.0)
    gw = 0.5 * gw
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    m = np.zeros(n)
    for i in range(n):
        xi_i = lagrange(nodes, i, gx)
        m[i] = lagrange(nodes, i, np.array([0.0]))[0]
        for j in range(n):
            M[i, j] = np.sum(gw * lagrange(nodes, j, gx) * xi_i)
            K[i, j] = (np.sum(gw * lagrange_der(nodes, j, gx) * xi_i)
                       + lagrange(nodes, j, np.array([0.0]))[0] * m[i])
    return nodes, M, K, m


# --------------------------------------------------------------- problem

@dataclass
class Problem:
    """Mesh, discretisation and model of one slab (uniform box mesh, Q2/P1disc x dG(k))."""
    n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    k_time: int = 1
    tau: float = 0.01
    p: float = 1.5
    delta: float = 1e-2
    nu: float = 1.0
    nu_inf: float = 1e-3
    gamma1: float = 40.0
    gamma2: float = 40.0
    sigma_max: float = 1.0
    convection: int = 1
    qsign: int = 1
    lin: int = MODIFIED_NEWTON
    gamma_cip: float = 0.0
    # Dirichlet lifting ghat_D (eq. def-b-gam): a Q2 velocity field per Radau
    # node, nt * nv values; its trace is g_D.  None: homogeneous data.
    lifting: object = dcfield(default=None, repr=False, compare=False)
    _c: object = dcfield(default=None, repr=False, compare=False)

    @property
    def dim(self):
        return len(self.n)

    def cstruct(self, **override) -> _CProblem:
        fields = dict(self.__dict__)
        fields.update(override)
        s = _CProblem()
        d = len(fields["n"])
        s.dim = d
        for k in range(3):
            s.n[k] = fields["n"][k] if k < d else 1
            s.lo[k] = fields["lo"][k]
            s.hi[k] = fields["hi"][k]
        _, M, K, m = time_matrices(fields["k_time"])
        nt = fields["k_time"] + 1
        s.nt = nt
        for i in range(nt):
            s.wt[i] = M[i, i]
            s.mt[i] = m[i]
            for j in range(nt):
                s.kt[i * nt + j] = K[i, j]
        s.tau = fields["tau"]
        for name in ("p", "delta", "nu", "nu_inf", "gamma1", "gamma2", "sigma_max", "gamma_cip"):
            setattr(s, name, float(fields[name]))
        s.convection = int(fields["convection"])
        s.qsign = int(fields["qsign"])
        s.lin = int(fields["lin"])
        lift = fields.get("lifting")
        if lift is not None:
            # the array stays referenced by the Problem for the call's lifetime
            assert lift.dtype == np.float64 and lift.flags.c_contiguous
            assert lift.size == nt * d * int(np.prod([2 * m + 1 for m in fields["n"]]))
            s.ghat = lift.ctypes.data
        return s

    def with_(self, **kw) -> "Problem":
        d = {k: v for k, v in self.__dict__.items() if k != "_c"}
        d.update(kw)
        if d.get("lifting") is not None:
            d["lifting"] = _f64(d["lifting"])
        return Problem(**d)

    def __post_init__(self):
        if self.lifting is not None:
            self.lifting = _f64(self.lifting)

    # sizes
    @property
    def nt(self):
        return self.k_time + 1

    @property
    def num_nodes(self):
        return int(np.prod([2 * m + 1 for m in self.n]))

    @property
    def num_cells(self):
        return int(np.prod(self.n))

    @property
    def nv(self):
        return self.dim * self.num_nodes

    @property
    def ns(self):
        return self.nv + (self.dim + 1) * self.num_cells

    @property
    def nst(self):
        return self.nt * self.ns

    @property
    def nloc(self):
        return self.dim * 3 ** self.dim + self.dim + 1

    @property
    def h(self):
        return tuple((self.hi[k] - self.lo[k]) / self.n[k] for k in range(self.dim))


def _cs(prob: Problem, gnode=None, **kw):
    """C view of the problem; `gnode`: the lifting of the one time node an
    element-level routine works on (d * num_nodes values, kept alive by the
    caller), None: zero."""
    s = prob.cstruct(**kw)
    if gnode is not None:
        assert gnode.dtype == np.float64 and gnode.flags.c_contiguous and gnode.size == prob.nv
        s.gnode = gnode.ctypes.data
    return ctypes.byref(s)


def lifting_blocks(prob: Problem):
    """The lifting of every Radau node (None for homogeneous data)."""
    if prob.lifting is None:
        return [None] * prob.nt
    return [np.ascontiguousarray(prob.lifting[m * prob.nv:(m + 1) * prob.nv])
            for m in range(prob.nt)]


# ------------------------------------------------------- pointwise (L0)

def stress(prob: Problem, A):
    A = _f64(A)
    S = np.zeros_like(A)
    lib().orc_stress(_cs(prob), _dp(A), _dp(S))
    return S


def tangent(prob: Problem, kind: int, A, B):
    A = _f64(A)
    B = _f64(B)
    T = np.zeros_like(B)
    lib().orc_tangent(_cs(prob), int(kind), _dp(A), _dp(B), _dp(T))
    return T


# ------------------------------------------------------------ elements

def local_dofs(prob: Problem):
    """(num_cells, nloc) spatial indices: velocity comp c / node a at c*3^d+a,
    then the d+1 pressure coefficients."""
    out = np.zeros((prob.num_cells, prob.nloc), dtype=np.int32)
    cs = _cs(prob)
    for c in range(prob.num_cells):
        lib().orc_local_dofs(cs, c, out[c].ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def element_matrices(prob: Problem, u_spatial, g_spatial=None, **kw):
    """All cell matrices of J_mu at velocity state u (length d*num_nodes), the
    Nitsche coefficients frozen at the lifting g_spatial of the same time node
    (None: zero)."""
    u = _f64(u_spatial)
    assert u.size == prob.nv
    g = _f64(g_spatial) if g_spatial is not None else None
    E = np.zeros((prob.num_cells, prob.nloc, prob.nloc))
    lib().orc_all_element_matrices(_cs(prob, gnode=g, **kw), _dp(u), _dp(E))
    return E


def element_mass(prob: Problem, cell: int = 0):
    nb = 3 ** prob.dim
    M = np.zeros((nb, nb))
    lib().orc_element_mass(_cs(prob), int(cell), _dp(M))
    return M


def cip_matrix(prob: Problem, u_weight):
    """Assembled CIP form of eq. (scip-def) on the interior faces, s_CIP(uw; x, v)
    (ns x ns, CSR, zero outside the velocity block), with the weight field
    uw (one time node's velocity, d * num_nodes values) and gamma_CIP of prob."""
    u_weight = _f64(u_weight)
    cs = _cs(prob)
    nf = lib().orc_cip_count(cs)
    nl = 2 * prob.dim * 3 ** prob.dim
    dofs = np.zeros(nl, dtype=np.int32)
    M = np.zeros((nl, nl))
    rows, cols, vals = [], [], []
    for f in range(nf):
        lib().orc_cip_face(cs, _dp(u_weight), f, dofs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           _dp(M))
        rows.append(np.repeat(dofs, nl))
        cols.append(np.tile(dofs, nl))
        vals.append(M.ravel().copy())
    if not rows:
        return sp.csr_matrix((prob.ns, prob.ns))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(prob.ns, prob.ns))


def assemble_spatial(prob: Problem, u_spatial, g_spatial=None, **kw):
    """Assembled spatial block J_mu (ns x ns, CSR) at velocity state u: the
    element matrices (Nitsche coefficients frozen at the lifting g_spatial)
    plus, with gamma_CIP > 0, the CIP form with its weight lagged at u
    (eq. Amu-decomp)."""
    E = element_matrices(prob, u_spatial, g_spatial, **kw)
    dofs = local_dofs(prob)
    rows = np.repeat(dofs, prob.nloc, axis=1).ravel()
    cols = np.tile(dofs, (1, prob.nloc)).ravel()
    J = sp.csr_matrix((E.ravel(), (rows, cols)), shape=(prob.ns, prob.ns))
    pk = prob.with_(**kw) if kw else prob
    if pk.gamma_cip > 0.0:
        J = J + cip_matrix(pk, u_spatial)
    return J


def assemble_velocity_mass(prob: Problem):
    """Velocity mass M_x embedded in the spatial (ns x ns) layout."""
    nb = 3 ** prob.dim
    dofs = local_dofs(prob)
    cs = _cs(prob)
    Me = np.zeros((prob.num_cells, nb, nb))
    for c in range(prob.num_cells):
        lib().orc_element_mass(cs, int(c), _dp(Me[c]))
    rows, cols, vals = [], [], []
    for comp in range(prob.dim):
        idx = dofs[:, comp * nb:(comp + 1) * nb]          # (cells, nb)
        rows.append(np.repeat(idx, nb, axis=1).ravel())   # row a repeated for every column b
        cols.append(np.tile(idx, (1, nb)).ravel())
        vals.append(Me.reshape(prob.num_cells, nb * nb).ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(prob.ns, prob.ns))


def assemble_slab(prob: Problem, uk_blocks, g_blocks=None, **kw):
    """J_n = [K_t (x) M_x, 0; 0, 0] + (tau M_t (x) I) diag(J_1..J_{k+1}),
    eq. (slab-underint-jac).  uk_blocks: nt velocity states; g_blocks: the
    lifting per time node (default: the problem's)."""
    _, Mt, Kt, _ = time_matrices(prob.k_time)
    Mx = assemble_velocity_mass(prob)
    if g_blocks is None:
        g_blocks = lifting_blocks(prob)
    Js = [assemble_spatial(prob, uk_blocks[m], g_blocks[m], **kw) for m in range(prob.nt)]
    blocks = [[None] * prob.nt for _ in range(prob.nt)]
    for i in range(prob.nt):
        for j in range(prob.nt):
            B = Kt[i, j] * Mx
            if i == j:
                B = B + prob.tau * Mt[i, i] * Js[i]
            blocks[i][j] = B
    return sp.bmat(blocks, format="csr")


def split_uk(prob: Problem, uk):
    uk = _f64(uk)
    return [uk[m * prob.nv:(m + 1) * prob.nv] for m in range(prob.nt)]


# ------------------------------------------------------------- actions

def apply(prob: Problem, uk, x, **kw):
    """Matrix-free oracle action y = J_n(u_k) x (element matrices built per cell)."""
    uk = _f64(uk)
    x = _f64(x)
    assert uk.size == prob.nt * prob.nv and x.size == prob.nst
    y = np.zeros(prob.nst)
    lib().orc_apply(_cs(prob, **kw), _dp(uk), _dp(x), _dp(y))
    return y


def apply_threads(prob: Problem, uk, x, nthreads, **kw):
    """The oracle action of `apply` on `nthreads` host threads (cells visited in
    parity classes; per-cell arithmetic unchanged).  Used to time the oracle on
    every core of the host."""
    uk = _f64(uk)
    x = _f64(x)
    assert uk.size == prob.nt * prob.nv and x.size == prob.nst
    y = np.zeros(prob.nst)
    lib().orc_apply_threads(_cs(prob, **kw), _dp(uk), _dp(x), _dp(y), int(nthreads))
    return y


def quadrature_points(prob: Problem):
    """Physical coordinates of the volume Gauss points (3 per direction) of
    every cell: array [cells, 3^d, d], cells lexicographic (x fastest), points
    q = qx + 3 qy (+ 9 qz)."""
    d = prob.dim
    g = 0.5 - np.sqrt(3.0 / 5.0) / 2.0
    gp = np.array([g, 0.5, 1.0 - g])
    h = [(prob.hi[k] - prob.lo[k]) / prob.n[k] for k in range(d)]
    cells = np.indices(prob.n[::-1]).reshape(d, -1)[::-1].T      # (cx, cy[, cz]), x fastest
    qs = np.indices((3,) * d).reshape(d, -1)[::-1].T                # (qx, qy[, qz]), qx fastest
    out = np.zeros((cells.shape[0], 3 ** d, d))
    for k in range(d):
        out[:, :, k] = prob.lo[k] + h[k] * (cells[:, k][:, None] + gp[qs[:, k]][None, :])
    return out


def radau_times(prob: Problem, t0: float):
    """Times of the Gauss-Radau nodes of the slab (t0, t0 + tau]."""
    t, _ = radau_right(prob.k_time)
    return t0 + prob.tau * np.asarray(t)


def load_vector(prob: Problem, f_qp):
    """F_v,mu = tau w_mu (f(t_mu), phi)_Omega (Gauss rule per cell), F_p = 0:
    the volume-force term of eq. (disc-residual) on one slab.  f_qp: f at the
    points of `quadrature_points` for every Radau node, [nt, cells, 3^d, d]."""
    f_qp = _f64(f_qp)
    assert f_qp.size == prob.nt * prob.num_cells * 3 ** prob.dim * prob.dim
    F = np.zeros(prob.nst)
    lib().orc_load(_cs(prob), _dp(f_qp), _dp(F))
    return F


def residual(prob: Problem, U, vprev=None, ulag=None, load=None, **kw):
    """Slab residual R_n(U), eq. (slab-underint), with the Dirichlet data of
    the problem's lifting (None: g_D = 0); `load` is the volume-force vector of
    `load_vector` (None: f = 0)."""
    U = _f64(U)
    R = np.zeros(prob.nst)
    vp = _f64(vprev) if vprev is not None else None
    ul = _f64(ulag) if ulag is not None else None
    lib().orc_residual(_cs(prob, **kw), _dp(U), _dp(vp) if vp is not None else None,
                       _dp(ul) if ul is not None else None, _dp(R))
    if load is not None:
        R += _f64(load)
    return R


def state_from_velocity(prob: Problem, uk):
    """Space-time vector whose velocity part is uk (per node) and pressure 0."""
    U = np.zeros(prob.nst)
    for m, u in enumerate(split_uk(prob, uk)):
        U[m * prob.ns:m * prob.ns + prob.nv] = u
    return U


# -------------------------------------------------------------- patches

def cell_patch(prob: Problem, cell: int, node_mask=None):
    """Space-time index set I_K of the cell patch (Sec. 6.3): every temporal
    coefficient of the cell's velocity nodes (those kept by node_mask) and of
    its pressure coefficients.  Order: time node, velocity comp, local node,
    then pressure."""
    nb = 3 ** prob.dim
    ld = local_dofs(prob)[cell]
    keep = np.arange(nb) if node_mask is None else np.flatnonzero(node_mask)
    idx = []
    for m in range(prob.nt):
        base = m * prob.ns
        for c in range(prob.dim):
            idx.extend(base + ld[c * nb + keep])
        idx.extend(base + ld[prob.dim * nb:])
    return np.asarray(idx, dtype=np.int64)


def all_patches(prob: Problem, node_masks=None):
    ld = local_dofs(prob)
    nb = 3 ** prob.dim
    out = []
    for c in range(prob.num_cells):
        keep = np.arange(nb) if node_masks is None else np.flatnonzero(node_masks[c])
        idx = []
        for m in range(prob.nt):
            base = m * prob.ns
            for comp in range(prob.dim):
                idx.extend(base + ld[c, comp * nb + keep])
            idx.extend(base + ld[c, prob.dim * nb:])
        out.append(np.asarray(idx, dtype=np.int64))
    return out


def local_patch_matrix(prob: Problem, uk_blocks, cell: int, node_mask=None, **kw):
    """R_K A R_K^T of the slab operator J_n = [K_t (x) M_x, 0; 0, 0] +
    (tau M_t (x) I) diag(J_1..J_{k+1}) (eq. slab-underint-jac) for the patch
    of one cell (Sec. 6.3), summed from the element matrices of the cells
    that share an unknown with the patch only, so that single patches of a
    large mesh can be formed without the global matrix.  uk_blocks: nt
    velocity states (the surrogate operator passes u_rep for every node).
    Returns (matrix, space-time index set in the order of cell_patch)."""
    idx = cell_patch(prob, cell, node_mask)
    pos = {int(g): k for k, g in enumerate(idx)}
    _, Mt, Kt, _ = time_matrices(prob.k_time)
    nb = 3 ** prob.dim
    nloc = prob.nloc
    cs = _cs(prob, **kw)
    # multi-index of the cell, x fastest
    ci, r = [], cell
    for k in range(prob.dim):
        ci.append(r % prob.n[k])
        r //= prob.n[k]
    A = np.zeros((idx.size, idx.size))
    ld = np.zeros(nloc, dtype=np.int32)
    import itertools
    for off in itertools.product((-1, 0, 1), repeat=prob.dim):
        cc = [ci[k] + off[k] for k in range(prob.dim)]
        if any(c < 0 or c >= prob.n[k] for k, c in enumerate(cc)):
            continue
        c, stride = 0, 1
        for k in range(prob.dim):
            c += cc[k] * stride
            stride *= prob.n[k]
        lib().orc_local_dofs(cs, int(c), ld.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        dofs = ld.copy()
        M = np.zeros((nb, nb))
        lib().orc_element_mass(cs, int(c), _dp(M))
        for m in range(prob.nt):
            uloc = _f64(uk_blocks[m][dofs[:prob.dim * nb]])
            E = np.zeros((nloc, nloc))
            lib().orc_element_matrix(cs, int(c), _dp(uloc), _dp(E))
            rows = [(i, pos.get(m * prob.ns + int(dofs[i]))) for i in range(nloc)]
            rows = [(i, p) for i, p in rows if p is not None]
            for i, pi in rows:
                for j, pj in rows:
                    A[pi, pj] += prob.tau * Mt[m, m] * E[i, j]
            for n in range(prob.nt):
                for comp in range(prob.dim):
                    for a in range(nb):
                        pi = pos.get(m * prob.ns + int(dofs[comp * nb + a]))
                        if pi is None:
                            continue
                        for b in range(nb):
                            pj = pos.get(n * prob.ns + int(dofs[comp * nb + b]))
                            if pj is not None:
                                A[pi, pj] += Kt[m, n] * M[a, b]
    return A, idx


def representative_velocity(prob: Problem, uk, t_rep: float = 0.5):
    """u at t_rep of the slab from its Radau nodal values, u_rep = sum_mu xi_mu(t_rep) u_mu."""
    nodes, _ = radau_right(prob.k_time)
    blocks = split_uk(prob, uk)
    return sum(lagrange(nodes, m, np.array([t_rep]))[0] * blocks[m] for m in range(prob.nt))


def assemble_surrogate(prob: Problem, uk, t_rep: float = 0.5):
    """Finest-level operator whose spatial blocks are all frozen at t_rep,
    eq. (surrogate-diag): diag(J_1..J_{k+1}) -> I (x) J(u_rep), the Nitsche
    coefficients at the lifting's value at t_rep."""
    ur = representative_velocity(prob, uk, t_rep)
    gr = (representative_velocity(prob, prob.lifting, t_rep) if prob.lifting is not None
          else None)
    return assemble_slab(prob, [ur] * prob.nt, [gr] * prob.nt)


def patch_matrices(A, patches):
    A = A.tocsr()
    return [A[idx][:, idx].toarray() for idx in patches]


def vanka_step(A, patch_mats, patches, r, d, omega):
    """One additive Vanka step, eq. (stmg-vanka-update):
    d <- d + omega sum_K R_K^T (A_K)^{-1} R_K (r - A d), with A_K the given
    patch matrices, each solved by LU with partial pivoting."""
    res = r - A @ d
    corr = np.zeros_like(d)
    for AK, idx in zip(patch_mats, patches):
        corr[idx] += sla.lu_solve(sla.lu_factor(AK), res[idx])
    return d + omega * corr


# ----------------------------------------------------------- hierarchy

def prolongation_spatial(coarse: Problem, fine: Problem):
    """Nested interpolation coarse -> fine: Q2 velocity by evaluating the coarse
    Q2 function at the fine nodes, P1disc pressure by restricting the coarse
    linear function to each child cell (exact for nested meshes)."""
    d = coarse.dim
    assert all(fine.n[k] == 2 * coarse.n[k] for k in range(d))
    Hc = coarse.h
    # velocity
    nnf = [2 * m + 1 for m in fine.n]
    nnc = [2 * m + 1 for m in coarse.n]
    grids = np.meshgrid(*[np.arange(m) for m in nnf], indexing="ij")
    # lexicographic with x fastest: index = i0 + nnf0*(i1 + nnf1*i2)
    fidx = [g.ravel(order="F") for g in grids]
    nf = fidx[0].size
    xf = [fine.lo[k] + fidx[k] * (fine.h[k] / 2.0) for k in range(d)]
    cell = [np.minimum(np.floor((xf[k] - coarse.lo[k]) / Hc[k]).astype(np.int64), coarse.n[k] - 1)
            for k in range(d)]
    s = [(xf[k] - coarse.lo[k]) / Hc[k] - cell[k] for k in range(d)]

    def q2(a, t):
        return [2 * (t - .5) * (t - 1), -4 * t * (t - 1), 2 * t * (t - .5)][a]

    frow = np.zeros(nf, dtype=np.int64)
    stride = 1
    for k in range(d):
        frow += fidx[k] * stride
        stride *= nnf[k]
    rows, cols, vals = [], [], []
    for a in range(3 ** d):
        ak = [(a // 3 ** k) % 3 for k in range(d)]
        w = np.ones(nf)
        col = np.zeros(nf, dtype=np.int64)
        stride = 1
        for k in range(d):
            w = w * q2(ak[k], s[k])
            col += (2 * cell[k] + ak[k]) * stride
            stride *= nnc[k]
        nz = np.abs(w) > 0
        rows.append(frow[nz])
        cols.append(col[nz])
        vals.append(w[nz])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Pv = sp.csr_matrix((vals, (rows, cols)), shape=(fine.num_nodes, coarse.num_nodes))
    Pv.sum_duplicates()
    # duplicates at nodes shared by coarse cells were not created (each fine
    # node is assigned to exactly one coarse cell), so Pv is the interpolant.
    # pressure: fine coefficient (1, (x-xf)/hf, ...) from coarse (1, (x-xc)/H, ...)
    prow, pcol, pval = [], [], []
    for fc in range(fine.num_cells):
        fi = [(fc // int(np.prod(fine.n[:k]))) % fine.n[k] for k in range(d)]
        ci = [m // 2 for m in fi]
        cc = 0
        stride = 1
        for k in range(d):
            cc += ci[k] * stride
            stride *= coarse.n[k]
        # coarse linear function q = a0 + sum_k a_k (x_k - xc_k)/H_k
        # on the child: value at child centre and slopes scaled by hf/H
        for k in range(d + 1):
            frow_ = fc * (d + 1) + k
            if k == 0:
                prow.append(frow_); pcol.append(cc * (d + 1)); pval.append(1.0)
                for m in range(d):
                    xf_c = fine.lo[m] + (fi[m] + 0.5) * fine.h[m]
                    xc_c = coarse.lo[m] + (ci[m] + 0.5) * Hc[m]
                    prow.append(frow_); pcol.append(cc * (d + 1) + 1 + m)
                    pval.append((xf_c - xc_c) / Hc[m])
            else:
                prow.append(frow_); pcol.append(cc * (d + 1) + k)
                pval.append(fine.h[k - 1] / Hc[k - 1])
    Pp = sp.csr_matrix((pval, (prow, pcol)), shape=((d + 1) * fine.num_cells,
                                                    (d + 1) * coarse.num_cells))
    return sp.block_diag([Pv] * d + [Pp], format="csr")


def prolongation(coarse: Problem, fine: Problem):
    """Space-time prolongation: identity in time (same dG degree on every level)."""
    Ps = prolongation_spatial(coarse, fine)
    return sp.kron(sp.identity(fine.nt), Ps, format="csr")


def coarse_problem(prob: Problem) -> Problem:
    """The mesh of the next coarser level (its operators are Galerkin products
    of the finest one, so it carries no Dirichlet lifting of its own)."""
    return prob.with_(n=tuple(m // 2 for m in prob.n), lifting=None)


@dataclass
class Hierarchy:
    probs: list          # level 0 = coarsest
    A: list              # operators per level
    P: list              # P[l] : level l -> level l+1
    patches: list        # per level (all but coarsest)
    patch_mats: list     # per level (all but coarsest)
    coarse_lu: object = None
    pin: list = None


def build_hierarchy(prob: Problem, uk, n_levels: int, surrogate: bool = True, node_masks=None):
    """Levels from coarse (0) to fine (n_levels-1).  Finest operator = exact J_n
    at u_k; coarse operators Galerkin P^T A P; finest patches from the
    surrogate operator (midpoint freezing), coarse patches exact."""
    probs = [prob]
    for _ in range(n_levels - 1):
        probs.insert(0, coarse_problem(probs[0]))
    A = [None] * n_levels
    A[-1] = assemble_slab(prob, split_uk(prob, uk))
    P = [None] * (n_levels - 1)
    for l in range(n_levels - 2, -1, -1):
        P[l] = prolongation(probs[l], probs[l + 1])
        A[l] = (P[l].T @ A[l + 1] @ P[l]).tocsr()
    patches = [None] * n_levels
    pmats = [None] * n_levels
    for l in range(1, n_levels):
        patches[l] = all_patches(probs[l], node_masks if l == n_levels - 1 else None)
        src = assemble_surrogate(prob, uk) if (l == n_levels - 1 and surrogate) else A[l]
        pmats[l] = patch_matrices(src, patches[l])
    H = Hierarchy(probs, A, P, patches, pmats)
    H.coarse_lu, H.pin = coarse_factor(probs[0], A[0])
    return H


def pressure_pin_indices(prob: Problem):
    """Constant pressure coefficient of cell 0 at every time node."""
    return [m * prob.ns + prob.nv for m in range(prob.nt)]


def coarse_factor(prob: Problem, A):
    """Dense LU of the coarsest operator with cell 0's constant pressure
    coefficient pinned per time node (row and column replaced by identity):
    with Dirichlet data on the whole boundary the constant pressure of each
    time node spans the kernel."""
    Ad = A.toarray()
    pin = pressure_pin_indices(prob)
    for i in pin:
        Ad[i, :] = 0.0
        Ad[:, i] = 0.0
        Ad[i, i] = 1.0
    return sla.lu_factor(Ad), pin


def coarse_solve(H: Hierarchy, r):
    rr = r.copy()
    rr[H.pin] = 0.0
    return sla.lu_solve(H.coarse_lu, rr)


def vcycle(H: Hierarchy, r, nu1=2, nu2=2, omega=0.5, level=None):
    """d = V(r): nu1 Vanka steps from d = 0, restrict the defect with P^T,
    recurse, add the prolongated correction, nu2 Vanka steps; dense LU on the
    coarsest level."""
    if level is None:
        level = len(H.probs) - 1
    if level == 0:
        return coarse_solve(H, r)
    A = H.A[level]
    d = np.zeros_like(r)
    for _ in range(nu1):
        d = vanka_step(A, H.patch_mats[level], H.patches[level], r, d, omega)
    rc = H.P[level - 1].T @ (r - A @ d)
    dc = vcycle(H, rc, nu1, nu2, omega, level - 1)
    d = d + H.P[level - 1] @ dc
    for _ in range(nu2):
        d = vanka_step(A, H.patch_mats[level], H.patches[level], r, d, omega)
    return d


def apply_rows(prob: Problem, uk, x, rows, **kw):
    """Selected rows of J_n(u_k) x (space-time row indices), each formed from the
    element matrices of the cells that carry it, so that sampled outputs of a
    large mesh can be checked without the whole action."""
    uk = _f64(uk)
    x = _f64(x)
    rows = np.asarray(rows, dtype=np.int64)
    assert prob.gamma_cip == 0.0, "apply_rows covers the cell terms only (no CIP)"
    _, _, Kt, _ = time_matrices(prob.k_time)
    _, w = radau_right(prob.k_time)
    gbl = lifting_blocks(prob)
    cs = _cs(prob, **kw)
    csm = [_cs(prob, gnode=gbl[m], **kw) for m in range(prob.nt)]
    nb = 3 ** prob.dim
    nloc = prob.nloc
    ld = np.zeros(prob.nloc, dtype=np.int32)
    out = np.zeros(rows.size)
    cache = {}

    def cell_data(c):
        if c not in cache:
            lib().orc_local_dofs(cs, int(c), ld.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
            dofs = ld.copy()
            Es = []
            for m in range(prob.nt):
                uloc = _f64(uk[m * prob.nv + dofs[:prob.dim * nb]])
                E = np.zeros((nloc, nloc))
                lib().orc_element_matrix(csm[m], int(c), _dp(uloc), _dp(E))
                Es.append(E)
            M = np.zeros((nb, nb))
            lib().orc_element_mass(cs, int(c), _dp(M))
            cache[c] = (dofs, Es, M)
        return cache[c]

    def cells_of(s):
        """cells whose local unknowns contain spatial index s"""
        if s >= prob.nv:
            return [int((s - prob.nv) // (prob.dim + 1))]
        node = s % prob.num_nodes
        idx = []
        r = node
        for k in range(prob.dim):
            nn_k = 2 * prob.n[k] + 1
            idx.append(r % nn_k)
            r //= nn_k
        cand = []
        for k in range(prob.dim):
            g = idx[k]
            cand.append([c for c in {(g - 1) // 2, g // 2, (g - 2) // 2 + 1 if g >= 2 else 0}
                         if 0 <= c < prob.n[k] and 2 * c <= g <= 2 * c + 2])
        cells = []
        import itertools
        for combo in itertools.product(*cand):
            cid, stride = 0, 1
            for k in range(prob.dim):
                cid += combo[k] * stride
                stride *= prob.n[k]
            cells.append(cid)
        return cells

    for t, row in enumerate(rows):
        mu, s = divmod(int(row), prob.ns)
        acc = 0.0
        for c in cells_of(s):
            dofs, Es, M = cell_data(c)
            i = int(np.flatnonzero(dofs == s)[0])
            acc += prob.tau * w[mu] * float(Es[mu][i] @ x[mu * prob.ns + dofs])
            if i < prob.dim * nb:
                comp, a = divmod(i, nb)
                vidx = dofs[comp * nb:(comp + 1) * nb]
                for nu in range(prob.nt):
                    acc += Kt[mu, nu] * float(M[a] @ x[nu * prob.ns + vidx])
        out[t] = acc
    return out


# ------------------------------------------------------------ slab solve

def assemble_pressure_mass(prob: Problem):
    """P1disc mass in the spatial (ns x ns) layout: on a cell of size
    h_1 x ... x h_d the basis 1, (x_k - c_k)/h_k is orthogonal, with integrals
    |K| and |K|/12."""
    d = prob.dim
    diag = np.zeros(prob.ns)
    area = float(np.prod(prob.h))
    base = prob.nv + (d + 1) * np.arange(prob.num_cells)
    diag[base] = area
    for k in range(1, d + 1):
        diag[base + k] = area / 12.0
    return sp.diags(diag)


def slab_mass(prob: Problem):
    """Block mass of the time step, velocity and pressure: the spatial masses
    weighted by tau times the Radau weights, tau M_t (x) M (Sec. 6.1, the norm
    of the algebraic residuals)."""
    _, Mt, _, _ = time_matrices(prob.k_time)
    Ms = assemble_velocity_mass(prob) + assemble_pressure_mass(prob)
    return sp.block_diag([prob.tau * Mt[m, m] * Ms for m in range(prob.nt)]).tocsr()


def mass_norm(prob: Problem, r, M=None):
    """||(r_v, r_p)||_M = sqrt(r_v^T M_v r_v + r_p^T M_p r_p) (Sec. 6.1)."""
    r = _f64(r)
    M = slab_mass(prob) if M is None else M
    return float(np.sqrt(r @ (M @ r)))


def velocity_blocks(prob: Problem, U):
    """The nt velocity blocks of a space-time vector (the linearisation state)."""
    U = _f64(U)
    return [U[m * prob.ns:m * prob.ns + prob.nv].copy() for m in range(prob.nt)]


@dataclass
class NewtonResult:
    U: np.ndarray
    residual_norms: list
    steps: list


def newton_solve(prob: Problem, vprev, U0=None, rtol=1e-8, atol=0.0, max_it=30, c_armijo=1e-4,
                 max_backtrack=30, load=None):
    """Newton iteration on R_n(U) = 0, eq. (nk-newton-lin): J_n(U^m) dU = R_n(U^m)
    with J_n the slab linearisation of prob.lin, solved directly (sparse LU, with
    the constant pressure coefficient of cell 0 pinned per time node: with
    Dirichlet data on the whole boundary the constant pressure of each time
    node spans the kernel), then U^{m+1} = U^m + lambda dU with Armijo
    backtracking on phi = ||R||_M^2 / 2 (halving lambda until
    ||R(U + lambda dU)||_M <= (1 - c lambda) ||R(U)||_M); stops when
    ||R||_M <= max(atol, rtol ||R(U^0)||_M), eq. (nk-stop).  U0 defaults to
    the left trace at both time nodes with zero pressure; `load` a
    volume-force vector (`load_vector`), None for f = 0."""
    import scipy.sparse.linalg as spla

    M = slab_mass(prob)
    vprev = _f64(vprev)
    U = state_from_velocity(prob, np.concatenate([vprev] * prob.nt)) if U0 is None else _f64(U0).copy()
    R = residual(prob, U, vprev, load=load)
    r0 = mass_norm(prob, R, M)
    norms, steps = [r0], []
    pin = pressure_pin_indices(prob)
    keep = np.setdiff1d(np.arange(prob.nst), pin)
    for _ in range(max_it):
        if norms[-1] <= max(atol, rtol * r0):
            break
        J = assemble_slab(prob, velocity_blocks(prob, U)).tocsc()
        dU = np.zeros(prob.nst)
        dU[keep] = spla.splu(J[keep][:, keep].tocsc()).solve(R[keep])
        lam = 1.0
        for _ in range(max_backtrack):
            Rn = residual(prob, U + lam * dU, vprev, load=load)
            nn = mass_norm(prob, Rn, M)
            if nn <= (1.0 - c_armijo * lam) * norms[-1]:
                break
            lam *= 0.5
        U = U + lam * dU
        R = Rn
        norms.append(nn)
        steps.append(lam)
    return NewtonResult(U, norms, steps)
