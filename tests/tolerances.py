"""FP64 tolerances of the parity tests of maps built on dense solves (Vanka
steps, V-cycles), derived from the conditioning of the matrices solved.

The GPU and the oracle solve the same patch and coarse systems by different
eliminations (time-diagonal complex Gauss-Jordan or real Gauss-Jordan on the
device, LU with partial pivoting in the oracle).  Partial pivoting is
invariant to the scaling of rows and columns, so the forward error of either
side is governed by the condition number of the equilibrated matrix (rows,
then columns scaled to unit max norm; within a small factor of Skeel's
condition number), not by the 2-norm condition number, which here mostly
measures the different scales of velocity and pressure rows.  The bound used
is  max(1e-12, kappa_eq * 1e-16):  1e-12 (the FP64 parity bound of the
action) wherever kappa_eq * u stays below it, the forward-error estimate
kappa_eq * u (u = 2^-53, rounded up to 1e-16) above that.
"""
import numpy as np
import scipy.linalg as sla

FP64_FLOOR = 1e-12
UNIT_ROUNDOFF = 1e-16


def _equilibrate(M):
    M = np.asarray(M, dtype=np.float64)
    M = M / np.abs(M).max(axis=-1, keepdims=True)
    return M / np.abs(M).max(axis=-2, keepdims=True)


def kappa_eq(mats):
    """Largest 2-norm condition number of the equilibrated matrices of a stack
    (or a list) of small dense matrices; 1 for an empty list."""
    mats = list(mats)
    if not mats:
        return 1.0
    out = 1.0
    for n in sorted({m.shape[0] for m in mats}):
        stack = np.stack([m for m in mats if m.shape[0] == n])
        out = max(out, float(np.max(np.linalg.cond(_equilibrate(stack)))))
    return out


def kappa_eq_dense(A):
    """1-norm condition estimate (LAPACK gecon after an LU) of one larger
    equilibrated matrix, e.g. the pinned coarsest operator."""
    E = _equilibrate(A.toarray() if hasattr(A, "toarray") else A)
    lu, piv = sla.lu_factor(E)
    rcond, info = sla.lapack.dgecon(lu, np.abs(E).sum(axis=0).max(), norm="1")
    assert info == 0
    return 1.0 / max(rcond, 1e-300)


def pinned_coarse(H):
    """The coarsest operator of an oracle hierarchy with the pinned pressure
    coefficients (row and column replaced by the identity)."""
    Ad = H.A[0].toarray()
    for i in H.pin:
        Ad[i, :] = 0.0
        Ad[:, i] = 0.0
        Ad[i, i] = 1.0
    return Ad


def hierarchy_kappa(H):
    """Largest equilibrated condition number over the patch matrices of every
    smoothed level and the pinned coarsest operator of a hierarchy."""
    k = 1.0
    for pm in H.patch_mats:
        if pm is not None:
            k = max(k, kappa_eq(pm))
    if len(H.probs) > 1:
        k = max(k, kappa_eq_dense(pinned_coarse(H)))
    return k


def fp64_tol(kappa):
    return max(FP64_FLOOR, kappa * UNIT_ROUNDOFF)
