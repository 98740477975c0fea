"""Dense-matrix forms of the smoothers and cycles of oracle.mg, for the pins:
the Chebyshev error polynomial through an eigendecomposition and the
error-propagation recursion of a multigrid cycle."""
import numpy as np


def cheb_error_matrix(A, dinv, degree, lo, hi):
    """p_k(D^-1 A) for the scaled Chebyshev polynomial of degree k on [lo, hi]
    (identity for k = 0), through the eigendecomposition of D^-1 A and numpy's
    Chebyshev basis."""
    n = A.shape[0]
    if degree == 0:
        return np.eye(n)
    lam, Vec = np.linalg.eig(dinv[:, None] * A)
    lam, Vec = lam.real, Vec.real
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = np.polynomial.chebyshev.Chebyshev.basis(degree)
    pk = Tk((theta - lam) / delta) / Tk(theta / delta)
    return Vec @ (pk[:, None] * np.linalg.inv(Vec))


def cycle_matrix(H, l=0):
    """B_l, the linear operator of the V-cycle on level l, from the textbook
    error propagation of a multigrid cycle: I - B_l A_l =
    S_post (I - P B_(l+1) P^T A_l) S_pre with the smoothers' Chebyshev error
    matrices S, and B = A^-1 on the coarsest level."""
    lev = H.levels[l]
    A = lev.A.toarray()
    if l == len(H.levels) - 1:
        return np.linalg.inv(A)
    o = H.opts
    Bc = cycle_matrix(H, l + 1)
    P = lev.P.toarray()
    n = A.shape[0]
    Spre = cheb_error_matrix(A, lev.dinv, o.pre(l), lev.lo, lev.hi)
    Spost = cheb_error_matrix(A, lev.dinv, o.post(l), lev.lo, lev.hi)
    E = Spost @ (np.eye(n) - P @ Bc @ P.T @ A) @ Spre
    return (np.eye(n) - E) @ np.linalg.inv(A)
