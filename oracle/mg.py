"""Oracle multigrid V-cycle for the pressure Schur blocks (test infrastructure).

The paper applies one algebraic-multigrid V-cycle to each diagonal block
S_p^i of the selfp Schur approximation (Method 1 and Method 2 of the solver
section: one sweep of the velocity-block solver and one V-cycle per S_p^i
inside GMRES), justified because S_p is spectrally equivalent to a Laplacian.
The particular V-cycle is not fixed by the paper.  This build uses a geometric
one on the structured box, defined here in plain steps:

  * interpolation P: P1 nodal interpolation from the box with ceil(n/2) cells
    per axis (coarse node C sits at fine index 2C, the last one at n when n is
    odd) -- a fine node with odd indices on the axes in set O lies on the Kuhn
    edge between coarse nodes lo and lo + 1_O and takes the mean of the two;
    with Q1 box cells, (bi/tri)linear interpolation: the tensor product of the
    one-dimensional linear interpolation of each axis;
  * coarse operators: Galerkin A_{l+1} = P^T A_l P;
  * coarsest level (at most ``coarse_max`` nodes, or no further coarsening
    possible): exact dense solve;
  * smoother: Chebyshev iterations (pre and post degrees per level class, see
    MGOptions) preconditioned by the
    diagonal D of A, on the interval [lo_frac*hi, hi], hi = hi_factor * lam,
    lam = ||D^-1 A x_k|| after ``power_iters`` normalised power steps from the
    integer-hash start vector x_0[i] = frac(i * 2654435761 / 2^32) - 1/2;
  * V-cycle: zero initial guess, pre-smooth, restrict the residual with P^T,
    recurse, prolongate and add, post-smooth with the same polynomial (the
    cycle is a symmetric operator).

This module is pinned by invariants (interpolation reproduces linear
functions, Galerkin coarse operators equal re-discretised ones on nested
meshes, the power steps equal M^k x_0 through the eigendecomposition of
M = D^-1 A, k Chebyshev steps multiply the error by the scaled Chebyshev
polynomial p_k(M), the V-cycle is symmetric, a one-level cycle is the exact
inverse) and, as a whole, by the error-propagation recursion of a multigrid
cycle, I - B_l A_l = S_post (I - P B_(l+1) P^T A_l) S_pre, evaluated with
dense matrices.  The paper fixes no particular cycle and prints no numbers
for its multigrid, so the cycle's definition is this build's reading.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def axis_map(n):
    """Per-axis fine->coarse map: (lo[i], odd[i]) for fine indices 0..n."""
    i = np.arange(n + 1)
    m = (n + 1) // 2 + 1  # coarse nodes on this axis
    odd = (i % 2 == 1)
    lo = i // 2
    if n % 2 == 1:
        odd[n] = False
        lo[n] = m - 1
    return lo, odd.astype(np.int64), m


def coarse_cells(n):
    return tuple((v + 1) // 2 for v in n)


def interpolation(dim, n):
    """P1 interpolation P (N_fine x N_coarse) on the structured Kuhn box."""
    n = tuple(int(v) for v in n)
    maps = [axis_map(v) for v in n]
    mc = [m for (_, _, m) in maps]
    # fine node ids in x-fastest order
    idx = np.indices([v + 1 for v in reversed(n)]).reshape(dim, -1)[::-1]  # idx[a] = index along axis a
    lo = np.stack([maps[a][0][idx[a]] for a in range(dim)])
    od = np.stack([maps[a][1][idx[a]] for a in range(dim)])
    stride = np.cumprod([1] + mc[:-1])
    c0 = (lo * stride[:, None]).sum(0)
    c1 = ((lo + od) * stride[:, None]).sum(0)
    nf = idx.shape[1]
    has = od.any(0)
    rows = np.concatenate([np.arange(nf), np.arange(nf)[has]])
    cols = np.concatenate([c0, c1[has]])
    vals = np.concatenate([np.where(has, 0.5, 1.0), np.full(has.sum(), 0.5)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, int(np.prod(mc))))


def interpolation_1d(n):
    """Linear interpolation on one axis (n + 1 fine nodes from the coarse
    nodes of axis_map): an odd fine node takes the mean of its two coarse
    neighbours, the others the value of the coarse node at their place."""
    lo, odd, m = axis_map(n)
    i = np.arange(n + 1)
    rows = np.concatenate([i, i[odd == 1]])
    cols = np.concatenate([lo, lo[odd == 1] + 1])
    vals = np.concatenate([np.where(odd == 1, 0.5, 1.0), np.full(int(odd.sum()), 0.5)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, m))


def interpolation_q1(dim, n):
    """Q1 interpolation (N_fine x N_coarse) on box cells: the Kronecker
    product of the axes' linear interpolations, x fastest."""
    P = interpolation_1d(int(n[0]))
    for a in range(1, dim):
        P = sp.kron(interpolation_1d(int(n[a])), P)
    return P.tocsr()


def hash_start(size):
    i = np.arange(size, dtype=np.uint64)
    h = (i * np.uint64(2654435761)) % np.uint64(2 ** 32)
    return h.astype(np.float64) / 2.0 ** 32 - 0.5


def power_lambda(A, dinv, iters):
    """lam = ||D^-1 A x_k|| after ``iters`` normalised power steps."""
    x = hash_start(A.shape[0])
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = dinv * (A @ x)
        lam = np.linalg.norm(y)
        x = y / lam
    return lam


def chebyshev(A, dinv, b, x, degree, lo, hi):
    """Chebyshev iteration for A x = b preconditioned by D (Saad, Iterative
    Methods for Sparse Linear Systems, Alg. 12.1, with a diagonal preconditioner)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = dinv * (b - A @ x)
    d = r / theta
    x = x + d
    for _ in range(1, degree):
        r = dinv * (b - A @ x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        x = x + d
        rho = rho_new
    return x


@dataclass
class MGOptions:
    coarse_max: int = 0    # 0 = by dimension: 2200 nodes in 3D, 400 in 2D
    degree: int = 2
    lo_frac: float = 0.0   # 0 = by dimension: 0.1 in 3D, 0.3 in 2D
    hi_factor: float = 1.1
    power_iters: int = 15
    # Chebyshev degrees of pre- and post-smoothing on the finest level and on
    # the coarser smoothing levels (-1 = degree; pre 0 = no pre-smoothing)
    pre_fine: int = 0
    post_fine: int = 2
    pre_coarse: int = 0
    post_coarse: int = 3

    def pre(self, l):
        v = self.pre_fine if l == 0 else self.pre_coarse
        return self.degree if v < 0 else v

    def post(self, l):
        v = self.post_fine if l == 0 else self.post_coarse
        return self.degree if v < 0 else v


@dataclass
class Level:
    A: sp.csr_matrix
    n: tuple
    dinv: np.ndarray = None
    lo: float = 0.0
    hi: float = 0.0
    P: sp.csr_matrix = None


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    coarse_dense: np.ndarray = None
    opts: MGOptions = None


def setup(A, dim, n, opts=None, elem="p1"):
    """Build the level list: Galerkin operators, smoother bounds, coarse matrix
    (elem "q1": the interpolation of box cells)."""
    opts = opts or MGOptions()
    H = Hierarchy(opts=opts)
    A = A.tocsr()
    n = tuple(int(v) for v in n)
    while True:
        lev = Level(A=A, n=n)
        H.levels.append(lev)
        nodes = int(np.prod([v + 1 for v in n]))
        nc = coarse_cells(n)
        cmax = opts.coarse_max if opts.coarse_max > 0 else (2200 if len(n) == 3 else 400)
        if nodes <= cmax or nc == n:
            break
        lev.dinv = 1.0 / A.diagonal()
        lam = power_lambda(A, lev.dinv, opts.power_iters)
        lev.hi = opts.hi_factor * lam
        lev.lo = (opts.lo_frac if opts.lo_frac > 0 else (0.1 if dim == 3 else 0.3)) * lev.hi
        lev.P = interpolation_q1(dim, n) if elem == "q1" else interpolation(dim, n)
        A = (lev.P.T @ A @ lev.P).tocsr()
        n = nc
    H.coarse_dense = H.levels[-1].A.toarray()
    return H


def vcycle(H, b, l=0):
    """V(pre, post) cycle: Chebyshev pre-smoothing from x = 0 (none when pre is
    0, so the residual is b), coarse-grid correction with P and P^T, Chebyshev
    post-smoothing; the coarsest level is solved exactly."""
    lev = H.levels[l]
    if l == len(H.levels) - 1:
        return np.linalg.solve(H.coarse_dense, b)
    o = H.opts
    x = np.zeros_like(b)
    if o.pre(l) > 0:
        x = chebyshev(lev.A, lev.dinv, b, x, o.pre(l), lev.lo, lev.hi)
    r = b - lev.A @ x
    e = vcycle(H, lev.P.T @ r, l + 1)
    x = x + lev.P @ e
    x = chebyshev(lev.A, lev.dinv, b, x, o.post(l), lev.lo, lev.hi)
    return x
