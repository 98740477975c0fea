"""Oracle block preconditioner, flexible GMRES and adjoint (test infrastructure).

Schur-complement fieldsplit (section "Proposed four-field solvers", Method 2,
splitting by fields; Method 1 gives the same operator because its A and D
blocks are the per-network diagonal blocks of Method 2):

    K = [A B; C D],  A = blockdiag(K_uu^1, K_uu^2), B = blockdiag(K_up^i),
                     C = blockdiag(K_pu^i),        D = [K_pp^1 K_pp^12; K_pp^21 K_pp^2]

and the "full" factorisation applied with approximate inverses

    y_u = A~^-1 r_u,   r^_p = r_p - C y_u,   z_p = S~^-1 r^_p,
    z_u = A~^-1 (r_u - B z_p)

where A~^-1 is one Jacobi sweep (the velocity blocks are mass matrices,
spectrally equivalent to their diagonal) and S~^-1 applies one V-cycle to each
diagonal block S_p^i of the selfp approximation (eqs. S4_sp1, S4_sp2), the
inter-network blocks being dropped (additive split of S_p).  The outer Krylov
method is GMRES on the whole 4x4 system; it is run right-preconditioned and
flexible here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dpp
from . import mg


class FieldSplit:
    """Schur fieldsplit preconditioner of the solver section (Method 2)."""

    def __init__(self, system, mg_opts=None, inner="vcycle", velocity="jacobi"):
        self.dim, self.N = system.dim, system.N
        self.F = dpp.fields(self.dim, self.N)
        self.B = dpp.blocks(system)
        self.dinv = [1.0 / self.B["Kuu"][i].diagonal() for i in range(2)]
        self.Sp = dpp.selfp(system)
        self.inner = inner
        self.velocity = velocity
        if velocity == "exact" or inner == "exact_schur":
            self.Ainv = [np.linalg.inv(self.B["Kuu"][i].toarray()) for i in range(2)]
        if inner == "vcycle":
            self.H = [mg.setup(self.Sp[i], self.dim, system.mesh.n, mg_opts, system.mesh.elem)
                      for i in range(2)]
        elif inner == "exact_selfp":
            self.lu = [spla.splu(self.Sp[i].tocsc()) for i in range(2)]
        elif inner == "exact_schur":
            # exact Schur complement of the whole 2x2 field split (K12, K21 kept)
            Ainv = sp.block_diag([sp.csr_matrix(self.Ainv[i]) for i in range(2)])
            Bm = sp.block_diag([self.B["Kup"][i] for i in range(2)])
            Cm = sp.block_diag([self.B["Kpu"][i] for i in range(2)])
            Dm = sp.bmat([[self.B["Kpp"][0], self.B["K12"]], [self.B["K21"], self.B["Kpp"][1]]])
            self.lu_full = spla.splu((Dm - Cm @ Ainv @ Bm).tocsc())
        else:
            raise ValueError(inner)

    def _vel(self, i, r):
        if hasattr(self, "Ainv"):
            return self.Ainv[i] @ r
        return self.dinv[i] * r

    def apply(self, r):
        F = self.F
        ru = [r[F["u1"]], r[F["u2"]]]
        rp = [r[F["p1"]], r[F["p2"]]]
        yu = [self._vel(i, ru[i]) for i in range(2)]
        rhat = [rp[i] - self.B["Kpu"][i] @ yu[i] for i in range(2)]
        if self.inner == "vcycle":
            zp = [mg.vcycle(self.H[i], rhat[i]) for i in range(2)]
        elif self.inner == "exact_selfp":
            zp = [self.lu[i].solve(rhat[i]) for i in range(2)]
        else:
            z = self.lu_full.solve(np.concatenate(rhat))
            zp = [z[:self.N], z[self.N:]]
        zu = [self._vel(i, ru[i] - self.B["Kup"][i] @ zp[i]) for i in range(2)]
        z = np.empty_like(r)
        z[F["u1"]], z[F["p1"]], z[F["u2"]], z[F["p2"]] = zu[0], zp[0], zu[1], zp[1]
        return z


def fgmres(K, b, M=None, restart=30, rtol=1e-8, maxiter=1000, x0=None, matvec=None):
    """Right-preconditioned flexible GMRES(m) (Saad, SIAM J. Sci. Comput. 14,
    1993) with modified Gram-Schmidt; stops on the true residual
    ||b - K x|| <= rtol ||b|| checked at each restart/exit.

    Returns (x, iterations, true relative residual)."""
    mv = matvec or (lambda v: K @ v)
    Mf = M or (lambda v: v)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0, 0.0
    its = 0
    while True:
        r = b - mv(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bn or its >= maxiter:
            return x, its, beta / bn
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        j = 0
        for j in range(restart):
            Z[j] = Mf(V[j])
            w = mv(Z[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            if abs(g[j + 1]) <= rtol * bn or its >= maxiter:
                break
        k = j + 1
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y


def solve(system, restart=30, rtol=1e-8, maxiter=1000, mg_opts=None):
    """The paper's method: GMRES on K u = f preconditioned by the fieldsplit."""
    P = FieldSplit(system, mg_opts)
    return fgmres(system.K, system.f, P.apply, restart, rtol, maxiter)


# ---------------------------------------------------------------- adjoint --

def adjoint_solve(system, g):
    """lambda with K^T lambda = g (plain sparse LU of the transpose)."""
    return spla.spsolve(system.K.T.tocsc(), g)


def _param_gradient_q1(msh, prob, mu, F, x, lam):
    """param_gradient on Q1 box cells: the same three terms with the box
    cell's exact mass and stiffness matrices, tensor products of the
    one-dimensional linear-element matrices (h/6)[[2, 1], [1, 2]] and
    (1/h)[[1, -1], [-1, 1]] (local corner v on the upper side of axis a when
    bit a of v is set)."""
    d, N = msh.dim, msh.N
    cells = msh.cells
    h = np.array([msh.L[a] / msh.n[a] for a in range(d)])
    nv = 2 ** d
    bits = np.array([[(v >> a) & 1 for a in range(d)] for v in range(nv)])
    same = bits[:, None, :] == bits[None, :, :]              # [v, w, axis]
    m1 = np.where(same, h / 3.0, h / 6.0)
    s1 = np.where(same, 1.0 / h, -1.0 / h)
    Mloc = np.prod(m1, axis=-1)
    Sloc = np.zeros((nv, nv))
    for a in range(d):
        Sloc += s1[:, :, a] * np.prod(np.delete(m1, a, axis=-1), axis=-1)
    out = []
    for u, p, kk in (("u1", "p1", prob.k1), ("u2", "p2", prob.k2)):
        xu = x[F[u]].reshape(N, d)[cells]
        lu = lam[F[u]].reshape(N, d)[cells]
        xp = x[F[p]][cells]
        lp = lam[F[p]][cells]
        k = np.asarray(kk, dtype=np.float64)
        uu = -(mu / (2.0 * k)) * np.einsum("ab,eac,ebc->e", Mloc, lu, xu)
        pp = (k / (2.0 * mu)) * np.einsum("ab,ea,eb->e", Sloc, lp, xp)
        out.append(-(uu + pp))
    dp_x = (x[F["p1"]] - x[F["p2"]])[cells]
    dp_l = (lam[F["p1"]] - lam[F["p2"]])[cells]
    gb = -np.sum(np.einsum("ab,ea,eb->e", Mloc, dp_l, dp_x) / mu)
    return out[0], out[1], gb


def param_gradient(system, prob, x, lam):
    """dJ/d(ln k1_e), dJ/d(ln k2_e), dJ/d beta for J(x(theta)), K x = f, given the
    adjoint lam (K^T lam = dJ/dx) and fixed boundary data (df/dtheta = 0):
        dJ/dtheta_e = -lam^T (dK/dtheta_e) x.
    K depends on k_i,e through 1/2 (w; mu/k u) (uu block) and
    1/2 (grad q; k/mu grad p) (pp block) of eq. S4_cg_stiffness_matrix, and on
    beta through (q1 - q2; beta/mu (p1 - p2)); beta is one global scalar."""
    msh = system.mesh
    d, N, mu = msh.dim, msh.N, system.mu
    F = dpp.fields(d, N)
    cells = msh.cells
    if getattr(prob, "face_bc", None) is not None and np.any(prob.face_bc):
        # velocity faces: K~ = P_f K P_f + P_c and f~ = P_f (f - K P_c g) + P_c g
        # both depend on theta; with x = g on the prescribed DOFs,
        # dJ/dtheta = lam^T (df~ - dK~ x) = -(P_f lam)^T (dK/dtheta) x
        fixed, _ = dpp.velocity_dofs(msh, prob)
        lam = np.where(fixed, 0.0, lam)
    if msh.elem == "q1":
        return _param_gradient_q1(msh, prob, mu, F, x, lam)
    X = msh.X[cells]                                    # [nc, d+1, d]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))  # columns X_a - X_0
    det = np.linalg.det(J)
    vol = np.abs(det) / (2.0 if d == 2 else 6.0)
    Ji = np.linalg.inv(J)                               # rows: grad lambda_a, a >= 1
    G = np.concatenate([-Ji.sum(1, keepdims=True), Ji], axis=1)  # [nc, d+1, d]
    gg = np.einsum("eac,ebc->eab", G, G)
    Mloc = (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    out = []
    for i, (u, p, kk) in enumerate((("u1", "p1", prob.k1), ("u2", "p2", prob.k2))):
        xu = x[F[u]].reshape(N, d)[cells]               # [nc, d+1, d]
        lu = lam[F[u]].reshape(N, d)[cells]
        xp = x[F[p]][cells]
        lp = lam[F[p]][cells]
        k = np.asarray(kk, dtype=np.float64)
        # d/dln k of (mu/(2k)) M (x) I  is  -(mu/(2k)) M (x) I
        uu = -(mu / (2.0 * k)) * vol * np.einsum("ab,eac,ebc->e", Mloc, lu, xu)
        # d/dln k of (k/(2 mu)) |e| grad.grad  is itself
        pp = (k / (2.0 * mu)) * vol * np.einsum("eab,ea,eb->e", gg, lp, xp)
        out.append(-(uu + pp))
    # beta: (q1 - q2; (beta/mu)(p1 - p2)) -> dK/dbeta = (1/mu) [M -M; -M M] on (p1, p2)
    dp_x = (x[F["p1"]] - x[F["p2"]])[cells]
    dp_l = (lam[F["p1"]] - lam[F["p2"]])[cells]
    gb = -np.sum(vol / mu * np.einsum("ab,ea,eb->e", Mloc, dp_l, dp_x))
    return out[0], out[1], gb
