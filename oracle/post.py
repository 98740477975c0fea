"""Oracle post-processing (test infrastructure): errors and balance checks.

  * L2 error against the manufactured solution (section "Mesh convergence":
    ||u_h - u||_L2 decays like C h^alpha, alpha = 2 for first-order VMS),
    by a collapsed-coordinate Gauss rule on each simplex (a tensor Gauss rule
    on each box cell with Q1 elements);
  * L2 distance to the nodal interpolant of the exact solution (the error
    measure of the appendix listings, which interpolate the exact fields);
  * boundary flux of each velocity and integral of each pressure: testing the
    mass balance with q_1 = 1 gives  oint u1.n = -(beta/mu) int (p1 - p2),
    and adding q_2 = 1 gives  oint (u1 + u2).n = 0  (the transfer terms
    of eq. Composable_mass_transfer cancel).
"""
from __future__ import annotations

import numpy as np

from . import dpp


def _gauss01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_rule(dim, q=8):
    """Barycentric points [m, d+1] and weights (summing to 1/d!) on the
    reference simplex by the collapsed (Duffy) map of a q^d Gauss grid."""
    t, w = _gauss01(q)
    if dim == 2:
        s, e = np.meshgrid(t, t, indexing="ij")
        ws = np.outer(w, w) * s
        l1 = s * (1 - e)
        l2 = s * e
        lam = np.stack([1 - s, l1, l2], -1).reshape(-1, 3)
        return lam, ws.reshape(-1)
    s, e, g = np.meshgrid(t, t, t, indexing="ij")
    ws = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * s * s * e
    l1 = s * (1 - e)
    l2 = s * e * (1 - g)
    l3 = s * e * g
    lam = np.stack([1 - s, l1, l2, l3], -1).reshape(-1, 4)
    return lam, ws.reshape(-1)


def box_rule(dim, q):
    """Tensor Gauss-Legendre rule on the unit box [0,1]^dim: points [q^dim, dim]
    (x fastest) and weights summing to 1."""
    t, w = _gauss01(q)
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    pts = np.stack([g.reshape(-1) for g in reversed(grids)], -1)
    wg = np.meshgrid(*([w] * dim), indexing="ij")
    wts = np.prod(np.stack([g.reshape(-1) for g in wg], -1), axis=-1)
    return pts, wts


def q1_basis(xi):
    """Q1 shape functions of the unit box at points xi [m, d]: [m, 2^d], local
    vertex v has coordinate bit (v >> a) & 1 on axis a."""
    d = xi.shape[1]
    B = np.ones((xi.shape[0], 2 ** d))
    for v in range(2 ** d):
        for a in range(d):
            B[:, v] *= xi[:, a] if (v >> a) & 1 else 1.0 - xi[:, a]
    return B


def _q1_cells(msh):
    """Corner coordinates [nc, d] and cell sizes [d] of the box cells."""
    h = np.array([msh.L[a] / msh.n[a] for a in range(msh.dim)])
    return msh.X[msh.cells[:, 0]], h


def _l2_errors_q1(system, x, exact, q, chunk):
    msh = system.mesh
    d, N = msh.dim, msh.N
    F = dpp.fields(d, N)
    xi, w = box_rule(d, q)
    B = q1_basis(xi)
    X0, h = _q1_cells(msh)
    vol = float(np.prod(h))
    acc = dict(u1=0.0, p1=0.0, u2=0.0, p2=0.0)
    for c0 in range(0, msh.nc, chunk):
        cells = msh.cells[c0:c0 + chunk]
        P = X0[c0:c0 + chunk, None, :] + xi[None, :, :] * h[None, None, :]
        p1e, p2e, u1e, u2e = exact(P.reshape(-1, d))
        ex = dict(p1=p1e.reshape(len(cells), -1), p2=p2e.reshape(len(cells), -1),
                  u1=u1e.reshape(len(cells), -1, d), u2=u2e.reshape(len(cells), -1, d))
        for f in ("p1", "p2"):
            vh = np.einsum("qv,ev->eq", B, x[F[f]][cells])
            acc[f] += vol * np.sum(w[None, :] * (vh - ex[f]) ** 2)
        for f in ("u1", "u2"):
            vh = np.einsum("qv,evc->eqc", B, x[F[f]].reshape(N, d)[cells])
            acc[f] += vol * np.sum(w[None, :] * ((vh - ex[f]) ** 2).sum(-1))
    return {k: float(np.sqrt(v)) for k, v in acc.items()}


def l2_errors(system, x, exact, q=8, chunk=4096):
    """True L2 errors of (u1, p1, u2, p2) against exact(X) -> (p1, p2, u1, u2)."""
    msh = system.mesh
    if msh.elem == "q1":
        return _l2_errors_q1(system, x, exact, q, chunk)
    d, N = msh.dim, msh.N
    F = dpp.fields(d, N)
    lam, w = simplex_rule(d, q)
    acc = dict(u1=0.0, p1=0.0, u2=0.0, p2=0.0)
    for c0 in range(0, msh.nc, chunk):
        cells = msh.cells[c0:c0 + chunk]
        V = msh.X[cells]                                  # [e, d+1, d]
        J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))
        detJ = np.abs(np.linalg.det(J))
        P = np.einsum("qa,eac->eqc", lam, V)              # quadrature points
        p1e, p2e, u1e, u2e = exact(P.reshape(-1, d))
        ex = dict(p1=p1e.reshape(len(cells), -1), p2=p2e.reshape(len(cells), -1),
                  u1=u1e.reshape(len(cells), -1, d), u2=u2e.reshape(len(cells), -1, d))
        for f in ("p1", "p2"):
            vh = np.einsum("qa,ea->eq", lam, x[F[f]][cells])
            acc[f] += np.sum(detJ[:, None] * w[None, :] * (vh - ex[f]) ** 2)
        for f in ("u1", "u2"):
            vh = np.einsum("qa,eac->eqc", lam, x[F[f]].reshape(N, d)[cells])
            acc[f] += np.sum(detJ[:, None] * w[None, :] * ((vh - ex[f]) ** 2).sum(-1))
    return {k: float(np.sqrt(v)) for k, v in acc.items()}


def interp_errors(system, x, exact):
    """L2 norm of u_h - I_h u (I_h = nodal P1 interpolation), via the P1 mass
    matrix assembled from exact simplex integrals (Q1 box cells: the nodal Q1
    interpolant, integrated exactly by the 2-point tensor Gauss rule)."""
    msh = system.mesh
    d, N = msh.dim, msh.N
    F = dpp.fields(d, N)
    p1, p2, u1, u2 = exact(msh.X)
    if msh.elem == "q1":
        xi, w = box_rule(d, 2)
        B = q1_basis(xi)
        vol = float(np.prod(_q1_cells(msh)[1]))
        out = {}
        for f, ex in (("p1", p1), ("p2", p2), ("u1", u1), ("u2", u2)):
            e = x[F[f]] - ex.reshape(-1) if f[0] == "p" else x[F[f]].reshape(N, d) - ex
            vh = np.einsum("qv,ev...->eq...", B, e[msh.cells])
            sq = vh ** 2 if f[0] == "p" else (vh ** 2).sum(-1)
            out[f] = float(np.sqrt(vol * np.sum(w[None, :] * sq)))
        return out
    V = msh.X[msh.cells]
    J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(J)) / (2.0 if d == 2 else 6.0)
    Mloc = (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    out = {}
    for f, ex in (("p1", p1), ("p2", p2)):
        e = (x[F[f]] - ex)[msh.cells]
        out[f] = float(np.sqrt(np.sum(vol * np.einsum("ab,ea,eb->e", Mloc, e, e))))
    for f, ex in (("u1", u1), ("u2", u2)):
        e = (x[F[f]].reshape(N, d) - ex)[msh.cells]
        out[f] = float(np.sqrt(np.sum(vol * np.einsum("ab,eac,ebc->e", Mloc, e, e))))
    return out


def boundary_facets(msh):
    """Boundary facets as (vertex array [m, d], outward normal [m, d], measure [m])."""
    d = msh.dim
    n = msh.n
    idx = []
    N1 = [v + 1 for v in n]
    ids = np.arange(msh.N)
    ax_index = []
    r = ids.copy()
    for a in range(d):
        ax_index.append(r % N1[a])
        r //= N1[a]
    ax_index = np.stack(ax_index, 1)                      # [N, d]
    verts, normals = [], []
    for lf in range(d + 1):
        face = np.delete(msh.cells, lf, axis=1)           # [nc, d]
        fi = ax_index[face]                               # [nc, d, d]
        for a in range(d):
            for side, target in ((-1.0, 0), (1.0, n[a])):
                on = np.all(fi[:, :, a] == target, axis=1)
                if on.any():
                    verts.append(face[on])
                    nv = np.zeros((on.sum(), d))
                    nv[:, a] = side
                    normals.append(nv)
    del idx
    verts = np.concatenate(verts)
    normals = np.concatenate(normals)
    P = msh.X[verts]
    if d == 2:
        meas = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    else:
        meas = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    return verts, normals, meas


def _balance_q1(system, x):
    msh = system.mesh
    d, N, n = msh.dim, msh.N, msh.n
    F = dpp.fields(d, N)
    _, h = _q1_cells(msh)
    vol = float(np.prod(h))
    # cell indices per axis
    ce = []
    r = np.arange(msh.nc)
    for a in range(d):
        ce.append(r % n[a])
        r = r // n[a]
    out = []
    for f in ("u1", "u2"):
        u = x[F[f]].reshape(N, d)
        tot = 0.0
        for a in range(d):
            area = vol / h[a]
            for side, target in ((0, 0), (1, n[a] - 1)):
                on = ce[a] == target
                vs = [v for v in range(2 ** d) if ((v >> a) & 1) == side]
                un = u[msh.cells[on][:, vs], a] * (1.0 if side else -1.0)
                # a (bi)linear function integrates to its vertex mean on a box face
                tot += float(np.sum(area * un.mean(1)))
        out.append(tot)
    for f in ("p1", "p2"):
        out.append(float(np.sum(vol * x[F[f]][msh.cells].mean(1))))
    return tuple(out)


def balance(system, x):
    """(oint u1.n, oint u2.n, int p1, int p2) of the discrete fields."""
    msh = system.mesh
    if msh.elem == "q1":
        return _balance_q1(system, x)
    d, N = msh.dim, msh.N
    F = dpp.fields(d, N)
    verts, normals, meas = boundary_facets(msh)
    out = []
    for f in ("u1", "u2"):
        u = x[F[f]].reshape(N, d)
        un = np.einsum("mvc,mc->mv", u[verts], normals)   # u.n at facet vertices
        out.append(float(np.sum(meas * un.mean(1))))
    V = msh.X[msh.cells]
    J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(J)) / (2.0 if d == 2 else 6.0)
    for f in ("p1", "p2"):
        out.append(float(np.sum(vol * x[F[f]][msh.cells].mean(1))))
    return tuple(out)


def rates(hs, errs):
    """Observed convergence rates log(e_i/e_{i+1}) / log(h_i/h_{i+1})."""
    hs, errs = np.asarray(hs, float), np.asarray(errs, float)
    return np.log(errs[:-1] / errs[1:]) / np.log(hs[:-1] / hs[1:])
