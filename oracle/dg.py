"""Oracle DG-VMS assembly on the Kuhn simplices (test infrastructure only: the
tests, the smoke check and the benchmark's CPU baseline use it; the HIP
library never does).

The DG-VMS form (section "Stabilized mixed discontinuous Galerkin formulation
(DG-VMS)", eq. VMS_DG_Weak_Form) with discontinuous P1 for every field, block
entries eq. S4_dg_stiffness_matrix and right-hand side eq. S4_dg_rhs, written
out per simplex T and per facet F (alpha = mu/k, kappa = k/mu, both per cell):

  volume, network i:   K_uu += 1/2 (w; alpha u)
                       K_up += -(div w; p) - 1/2 (w; grad p)
                       K_pu += (q; div u) + 1/2 (grad q; u)
                       K_pp += 1/2 (grad q; kappa grad p) + (beta/mu)(q; p)
                       K_12 = K_21^T += -(beta/mu)(q1; p2)
  interior facet:      K_up += ([[w]]; {p})          K_pu += -({q}; [[u]])
                       K_uu += eta_u h {alpha} ([[w]]; [[u]])
                       K_pp += eta_p / h {kappa} ([[q]]; [[p]])
  boundary facet:      f_u += -(w.n; p0)   (every face a pressure face)
  body force:          f_u += 1/2 (w; gamma b),  f_p += 1/2 (grad q; kappa gamma b)

with [[w]] = w+.n+ + w-.n-, [[q]] = q+ n+ + q- n-, {p} = (p+ + p-)/2 and
eta_u = eta_p = 10 (the data tables and the appendix DG-VMS listing).
Readings: h is the cell size of the listing, twice the circumradius, which
for Kuhn simplices (their vertices are box-cell corners) is the box-cell
diagonal, the same on both sides of every facet; p0 enters through its
linear interpolant on each boundary facet (the DG1 interpolant of the nodal
data); velocity faces are not part of this row.

Every integral is exact: P1 products on simplices and facets have the closed
forms |T|(1 + delta_ij)/((d+1)(d+2)) and |F|(1 + delta_ab)/(d(d+1)), and
gradients are constant per simplex.  Facet neighbours are found by matching
sorted vertex sets (no adjacency rules of the structured mesh are used).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import dpp as odpp

ETA_U = 10.0
ETA_P = 10.0


@dataclass
class DGSystem:
    mesh: object
    K: sp.csr_matrix
    f: np.ndarray
    mu: float
    S: int            # vertex slots per field component

    @property
    def dim(self):
        return self.mesh.dim


def fields(dim, S):
    """Slices of u1, p1, u2, p2 in the slot layout [u1 | p1 | u2 | p2]."""
    d = dim
    c = [0, d * S, (d + 1) * S, (2 * d + 1) * S, (2 * d + 2) * S]
    return {f: slice(c[i], c[i + 1]) for i, f in enumerate(("u1", "p1", "u2", "p2"))}


def cell_size(msh):
    """Twice the circumradius of a Kuhn simplex = the box-cell diagonal."""
    h = [msh.L[a] / msh.n[a] for a in range(msh.dim)]
    return float(np.sqrt(np.sum(np.square(h))))


def geometry(msh):
    """Per simplex: vertex coordinates, volume, P1 basis gradients G[e, v, :]."""
    d = msh.dim
    P = msh.X[msh.cells]                           # [nc, d+1, d]
    B = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))   # columns x_k - x_0
    vol = np.abs(np.linalg.det(B)) / np.prod(np.arange(1, d + 1))
    Binv = np.linalg.inv(B)                        # row k-1: grad of phi_k
    G = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)
    return P, vol, G


def facets(msh, vol, G):
    """Interior facet pairs and boundary facets.

    Returns (e, k, e2, k2, area, normal) for interior facets (normal outward
    from e; k, k2 the local vertices opposite the facet) and (e, k, area,
    normal) for boundary facets."""
    d = msh.dim
    nc = msh.cells.shape[0]
    e_all = np.repeat(np.arange(nc), d + 1)
    k_all = np.tile(np.arange(d + 1), nc)
    keep = np.ones((nc * (d + 1), d + 1), dtype=bool)
    keep[np.arange(nc * (d + 1)), k_all] = False
    verts = np.repeat(msh.cells, d + 1, axis=0)[keep].reshape(-1, d)
    key = np.sort(verts, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    gk = G[e_all, k_all]                            # [nf, d]
    gn = np.linalg.norm(gk, axis=1)
    area = d * vol[e_all] * gn
    normal = -gk / gn[:, None]
    order = np.argsort(inv, kind="stable")
    inner = cnt[inv[order]] == 2
    pairs = order[inner].reshape(-1, 2)
    a, b = pairs[:, 0], pairs[:, 1]
    interior = (e_all[a], k_all[a], e_all[b], k_all[b], area[a], normal[a])
    bnd = order[~inner]
    boundary = (e_all[bnd], k_all[bnd], area[bnd], normal[bnd])
    return interior, boundary


def assemble(prob):
    """K, f of the DG-VMS system for a ``dpp_inputs.Problem`` with elem "dg"."""
    d = prob.dim
    msh = odpp.mesh(d, prob.n, prob.L, "p1")
    nc = msh.cells.shape[0]
    nv = d + 1
    S = nc * nv
    mu = float(prob.mu)
    F = fields(d, S)
    off_u = [F["u1"].start, F["u2"].start]
    off_p = [F["p1"].start, F["p2"].start]
    ndof = (2 * d + 2) * S
    P, vol, G = geometry(msh)
    k = [np.asarray(prob.k1, dtype=np.float64), np.asarray(prob.k2, dtype=np.float64)]
    beta = np.broadcast_to(np.asarray(prob.beta, dtype=np.float64), (nc,))
    alpha = [mu / k[0], mu / k[1]]
    kappa = [k[0] / mu, k[1] / mu]
    slot = np.arange(S).reshape(nc, nv)            # slot[e, v]
    rows, cols, vals = [], [], []

    def add(r, c, v):
        r, c, v = np.broadcast_arrays(r, c, v)
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(v.ravel())

    eye = np.eye(nv)
    M = vol[:, None, None] * (1.0 + eye)[None] / ((d + 1) * (d + 2))      # [nc, v, w]
    GG = np.einsum("evc,ewc->evw", G, G)
    sv = slot[:, :, None]                          # row slot, broadcast over w
    sw = slot[:, None, :]                          # column slot
    vm = (vol / (d + 1))[:, None, None]
    for i in range(2):
        ou, op = off_u[i], off_p[i]
        a_ = alpha[i][:, None, None]
        for c in range(d):
            add(ou + d * sv + c, ou + d * sw + c, 0.5 * a_ * M)
            gvc, gwc = G[:, :, c][:, :, None], G[:, :, c][:, None, :]
            add(ou + d * sv + c, op + sw, -vm * (gvc + 0.5 * gwc))
            add(op + sv, ou + d * sw + c, vm * (gwc + 0.5 * gvc))
        add(op + sv, op + sw, 0.5 * kappa[i][:, None, None] * vol[:, None, None] * GG
            + (beta / mu)[:, None, None] * M)
    add(off_p[0] + sv, off_p[1] + sw, -(beta / mu)[:, None, None] * M)
    add(off_p[1] + sv, off_p[0] + sw, -(beta / mu)[:, None, None] * M)

    # interior facets: sides + (e) and - (e2), facet vertices matched by id
    (e1, k1, e2, k2, area, nrm), (eb, kb, areab, nrmb) = facets(msh, vol, G)
    h = cell_size(msh)
    nf = e1.shape[0]
    if nf:
        gv1 = msh.cells[e1]                        # [nf, nv] global vertex ids
        gv2 = msh.cells[e2]
        loc1 = np.array([[v for v in range(nv) if v != kk] for kk in range(nv)])[k1]   # [nf, d]
        g_face = np.take_along_axis(gv1, loc1, axis=1)                             # facet vertices
        loc2 = np.argmax(gv2[:, None, :] == g_face[:, :, None], axis=2)            # their slots in e2
        lv = [loc1, loc2]
        es = [e1, e2]
        sg = [1.0, -1.0]
        Mf = area[:, None, None] * (1.0 + np.eye(d))[None] / (d * (d + 1))
        for i in range(2):
            ou, op = off_u[i], off_p[i]
            aavg = 0.5 * (alpha[i][e1] + alpha[i][e2])
            kavg = 0.5 * (kappa[i][e1] + kappa[i][e2])
            for s in range(2):
                rs = slot[es[s][:, None], lv[s]][:, :, None]        # [nf, a, 1]
                for t in range(2):
                    ct = slot[es[t][:, None], lv[t]][:, None, :]    # [nf, 1, b]
                    st = sg[s] * sg[t]
                    add(op + rs, op + ct, (ETA_P / h) * st * kavg[:, None, None] * Mf)
                    for c in range(d):
                        nc_ = nrm[:, c][:, None, None]
                        add(ou + d * rs + c, op + ct, sg[s] * 0.5 * nc_ * Mf)
                        add(op + rs, ou + d * ct + c, -0.5 * sg[t] * nc_ * Mf)
                        for c2 in range(d):
                            add(ou + d * rs + c, ou + d * ct + c2,
                                ETA_U * h * st * aavg[:, None, None] * nc_ * nrm[:, c2][:, None, None] * Mf)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ndof, ndof))
    K.sum_duplicates()

    f = np.zeros(ndof)
    # boundary facets: -(w.n; p0) with p0 linear on the facet
    if eb.size:
        locb = np.array([[v for v in range(nv) if v != kk] for kk in range(nv)])[kb]
        gvb = np.take_along_axis(msh.cells[eb], locb, axis=1)
        Mfb = areab[:, None, None] * (1.0 + np.eye(d))[None] / (d * (d + 1))
        rsb = slot[eb[:, None], locb]                                   # [nb, a]
        for i, p0 in enumerate((prob.p0_1, prob.p0_2)):
            p0 = np.asarray(p0, dtype=np.float64)
            tr = np.einsum("fab,fb->fa", Mfb, p0[gvb])                  # int phi_a p0
            for c in range(d):
                np.add.at(f, off_u[i] + d * rsb + c, -nrmb[:, c][:, None] * tr)
    if prob.body is not None:
        body = np.broadcast_to(np.asarray(prob.body, dtype=np.float64) * prob.gamma, (nc, d))
        for i in range(2):
            for c in range(d):
                np.add.at(f, off_u[i] + d * slot + c, 0.5 * (vol / (d + 1))[:, None] * body[:, c][:, None])
            gb = np.einsum("evc,ec->ev", G, body)
            np.add.at(f, off_p[i] + slot, 0.5 * (kappa[i] * vol)[:, None] * gb)
    return DGSystem(msh, K.tocsr(), f, mu, S)


def slot_coords(msh):
    """Coordinates of every slot [S, d] (the vertex it sits on)."""
    return msh.X[msh.cells].reshape(-1, msh.dim)


def interpolate(msh, func_p, func_u, dim):
    """DG1 interpolant (vertex values per slot) of pressure / velocity fields."""
    X = slot_coords(msh)
    return func_p(X), func_u(X)


def l2_errors(S_sys, x, exact, q=4, relative=True):
    """L2 errors per field of the DG solution x against callables
    exact[f](X) -> values at points X, by oracle.post's q-point-per-axis
    simplex rule; relative to the exact field's norm unless relative=False."""
    from . import post as opost
    msh = S_sys.mesh
    d = msh.dim
    P, vol, G = geometry(msh)
    pts, wts = opost.simplex_rule(d, q)            # barycentric points [q^d, d+1], weights summing to 1/d!
    wts = wts * np.prod(np.arange(1, d + 1))
    F = fields(d, S_sys.S)
    out = {}
    Xq = np.einsum("qv,evc->eqc", pts, P)          # [nc, q, d]
    for f in ("u1", "p1", "u2", "p2"):
        ex = exact[f](Xq.reshape(-1, d)).reshape(Xq.shape[0], Xq.shape[1], -1)
        if f.startswith("u"):
            vals = x[F[f]].reshape(-1, d + 1, d)   # [nc, v, c]
            num = np.einsum("qv,evc->eqc", pts, vals)
        else:
            vals = x[F[f]].reshape(-1, d + 1)
            num = np.einsum("qv,ev->eq", pts, vals)[:, :, None]
        w = vol[:, None] * wts[None, :]
        err = np.sqrt(np.sum(w[:, :, None] * (num - ex) ** 2))
        ref = np.sqrt(np.sum(w[:, :, None] * ex ** 2))
        out[f] = err / ref if (relative and ref > 0) else err
    return out


VEL_DEGREE = 8       # Chebyshev steps of the velocity-block solve
NODAL_COARSE_2D = 1800   # default coarsest size of the nodal cycle in 2D
VEL_LO_FRAC = 0.01   # its interval [0.01 hi, hi]
PRES_DEGREE = 3      # Chebyshev steps on S_i after the nodal correction


def power_bound(apply_A, apply_M, size, iters):
    """lam = ||M A x_k|| after ``iters`` normalised power steps from the
    integer-hash start vector (as oracle.mg.power_lambda, M any linear map)."""
    from . import mg
    x = mg.hash_start(size)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply_M(apply_A(x))
        lam = np.linalg.norm(y)
        x = y / lam
    return lam


def chebyshev_op(apply_A, apply_M, b, x, degree, lo, hi):
    """Chebyshev iteration for A x = b preconditioned by M on [lo, hi]
    (Saad, Alg. 12.1; oracle.mg.chebyshev with a general M)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = apply_M(b - apply_A(x))
    d = r / theta
    x = x + d
    for _ in range(1, degree):
        r = apply_M(b - apply_A(x))
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        x = x + d
        rho = rho_new
    return x


class FieldSplitDG:
    """Schur fieldsplit of the solver section (Method 2, selfp) on the DG-VMS
    blocks, the appendix listing's splitting of velocities and pressures
    (pressure blocks additive per network), per network i:

      y_u = V_i(r_u),  rhat = r_p - K_pu y_u,  z_p = B_i(rhat),  z_u = V_i(r_u - K_up z_p)

    * V_i approximates K_uu^-1: VEL_DEGREE Chebyshev steps from zero,
      preconditioned by the inverses of K_uu's diagonal blocks (one per
      simplex, its (d+1) d velocity unknowns), on [VEL_LO_FRAC hi, hi] with
      hi = hi_factor x the power-step estimate.  The velocity-jump penalty
      couples neighbouring simplices as strongly as the mass term couples a
      simplex's own unknowns, so the diagonal of K_uu (enough for CG-VMS)
      needs hundreds of outer iterations here; the listing's block Jacobi
      with ILU sub-blocks plays this part there.
    * S_i = K_pp - K_pu diag(K_uu)^-1 K_up (selfp), and B_i a two-level cycle
      whose coarse level is the nodal CG-VMS problem of the same box and
      coefficients (its selfp block and multigrid hierarchy, oracle.mg, whose
      coarsest level by default takes up to NODAL_COARSE_2D nodes in 2D):
      restrict by summing the slot values on each node (R), one V-cycle,
      copy the node values back to the slots (R^T), then PRES_DEGREE
      Chebyshev post-smoothing steps on S_i with its diagonal (the nodal
      levels' power-step bound and interval [lo_frac hi, hi])."""

    def __init__(self, system, prob, mg_opts=None):
        from dataclasses import replace

        from . import mg, solver
        d, S = system.dim, system.S
        F = fields(d, S)
        self.F = F
        K = system.K.tocsr()
        nc = system.mesh.cells.shape[0]
        NU = (d + 1) * d
        o = mg_opts or mg.MGOptions()
        self.opts = o
        self.Kuu, self.Kup, self.Kpu, self.Binv, self.Sp, self.dS = [], [], [], [], [], []
        self.vhi, self.vlo = [], []
        for u, p in (("u1", "p1"), ("u2", "p2")):
            Kuu = K[F[u], F[u]].tocsr()
            dinv = 1.0 / Kuu.diagonal()
            Kup, Kpu, Kpp = K[F[u], F[p]], K[F[p], F[u]], K[F[p], F[p]]
            Sp = (Kpp - Kpu @ sp.diags(dinv) @ Kup).tocsr()
            blocks = [np.linalg.inv(Kuu[e * NU:(e + 1) * NU, e * NU:(e + 1) * NU].toarray()) for e in range(nc)]
            Binv = sp.block_diag(blocks).tocsr()
            lam = power_bound(lambda v, A=Kuu: A @ v, lambda v, B=Binv: B @ v, Kuu.shape[0], o.power_iters)
            self.vhi.append(o.hi_factor * lam)
            self.vlo.append(VEL_LO_FRAC * o.hi_factor * lam)
            self.Kuu.append(Kuu)
            self.Kup.append(Kup)
            self.Kpu.append(Kpu)
            self.Binv.append(Binv)
            self.Sp.append(Sp)
            self.dS.append(1.0 / Sp.diagonal())
        lo_frac = o.lo_frac if o.lo_frac > 0 else (0.1 if d == 3 else 0.3)
        self.hi = [o.hi_factor * mg.power_lambda(self.Sp[i], self.dS[i], o.power_iters) for i in range(2)]
        self.lo = [lo_frac * h for h in self.hi]
        self.deg = PRES_DEGREE
        cg = odpp.assemble(replace(prob, elem="p1"))
        oc = replace(o, coarse_max=NODAL_COARSE_2D) if (o.coarse_max == 0 and d == 2) else o
        self.H = solver.FieldSplit(cg, oc).H
        msh = system.mesh
        self.R = sp.csr_matrix((np.ones(S), (msh.cells.ravel(), np.arange(S))), shape=(msh.N, S))

    def velocity(self, i, b):
        return chebyshev_op(lambda v: self.Kuu[i] @ v, lambda v: self.Binv[i] @ v, b, np.zeros_like(b),
                            VEL_DEGREE, self.vlo[i], self.vhi[i])

    def pressure(self, i, rhat):
        """B_i(rhat): the nodal V-cycle on the summed residual, copied back to
        the slots, then Chebyshev post-smoothing on S_i."""
        from . import mg
        zp = self.R.T @ mg.vcycle(self.H[i], self.R @ rhat)
        return mg.chebyshev(self.Sp[i], self.dS[i], rhat, zp, self.deg, self.lo[i], self.hi[i])

    def apply(self, r):
        F = self.F
        z = np.empty_like(r)
        for i, (u, p) in enumerate((("u1", "p1"), ("u2", "p2"))):
            ru, rp = r[F[u]], r[F[p]]
            rhat = rp - self.Kpu[i] @ self.velocity(i, ru)
            zp = self.pressure(i, rhat)
            z[F[p]] = zp
            z[F[u]] = self.velocity(i, ru - self.Kup[i] @ zp)
        return z
