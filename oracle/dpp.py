"""Oracle assembly of the CG-VMS four-field DPP system (test infrastructure).

K and f are the block entries of eq. S4_cg_stiffness_matrix and eq. S4_cg_rhs
(section "Proposed four-field solvers") obtained from the CG-VMS weak form
(eq. CG_VMS_Weak_form) on P1 simplices; the numeric work is done in
``dpp_oracle.c`` in plain FP64.  Unknown ordering [u1 | p1 | u2 | p2] with the
velocity components interleaved per node (the ordering of the mixed space in
the appendix listings: fields 0..3 = u1, p1, u2, p2).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import build as _build

_lib = None
MAXADJ = 32


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.ensure_built())
        P = C.c_void_p
        _lib.or_num_nodes.restype = C.c_long
        _lib.or_num_nodes.argtypes = [C.c_int, P]
        _lib.or_num_cells.restype = C.c_long
        _lib.or_num_cells.argtypes = [C.c_int, P]
        _lib.or_mesh.restype = None
        _lib.or_mesh.argtypes = [C.c_int, P, P, P, P]
        _lib.or_adjacency.restype = None
        _lib.or_adjacency.argtypes = [C.c_int, C.c_int, C.c_long, C.c_long, P, P, P, P, P]
        _lib.or_num_cells_q1.restype = C.c_long
        _lib.or_num_cells_q1.argtypes = [C.c_int, P]
        _lib.or_mesh_q1.restype = None
        _lib.or_mesh_q1.argtypes = [C.c_int, P, P, P, P]
        _lib.or_assemble_q1.restype = None
        _lib.or_assemble_q1.argtypes = [C.c_int, P, P, C.c_long, P, P, P, P, P, P, P, P, P,
                                        P, C.c_double, P, P, P]
        _lib.or_rowptr.restype = C.c_int64
        _lib.or_rowptr.argtypes = [C.c_int, C.c_long, P, P]
        _lib.or_cols.restype = None
        _lib.or_cols.argtypes = [C.c_int, C.c_long, P, P, P, P]
        _lib.or_assemble.restype = None
        _lib.or_assemble.argtypes = [C.c_int, P, C.c_long, C.c_long, P, P, P, P, P, P, P, P,
                                     P, P, P, C.c_double, P, P, P]
        _lib.or_spmv.restype = None
        _lib.or_spmv.argtypes = [C.c_long, P, P, P, P, P]
        _lib.or_max_threads.restype = C.c_int
        _lib.or_max_threads.argtypes = []
    return _lib


def threads():
    """Threads of the oracle's OpenMP loops (assembly, CSR product)."""
    return int(lib().or_max_threads())


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Mesh:
    dim: int
    n: tuple
    L: tuple
    X: np.ndarray        # [N, d]
    cells: np.ndarray    # [nc, d+1] simplices, or [nc, 2^d] box cells (Q1)
    incptr: np.ndarray
    inc: np.ndarray
    adjcnt: np.ndarray
    adj: np.ndarray
    elem: str = "p1"

    @property
    def N(self):
        return self.X.shape[0]

    @property
    def nc(self):
        return self.cells.shape[0]


def mesh(dim, n, L=None, elem="p1"):
    """Structured box mesh (spec in the module docstring of dpp_inputs): Kuhn
    simplices for P1, the box cells themselves for Q1."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    L = np.ascontiguousarray(L if L is not None else [1.0] * dim, dtype=np.float64)
    lb = lib()
    N = lb.or_num_nodes(dim, _p(n))
    X = np.empty((N, dim))
    if elem == "q1":
        nv = 2 ** dim
        nc = lb.or_num_cells_q1(dim, _p(n))
        cells = np.empty((nc, nv), dtype=np.int32)
        lb.or_mesh_q1(dim, _p(n), _p(L), _p(X), _p(cells))
    else:
        nv = dim + 1
        nc = lb.or_num_cells(dim, _p(n))
        cells = np.empty((nc, nv), dtype=np.int32)
        lb.or_mesh(dim, _p(n), _p(L), _p(X), _p(cells))
    incptr = np.empty(N + 1, dtype=np.int64)
    inc = np.empty(nc * nv, dtype=np.int32)
    adjcnt = np.empty(N, dtype=np.int32)
    adj = np.zeros((N, MAXADJ), dtype=np.int32)
    lb.or_adjacency(dim, nv, N, nc, _p(cells), _p(incptr), _p(inc), _p(adjcnt), _p(adj))
    return Mesh(dim, tuple(int(v) for v in n), tuple(float(v) for v in L), X, cells, incptr,
                inc, adjcnt, adj, elem)


@dataclass
class System:
    mesh: Mesh
    K: sp.csr_matrix
    f: np.ndarray
    mu: float

    @property
    def dim(self):
        return self.mesh.dim

    @property
    def N(self):
        return self.mesh.N


def fields(dim, N):
    """Index slices of the four fields in the global vector (u1, p1, u2, p2)."""
    d = dim
    return dict(u1=slice(0, d * N), p1=slice(d * N, (d + 1) * N),
                u2=slice((d + 1) * N, (2 * d + 1) * N), p2=slice((2 * d + 1) * N, (2 * d + 2) * N))


def assemble(prob, msh=None):
    """Assemble K, f of the CG-VMS system for a ``dpp_inputs.Problem``.

    Follows eq. S4_cg_stiffness_matrix / eq. S4_cg_rhs; pressure boundary data
    enter weakly through -(w.n; p0) (eq. VMS_classical_mixed_formulation and the
    linear functional of the appendix CG-VMS listing), with p0 the nodal
    interpolant (P1, or Q1 on box cells) integrated exactly on each boundary
    facet.  Q1 box cells (prob.elem == "q1") are the [Q1 + Q1]^2 rows of the
    element table: the same forms, integrated exactly cell by cell.
    """
    d = prob.dim
    elem = getattr(prob, "elem", "p1")
    msh = msh or mesh(d, prob.n, prob.L, elem)
    lb = lib()
    N, nc = msh.N, msh.nc
    ndof = (2 * d + 2) * N
    rowptr = np.empty(ndof + 1, dtype=np.int64)
    nnz = lb.or_rowptr(d, N, _p(msh.adjcnt), _p(rowptr))
    cols = np.empty(nnz, dtype=np.int32)
    lb.or_cols(d, N, _p(msh.adjcnt), _p(msh.adj), _p(rowptr), _p(cols))
    vals = np.empty(nnz)
    f = np.empty(ndof)
    k1 = np.ascontiguousarray(prob.k1, dtype=np.float64)
    k2 = np.ascontiguousarray(prob.k2, dtype=np.float64)
    beta = np.ascontiguousarray(np.broadcast_to(np.asarray(prob.beta, dtype=np.float64), (nc,)))
    body = None
    if prob.body is not None:
        body = np.ascontiguousarray(np.broadcast_to(np.asarray(prob.body, dtype=np.float64) *
                                                    prob.gamma, (nc, d)))
    p01 = np.ascontiguousarray(prob.p0_1, dtype=np.float64)
    p02 = np.ascontiguousarray(prob.p0_2, dtype=np.float64)
    nn = np.ascontiguousarray(msh.n, dtype=np.int32)
    if elem == "q1":
        LL = np.ascontiguousarray(msh.L, dtype=np.float64)
        lb.or_assemble_q1(d, _p(nn), _p(LL), N, _p(msh.cells), _p(msh.incptr), _p(msh.inc),
                          _p(rowptr), _p(cols), _p(vals), _p(f), _p(k1), _p(k2), _p(beta),
                          float(prob.mu), _p(body) if body is not None else None, _p(p01),
                          _p(p02))
    else:
        lb.or_assemble(d, _p(nn), N, nc, _p(msh.X), _p(msh.cells), _p(msh.incptr),
                       _p(msh.inc), _p(rowptr), _p(cols), _p(vals), _p(f), _p(k1), _p(k2),
                       _p(beta), float(prob.mu), _p(body) if body is not None else None,
                       _p(p01), _p(p02))
    K = sp.csr_matrix((vals, cols, rowptr), shape=(ndof, ndof))
    if getattr(prob, "face_bc", None) is not None and np.any(prob.face_bc):
        K, f = velocity_bc(K, f, msh, prob)
    return System(msh, K, f, float(prob.mu))


def velocity_dofs(msh, prob):
    """Prescribed velocity DOFs and their values (section "Boundary
    conditions", eq. DG_GE_vBC): on a velocity face of network i (normal along
    axis a) the normal component u_i,a of every node of the face is given,
    from the nodal data u_bc_i.  Returns (mask [n_dof] bool, values [n_dof])."""
    d, N, n = msh.dim, msh.N, msh.n
    fb = np.asarray(prob.face_bc, dtype=np.int8).reshape(2, 2 * d)
    ids = np.arange(N)
    ax = []
    r = ids.copy()
    for a in range(d):
        ax.append(r % (n[a] + 1))
        r //= n[a] + 1
    fixed = np.zeros((2 * d + 2) * N, dtype=bool)
    g = np.zeros((2 * d + 2) * N)
    F = fields(d, N)
    for i, fu in enumerate(("u1", "u2")):
        ub = prob.u_bc_1 if i == 0 else prob.u_bc_2
        for a in range(d):
            for side in range(2):
                if not fb[i, 2 * a + side]:
                    continue
                nodes = ids[ax[a] == (n[a] if side else 0)]
                dof = F[fu].start + d * nodes + a
                fixed[dof] = True
                g[dof] = np.asarray(ub, dtype=np.float64).reshape(N, d)[nodes, a]
    return fixed, g


def velocity_bc(K, f, msh, prob):
    """Impose the prescribed normal velocities as essential conditions: the
    test space has w.n = 0 on the velocity faces, so their rows become identity
    rows with the data on the right, and the known values are moved out of the
    other rows (f - K g, columns removed).  The weak pressure term of those
    faces sits in exactly the rows that are replaced."""
    fixed, g = velocity_dofs(msh, prob)
    free = (~fixed).astype(np.float64)
    f2 = np.where(fixed, g, f - K @ g)
    Pf = sp.diags(free)
    K2 = (Pf @ K @ Pf + sp.diags(fixed.astype(np.float64))).tocsr()
    K2.sort_indices()
    return K2, f2


def spmv(K, x):
    """y = K x with the oracle's OpenMP CSR loop (large residual checks)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(K.shape[0])
    rp = np.ascontiguousarray(K.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(K.indices, dtype=np.int32)
    vv = np.ascontiguousarray(K.data, dtype=np.float64)
    lib().or_spmv(K.shape[0], _p(rp), _p(ci), _p(vv), _p(x), _p(y))
    return y


def blocks(sys_or_K, dim=None, N=None):
    """Sub-blocks of K by field (the fieldsplit index sets of the solver
    options listings): Kuu[i], Kup[i], Kpu[i], Kpp[i], K12, K21."""
    if isinstance(sys_or_K, System):
        K, dim, N = sys_or_K.K, sys_or_K.dim, sys_or_K.N
    else:
        K = sys_or_K
    F = fields(dim, N)
    K = K.tocsr()
    # a block is the rows of one field (a contiguous row range) restricted to
    # the columns of another: a selection of stored entries, no arithmetic
    def block(a, b):
        ra, cb = F[a], F[b]
        lo, hi = K.indptr[ra.start], K.indptr[ra.stop]
        cols = K.indices[lo:hi]
        keep = (cols >= cb.start) & (cols < cb.stop)
        counts = np.add.reduceat(keep.astype(np.int64), K.indptr[ra.start:ra.stop] - lo) \
            if hi > lo else np.zeros(ra.stop - ra.start, dtype=np.int64)
        # reduceat repeats the next value for empty rows: zero them
        counts[np.diff(K.indptr[ra.start:ra.stop + 1]) == 0] = 0
        indptr = np.concatenate([[0], np.cumsum(counts)])
        return sp.csr_matrix((K.data[lo:hi][keep], cols[keep] - cb.start, indptr),
                             shape=(ra.stop - ra.start, cb.stop - cb.start))

    out = dict(Kuu=[], Kup=[], Kpu=[], Kpp=[])
    for u, p in (("u1", "p1"), ("u2", "p2")):
        out["Kuu"].append(block(u, u))
        out["Kup"].append(block(u, p))
        out["Kpu"].append(block(p, u))
        out["Kpp"].append(block(p, p))
    out["K12"] = block("p1", "p2")
    out["K21"] = block("p2", "p1")
    return out


def selfp(sys_or_K, dim=None, N=None):
    """S_p^i = K_pp^i - K_pu^i diag(K_uu^i)^-1 K_up^i  (eqs. S4_sp1, S4_sp2).

    The inter-network blocks K12, K21 are left out: the preconditioner treats
    the two diagonal blocks of S_p separately (Method 2 of the solver section).
    """
    B = blocks(sys_or_K, dim, N)
    out = []
    for i in range(2):
        dinv = sp.diags(1.0 / B["Kuu"][i].diagonal())
        out.append((B["Kpp"][i] - B["Kpu"][i] @ dinv @ B["Kup"][i]).tocsr())
    return out


def solve_direct(K, f):
    """x* = K^-1 f by sparse LU (the plain definition of the discrete solution)."""
    return spla.spsolve(K.tocsc(), f)


def solve_dense(K, f):
    return np.linalg.solve(K.toarray(), f)


def sign_matrix(dim, N):
    """D = diag(I_u, -I_p): D K is symmetric for the CG-VMS operator."""
    F = fields(dim, N)
    s = np.ones((2 * dim + 2) * N)
    s[F["p1"]] = -1.0
    s[F["p2"]] = -1.0
    return s


def pure_flux(prob):
    """Velocity faces on every face of both networks: K is singular."""
    fb = getattr(prob, "face_bc", None)
    return fb is not None and bool(np.all(np.asarray(fb) != 0))


def nullspace(dim, N):
    """Kernel of K in the pure-flux case: u = 0, p1 = p2 = constant.  The
    test functions have w.n = 0 on the whole boundary, so -(div w; c) = 0,
    the pressure-gradient terms vanish on constants and the mass transfer
    beta (p1 - p2) pins p1 = p2.  Since K^T = D K D, it spans the left kernel
    as well."""
    F = fields(dim, N)
    n = np.zeros((2 * dim + 2) * N)
    n[F["p1"]] = 1.0
    n[F["p2"]] = 1.0
    return n


def consistent_rhs(f, dim, N):
    """The part of f in the range of K (f minus its component along the
    kernel): the nodal boundary data satisfy the compatibility condition of
    the continuous problem only up to the discretisation error."""
    n = nullspace(dim, N)
    return f - (n @ f) / (n @ n) * n


def pressure_mean(msh, p):
    """(1/|Omega|) int_Omega p_h for a P1 nodal vector p (exact for P1); on Q1
    box cells (all of one volume) a cell's integral is its volume times its
    vertex mean, also exact."""
    if msh.elem == "q1":
        return float(p[msh.cells].mean(1).mean())
    V = msh.X[msh.cells]
    J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(J)) / (2.0 if msh.dim == 2 else 6.0)
    return float(np.sum(vol * p[msh.cells].mean(1)) / vol.sum())


def normalize_pressures(msh, x):
    """Pure-flux case: the solution is fixed up to the kernel; the function
    space Q asks (int p1)(int p2) = 0, of which this takes int p1 = 0 (shift
    both pressures by the same constant)."""
    F = fields(msh.dim, msh.N)
    c = pressure_mean(msh, x[F["p1"]])
    y = x.copy()
    y[F["p1"]] -= c
    y[F["p2"]] -= c
    return y


def solve_pure_flux(S, f=None, transpose=False):
    """Solve the singular pure-flux system: the consistent part of the
    right-hand side, the solution orthogonal to the kernel (bordered system),
    then the pressure normalisation."""
    d, N = S.dim, S.N
    n = nullspace(d, N)
    b = consistent_rhs(S.f if f is None else f, d, N)
    K = S.K.T if transpose else S.K
    A = sp.bmat([[K, sp.csr_matrix(n[:, None])], [sp.csr_matrix(n[None, :]), None]]).tocsc()
    z = spla.spsolve(A, np.concatenate([b, [0.0]]))
    return normalize_pressures(S.mesh, z[:-1])
