"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test targets a plausible mistake: a dropped stabilisation term, a wrong
sign or index, a transposed block, a wrong facet integral, a wrong mesh.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import dpp_inputs as I
from oracle import dpp, mg, post, solver
from dense_cycles import cheb_error_matrix, cycle_matrix

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append(line.split())
    return out


# ------------------------------------------------------------ mesh / DoF --

def test_dof_table_2d_matches_paper():
    for n, dof in _rows("dof_2d_tri_cgvms.txt"):
        m = dpp.mesh(2, (int(n), int(n)))
        assert 6 * m.N == int(dof)
        assert m.nc == 2 * int(n) ** 2


def test_dof_table_3d_matches_paper():
    for n, printed, used in _rows("dof_3d_tet_cgvms.txt"):
        m = dpp.mesh(3, (int(n),) * 3) if int(n) <= 36 else None
        N = (int(n) + 1) ** 3 if m is None else m.N
        assert 8 * N == int(used)
        assert abs(int(printed) - int(used)) <= 1


def test_mesh_cells_are_kuhn_simplices():
    m = dpp.mesh(3, (3, 2, 2), (1.0, 2.0, 0.5))
    V = m.X[m.cells]
    J = V[:, 1:, :] - V[:, :1, :]
    vol = np.abs(np.linalg.det(J)) / 6.0
    assert np.allclose(vol, (1 / 3) * (2 / 2) * (0.5 / 2) / 6.0)
    assert np.isclose(vol.sum(), 1.0 * 2.0 * 0.5)
    # all 6 tets of a hex share the main diagonal
    assert np.all(m.cells.reshape(-1, 6, 4)[:, :, 0] == m.cells.reshape(-1, 6, 4)[:, :1, 0])


def test_nnz_formula():
    for dim, n, per_pair in ((2, 16, 16), (3, 5, 22), (2, 7, 16)):
        S = dpp.assemble(I.mms_problem(dim, n))
        assert S.K.nnz == per_pair * int(S.mesh.adjcnt.sum())
    S = dpp.assemble(I.mms_problem(2, 16))
    assert S.K.nnz == 30224
    # interior node stencils: 7 (TRI) and 15 (Kuhn TET) nodes
    assert dpp.mesh(2, (4, 4)).adjcnt.max() == 7
    assert dpp.mesh(3, (4, 4, 4)).adjcnt.max() == 15


# ------------------------------------------------------ element entries --

def test_hand_derived_entries_unit_square():
    prob = I.mms_problem(2, 1, k1=1.0, k2=0.1, beta=1.0, mu=1.0)
    X = dpp.mesh(2, (1, 1)).X
    prob.p0_1 = X[:, 0].copy()
    prob.p0_2 = np.ones(4)
    S = dpp.assemble(prob)
    K = S.K.toarray()
    N, d = 4, 2
    F = dpp.fields(d, N)

    def idx(field, node, comp):
        base = F[field].start
        return base + (d * node + comp if field.startswith("u") else node)

    n_checked = 0
    for row in _rows("element_2d_n1.txt"):
        if row[0] == "f":
            _, fld, node, comp, val = row
            assert S.f[idx(fld, int(node), int(comp))] == pytest.approx(float(val), abs=1e-15)
        else:
            rf, rn, rc, cf, cn, cc, val = row
            got = K[idx(rf, int(rn), int(rc)), idx(cf, int(cn), int(cc))]
            assert got == pytest.approx(float(val), abs=1e-15), row
        n_checked += 1
    assert n_checked >= 20


def test_block_identities():
    """K_pu = -K_up^T, D K symmetric, K12 = K21 = -(beta/mu) M (eq. S4_cg_stiffness_matrix)."""
    prob = I.grf_problem(3, 4)
    prob.beta = 0.7
    prob.mu = 1.3
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    for i in range(2):
        assert abs(B["Kpu"][i] + B["Kup"][i].T).max() == 0.0
        assert abs(B["Kpp"][i] - B["Kpp"][i].T).max() < 1e-15
    assert abs(B["K12"] - B["K21"].T).max() == 0.0
    DK = sp.diags(dpp.sign_matrix(3, S.N)) @ S.K
    assert abs(DK - DK.T).max() < 1e-15
    # K12 is -beta/mu times the P1 mass matrix: total = -beta/mu |Omega|
    assert B["K12"].sum() == pytest.approx(-0.7 / 1.3, rel=1e-13)
    # [K_pp^i  K_pp^ij] annihilates constants: the stiffness part has zero row
    # sums and the beta terms cancel
    one = np.ones(S.N)
    assert np.abs(B["Kpp"][0] @ one + B["K12"] @ one).max() < 1e-14
    assert np.abs(B["Kpp"][1] @ one + B["K21"] @ one).max() < 1e-14


@pytest.mark.parametrize("dim,n", [(3, (4, 3, 5)), (3, (1, 2, 3)), (2, (6, 5)), (2, (1, 4))])
def test_velocity_pressure_blocks_carry_no_coefficient(dim, n):
    """K_up^i has no permeability, beta or mu in it: in eq. CG_VMS_Weak_form the
    Galerkin term -(div w; p) has none and the stabilisation's mu k^-1 and k/mu
    cancel.  So with per-cell random k1, k2, beta and any mu, K_up^1 = K_up^2
    exactly, and on the box each entry (row node a, offset o, component c)
    depends only on a's boundary class (per axis: first, interior or last
    node).  Checked on the oracle's assembled K against the same box with
    unit coefficients; within a class the offsets agree exactly and the values
    to rounding (the oracle builds each cell's geometry from node coordinates,
    so differences like (i + 1) h - i h round differently across the box)."""
    rng = np.random.default_rng(11)
    prob = I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.7)
    prob.k1 = 10 ** rng.uniform(-2, 2, prob.n_cells)
    prob.k2 = 10 ** rng.uniform(-3, 1, prob.n_cells)
    prob.beta = 10 ** rng.uniform(-1, 1, prob.n_cells)
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    assert abs(B["Kup"][0] - B["Kup"][1]).max() == 0.0
    ref = dpp.assemble(I.mms_problem(dim, n, k1=1.0, k2=1.0, beta=1.0, mu=1.0))
    assert abs(dpp.blocks(ref)["Kup"][0] - B["Kup"][0]).max() <= 1e-15 * abs(B["Kup"][0]).max()
    # per boundary class: every node's row of K_up, arranged by offset, is the same
    m = [k + 1 for k in n]
    ijk = np.stack(np.unravel_index(np.arange(S.N), m[::-1])[::-1], axis=1)
    cls = sum(np.where(ijk[:, a] == 0, 0, np.where(ijk[:, a] == n[a], 2, 1)) * 3 ** a for a in range(dim))
    K = B["Kup"][0].tocsr()
    scale = abs(K).max()
    first = {}
    for a in range(S.N):
        for c in range(dim):
            r = dim * a + c
            cols = K.indices[K.indptr[r]:K.indptr[r + 1]]
            row = {tuple(ijk[b] - ijk[a]): v for b, v in zip(cols, K.data[K.indptr[r]:K.indptr[r + 1]])}
            ref_row = first.setdefault((cls[a], c), row)
            assert row.keys() == ref_row.keys(), (a, c)
            assert max(abs(row[o] - ref_row[o]) for o in row) <= 1e-13 * scale, (a, c)
    assert len({k[0] for k in first}) == np.unique(cls).size


def test_velocity_mass_and_boundary_identities():
    prob = I.mms_problem(3, 3, k1=2.0, k2=0.25, beta=1.0, mu=1.5)
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    N, d = S.N, 3
    # one component block of K_uu integrates to (mu/(2k)) |Omega|
    for i, k in enumerate((2.0, 0.25)):
        Kxx = B["Kuu"][i].toarray()[0::3, 0::3]
        assert Kxx.sum() == pytest.approx(1.5 / (2 * k), rel=1e-13)
    # K_up 1 = -oint psi_a n_c : zero on interior rows, facet moments on the boundary
    verts, normals, meas = post.boundary_facets(S.mesh)
    expect = np.zeros(d * N)
    for v, nv, m in zip(verts, normals, meas):
        for a in v:
            expect[d * a:d * a + d] -= nv * m / d
    got = B["Kup"][0] @ np.ones(N)
    assert np.abs(got - expect).max() < 1e-14


# ------------------------------------------------------ exact solutions --

@pytest.mark.parametrize("dim,n", [(2, 6), (3, 3)])
def test_patch_test_linear_solution_is_exact(dim, n):
    """p1 = p2 = a.x + c, u_i = (k_i/mu)(gamma b - a) solves the DPP equations
    (div u_i = 0, p1 - p2 = 0) and lies in P1; the residual-based CG-VMS terms
    vanish on it, so the discrete solution reproduces it exactly."""
    a = np.array([0.7, -1.3, 0.4][:dim])
    gb = np.array([0.2, 0.5, -0.1][:dim])
    k1, k2, mu = 2.0, 0.3, 1.7
    prob = I.mms_problem(dim, n, k1=k1, k2=k2, beta=3.0, mu=mu)
    X = dpp.mesh(dim, prob.n).X
    p = X @ a + 0.25
    prob.p0_1, prob.p0_2 = p.copy(), p.copy()
    prob.body = gb
    S = dpp.assemble(prob)
    x = dpp.solve_direct(S.K, S.f)
    F = dpp.fields(dim, S.N)
    assert np.abs(x[F["p1"]] - p).max() < 1e-12
    assert np.abs(x[F["p2"]] - p).max() < 1e-12
    assert np.abs(x[F["u1"]].reshape(-1, dim) - (k1 / mu) * (gb - a)).max() < 1e-12
    assert np.abs(x[F["u2"]].reshape(-1, dim) - (k2 / mu) * (gb - a)).max() < 1e-12


def test_dense_and_sparse_direct_agree():
    for dim, n in ((2, 8), (3, 3)):
        S = dpp.assemble(I.mms_problem(dim, n))
        xs = dpp.solve_direct(S.K, S.f)
        xd = dpp.solve_dense(S.K, S.f)
        assert np.linalg.norm(xs - xd) <= 1e-12 * np.linalg.norm(xd)


def _mms_errors(dim, ns, k2):
    out = []
    for n in ns:
        prob = I.mms_problem(dim, n, k1=1.0, k2=k2, beta=1.0, mu=1.0)
        S = dpp.assemble(prob)
        if S.K.shape[0] < 20000:
            x = dpp.solve_direct(S.K, S.f)
        else:  # the oracle's FGMRES, pinned against the direct solve elsewhere
            x = solver.solve(S, rtol=1e-12)[0]
        out.append(post.l2_errors(S, x, lambda X: I.mms_fields(dim, X, 1.0, k2, 1.0, 1.0),
                                   q=8 if dim == 2 else 6))
    return out


def test_mms_convergence_2d():
    """L2 errors decay as h^2 for all four fields (section "Two-dimensional study":
    slope alpha/d = 1 in DoA vs DoS, i.e. alpha = 2)."""
    ns = [8, 16, 32, 64]
    errs = _mms_errors(2, ns, 0.1)
    for f in ("p1", "p2"):
        assert post.rates([1 / n for n in ns], [e[f] for e in errs]).min() > 1.9
    for f in ("u1", "u2"):
        assert post.rates([1 / n for n in ns], [e[f] for e in errs]).min() > 1.8


def test_mms_convergence_3d():
    """3D manufactured solution with the parameters of the paper's 3D table
    (k1 = 1, k2 = 0.1, beta = mu = 1, section "Three-dimensional study")."""
    ns = [4, 8, 16]
    errs = _mms_errors(3, ns, 0.1)
    for f in ("p1", "p2"):
        assert post.rates([1 / n for n in ns], [e[f] for e in errs])[-1] > 1.9
    for f in ("u1", "u2"):
        assert post.rates([1 / n for n in ns], [e[f] for e in errs])[-1] > 1.8


def test_mms_3d_p2_reading():
    """The 3D micro-pressure uses mu/(beta k2): with k1 in its place the fields
    would not satisfy the mass balances, so errors would not decay."""
    for X in (np.random.default_rng(0).random((20, 3)),):
        k1, k2, beta, mu = 1.0, 0.1, 1.0, 1.0
        h = 1e-4
        p1, p2, u1, u2 = I.mms_fields(3, X, k1, k2, beta, mu)
        div = []
        for u_idx in (2, 3):
            dv = 0.0
            for c in range(3):
                e = np.zeros(3)
                e[c] = h
                up = I.mms_fields(3, X + e, k1, k2, beta, mu)[u_idx][:, c]
                um = I.mms_fields(3, X - e, k1, k2, beta, mu)[u_idx][:, c]
                dv = dv + (up - um) / (2 * h)
            div.append(dv)
        chi = -(beta / mu) * (p1 - p2)
        assert np.allclose(div[0], chi, rtol=1e-6, atol=1e-6)
        assert np.allclose(div[1], -chi, rtol=1e-6, atol=1e-6)


def test_mass_balance():
    """Testing with q1 = 1: oint u1.n = -(beta/mu) int (p1 - p2); with q1 = q2 = 1
    the transfer terms cancel: oint (u1 + u2).n = 0."""
    for dim, n, beta, mu in ((2, 12, 2.5, 1.3), (3, 4, 0.5, 2.0)):
        prob = I.mms_problem(dim, n, k1=1.0, k2=0.05, beta=beta, mu=mu)
        prob.k1 = prob.k1 * np.linspace(0.5, 2.0, prob.n_cells)
        S = dpp.assemble(prob)
        x = dpp.solve_direct(S.K, S.f)
        f1, f2, P1, P2 = post.balance(S, x)
        scale = abs(f1) + abs(f2) + abs(P1) + abs(P2)
        assert abs(f1 + beta / mu * (P1 - P2)) < 1e-11 * scale
        assert abs(f1 + f2) < 1e-11 * scale
        assert abs(f1) > 1e-3 * scale  # the check is not vacuous


def test_beta_zero_decouples_networks():
    prob = I.mms_problem(2, 6, k1=1.0, k2=0.2, beta=0.0, bc_params=(1.0, 0.2, 1.0, 1.0))
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    assert B["K12"].nnz == 0 or abs(B["K12"]).max() == 0.0
    F = dpp.fields(2, S.N)
    x = dpp.solve_direct(S.K, S.f)
    for u, p in (("u1", "p1"), ("u2", "p2")):
        idx = np.r_[np.arange(S.K.shape[0])[F[u]], np.arange(S.K.shape[0])[F[p]]]
        Ki = S.K[idx, :][:, idx]
        xi = dpp.solve_direct(Ki, S.f[idx])
        assert np.abs(xi - x[idx]).max() < 1e-12 * np.abs(x).max()


def test_network_swap_symmetry():
    prob = I.grf_problem(2, 6)
    S = dpp.assemble(prob)
    x = dpp.solve_direct(S.K, S.f)
    sw = I.grf_problem(2, 6)
    sw.k1, sw.k2 = prob.k2, prob.k1
    sw.p0_1, sw.p0_2 = prob.p0_2, prob.p0_1
    Sw = dpp.assemble(sw)
    y = dpp.solve_direct(Sw.K, Sw.f)
    F = dpp.fields(2, S.N)
    for a, b in (("u1", "u2"), ("p1", "p2")):
        assert np.abs(x[F[a]] - y[F[b]]).max() < 1e-11 * np.abs(x).max()


# ------------------------------------------------------- preconditioner --

def test_selfp_is_spd_and_matches_definition():
    S = dpp.assemble(I.grf_problem(3, 4))
    B = dpp.blocks(S)
    for i, Sp in enumerate(dpp.selfp(S)):
        A = Sp.toarray()
        assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
        np.linalg.cholesky(A)
        # against a dense evaluation of K_pp - K_pu diag(K_uu)^-1 K_up
        Kuu = B["Kuu"][i].toarray()
        ref = B["Kpp"][i].toarray() - B["Kpu"][i].toarray() @ np.diag(1 / np.diag(Kuu)) @ \
            B["Kup"][i].toarray()
        assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()
        # 65-point stencil in 3D
        assert np.diff(Sp.indptr).max() == 65


def test_interpolation_reproduces_linear_functions():
    for dim, n in ((2, (6, 5)), (3, (4, 3, 5)), (2, (7, 7))):
        P = mg.interpolation(dim, n)
        nc = mg.coarse_cells(n)
        # coarse node coordinates in fine index units (last node at n when n odd)
        ax = []
        for a in range(dim):
            lo, od, m = mg.axis_map(n[a])
            pos = np.zeros(m)
            for i in range(n[a] + 1):
                if od[i] == 0:
                    pos[lo[i]] = i
            ax.append(pos)
            assert m == nc[a] + 1
        Xc = np.stack(np.meshgrid(*ax, indexing="ij"), -1).transpose(
            tuple(range(dim))[::-1] + (dim,)).reshape(-1, dim)
        Xf = np.stack(np.meshgrid(*[np.arange(v + 1.0) for v in n], indexing="ij"), -1).transpose(
            tuple(range(dim))[::-1] + (dim,)).reshape(-1, dim)
        c = np.array([0.3, -1.1, 0.7][:dim])
        assert np.abs(P @ (Xc @ c + 2.0) - (Xf @ c + 2.0)).max() < 1e-13
        assert np.allclose(P.sum(1), 1.0)


def test_galerkin_coarse_operator_equals_rediscretisation():
    """On nested Kuhn meshes (n even) P^T A_h P of the P1 pressure stiffness
    equals the matrix assembled on the coarse mesh (Galerkin property)."""
    for dim, n in ((2, 8), (3, 4)):
        fine = dpp.assemble(I.mms_problem(dim, n, k1=1.0, k2=1.0, beta=0.0, bc_params=(1, 1, 1, 1)))
        coarse = dpp.assemble(I.mms_problem(dim, n // 2, k1=1.0, k2=1.0, beta=0.0, bc_params=(1, 1, 1, 1)))
        Af = dpp.blocks(fine)["Kpp"][0]
        Ac = dpp.blocks(coarse)["Kpp"][0]
        P = mg.interpolation(dim, (n,) * dim)
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac.toarray()).max() < 1e-14 * np.abs(Ac).max()


def test_chebyshev_degree_one_is_damped_jacobi_and_converges():
    S = dpp.assemble(I.mms_problem(2, 10))
    A = dpp.selfp(S)[0]
    dinv = 1 / A.diagonal()
    b = I.random_vector(A.shape[0], 7)
    x1 = mg.chebyshev(A, dinv, b, np.zeros_like(b), 1, 0.2, 1.8)
    assert np.allclose(x1, dinv * b / 1.0)
    lam = np.linalg.eigvals(np.diag(dinv) @ A.toarray()).real
    x = np.zeros_like(b)
    for _ in range(60):
        x = mg.chebyshev(A, dinv, b, x, 4, lam.min(), lam.max())
    assert np.linalg.norm(A @ x - b) < 1e-10 * np.linalg.norm(b)


def test_power_lambda_matches_dense_eigenvalue():
    """The smoother's upper bound.  After k normalised power steps from the
    hash start x_0 the estimate is ||M^k x_0|| / ||M^(k-1) x_0|| with
    M = D^-1 A; M^k is evaluated here through the eigendecomposition of M
    (real spectrum: M is similar to the SPD D^-1/2 A D^-1/2), so a dropped
    D^-1, a missing normalisation or an off-by-one step count fails it.  The
    estimate tends to the largest eigenvalue and the 15-step value the setup
    uses is within 10% of it."""
    for dim, n in ((2, 7), (3, 3)):
        S = dpp.assemble(I.grf_problem(dim, n))
        for A in dpp.selfp(S):
            dinv = 1.0 / A.diagonal()
            lam, Vec = np.linalg.eig(np.diag(dinv) @ A.toarray())
            assert np.abs(lam.imag).max() < 1e-10 * np.abs(lam.real).max()
            lam, Vec = lam.real, Vec.real
            lmax = lam.max()
            c0 = np.linalg.solve(Vec, mg.hash_start(A.shape[0]))
            for k in (1, 2, 15, 60):
                est = mg.power_lambda(A, dinv, k)
                ref = np.linalg.norm(Vec @ (lam ** k * c0)) / np.linalg.norm(Vec @ (lam ** (k - 1) * c0))
                assert abs(est - ref) < 1e-10 * ref, (dim, k, est, ref)
            assert abs(mg.power_lambda(A, dinv, 2000) - lmax) < 1e-3 * lmax
            assert 0.9 * lmax < mg.power_lambda(A, dinv, 15) < 1.1 * lmax
            # the undivided operator has a different spectrum (the D^-1 matters)
            assert abs(np.abs(np.linalg.eigvals(A.toarray())).max() - lmax) > 0.1 * lmax


@pytest.mark.parametrize("degree", [2, 3, 4])
def test_chebyshev_error_is_the_scaled_chebyshev_polynomial(degree):
    """k Chebyshev steps on [lo, hi] with diagonal preconditioning multiply the
    error by p_k(D^-1 A), p_k(t) = T_k((theta - t)/delta) / T_k(theta/delta)
    (theta, delta: centre and half-width of the interval).  The polynomial is
    evaluated on the eigenvalues of D^-1 A from numpy's Chebyshev basis, not
    from the three-term recurrence the smoother runs, so a wrong rho update or
    step coefficient fails it, on an interval that is not the spectrum's."""
    S = dpp.assemble(I.grf_problem(2, 5))
    A = dpp.selfp(S)[0]
    dinv = 1.0 / A.diagonal()
    Ad = A.toarray()
    lam, Vec = np.linalg.eig(np.diag(dinv) @ Ad)
    lam, Vec = lam.real, Vec.real
    lmax = lam.max()
    b = I.random_vector(A.shape[0], 11)
    xs = np.linalg.solve(Ad, b)
    x0 = I.random_vector(A.shape[0], 12)
    for lo, hi in ((0.3 * lmax, 1.1 * lmax), (0.05 * lmax, 0.9 * lmax)):
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(degree)
        pk = Tk((theta - lam) / delta) / Tk(theta / delta)
        e_pred = Vec @ (pk * np.linalg.solve(Vec, x0 - xs))
        x = mg.chebyshev(A, dinv, b, x0, degree, lo, hi)
        assert np.linalg.norm((x - xs) - e_pred) < 1e-10 * np.linalg.norm(x0 - xs), (lo, hi)


def test_interp_errors_pinned():
    """The interpolant-based error measure ||u_h - I_h u||_L2: zero on the nodal
    interpolant of any field; for linear exact fields (I_h u = u) it equals the
    quadrature-based true L2 error of random nodal data (a wrong mass matrix,
    volume or velocity reshape fails it); a constant pressure offset c gives
    |c| |Omega|^(1/2)."""
    for dim, n, L in ((2, (5, 4), (1.0, 0.7)), (3, (3, 2, 4), (1.0, 0.6, 0.8))):
        S = dpp.assemble(I.mms_problem(dim, n, L=L))
        msh = S.mesh
        N = msh.N
        F = dpp.fields(dim, N)

        def mms(X):
            return I.mms_fields(dim, X, 1.0, 0.1, 1.0, 1.0)

        x = np.zeros(S.K.shape[0])
        p1, p2, u1, u2 = mms(msh.X)
        x[F["p1"]], x[F["p2"]] = p1, p2
        x[F["u1"]], x[F["u2"]] = u1.reshape(-1), u2.reshape(-1)
        e = post.interp_errors(S, x, mms)
        assert max(e.values()) < 1e-13, e
        c = 0.37
        xc = x.copy()
        xc[F["p1"]] += c
        e = post.interp_errors(S, xc, mms)
        assert abs(e["p1"] - c * np.sqrt(np.prod(L))) < 1e-13 and e["p2"] < 1e-13

        a = np.array([0.4, -1.3, 0.8][:dim])

        def linear(X):
            s = X @ a
            return (s + 1.0, 2.0 * s - 0.5, np.outer(s, [1.0, -2.0, 0.5][:dim]) + 0.3,
                    np.outer(s, [-0.7, 0.2, 1.1][:dim]))

        xr = I.random_vector(S.K.shape[0], 21)
        ei, el = post.interp_errors(S, xr, linear), post.l2_errors(S, xr, linear, q=4)
        for f in ("u1", "p1", "u2", "p2"):
            assert abs(ei[f] - el[f]) < 1e-12 * el[f], (f, ei[f], el[f])


def test_vcycle_symmetric_and_contracting():
    S = dpp.assemble(I.mms_problem(3, 8, k2=1e-2))
    A = dpp.selfp(S)[1]
    # equal pre- and post-smoothing: the cycle is a symmetric operator
    sym = mg.MGOptions(coarse_max=50, pre_fine=2, post_fine=2, pre_coarse=2, post_coarse=2)
    H = mg.setup(A, 3, (8, 8, 8), sym)
    assert len(H.levels) == 3
    x, y = I.random_vector(A.shape[0], 1), I.random_vector(A.shape[0], 2)
    assert abs(mg.vcycle(H, x) @ y - x @ mg.vcycle(H, y)) < 1e-11 * np.linalg.norm(x) ** 2
    # error contraction of the stationary iteration e <- (I - V A) e, for the
    # symmetric cycle and the default post-smoothing-only cycle
    for opts in (sym, mg.MGOptions(coarse_max=50)):
        H = mg.setup(A, 3, (8, 8, 8), opts)
        e = I.random_vector(A.shape[0], 3)
        for _ in range(5):
            e = e - mg.vcycle(H, A @ e)
        e0 = e.copy()
        e = e - mg.vcycle(H, A @ e)
        assert np.sqrt(e @ (A @ e)) < 0.5 * np.sqrt(e0 @ (A @ e0)), opts
    # one level = exact inverse
    H1 = mg.setup(A, 3, (8, 8, 8), mg.MGOptions(coarse_max=10 ** 6))
    assert len(H1.levels) == 1
    b = I.random_vector(A.shape[0], 4)
    assert np.linalg.norm(A @ mg.vcycle(H1, b) - b) < 1e-11 * np.linalg.norm(b)


def test_post_only_two_grid_cycle_is_smoother_after_coarse_correction():
    """Without pre-smoothing, a two-level cycle is x = S_post(b; x0 = P Ac^-1
    P^T b): its error operator is E = M^post (I - P Ac^-1 P^T A), with the
    Chebyshev error polynomial M of the post-smoother, so applying the cycle to
    A e for e in range(P) (where the coarse correction is exact) leaves only
    the smoother's action on a zero error: V A e = e."""
    S = dpp.assemble(I.mms_problem(2, 12))
    A = dpp.selfp(S)[0]
    H = mg.setup(A, 2, (12, 12), mg.MGOptions(coarse_max=60))
    assert len(H.levels) == 2
    ec = I.random_vector(H.levels[1].A.shape[0], 8)
    e = H.levels[0].P @ ec
    assert np.linalg.norm(mg.vcycle(H, A @ e) - e) < 1e-11 * np.linalg.norm(e)


@pytest.mark.parametrize("case", ["default", "symmetric", "pre_fine", "pre_coarse", "q1"])
def test_vcycle_is_the_multigrid_error_propagation(case):
    """The cycle's values as a whole: vcycle(b) = B b with B from the
    error-propagation recursion of a multigrid cycle, built here from dense
    matrices (Chebyshev error polynomials through an eigendecomposition,
    explicit P, exact coarsest inverse) on three-level hierarchies.  Restricting
    b instead of the residual, P in place of P^T, adding the correction where
    it is assigned, a level class with the wrong degrees or a missing level
    fails it."""
    opts = {
        "default": mg.MGOptions(coarse_max=50),
        "symmetric": mg.MGOptions(coarse_max=50, pre_fine=2, post_fine=2, pre_coarse=2, post_coarse=2),
        "pre_fine": mg.MGOptions(coarse_max=50, pre_fine=1, post_fine=2, pre_coarse=0, post_coarse=3),
        "pre_coarse": mg.MGOptions(coarse_max=50, pre_fine=0, post_fine=3, pre_coarse=2, post_coarse=1),
        "q1": mg.MGOptions(coarse_max=50),
    }[case]
    if case == "q1":
        S = dpp.assemble(I.grf_problem(3, (6, 5, 6), elem="q1"))
        A, n, elem = dpp.selfp(S)[0], (6, 5, 6), "q1"
    elif case == "pre_coarse":
        S = dpp.assemble(I.grf_problem(2, (12, 11)))
        A, n, elem = dpp.selfp(S)[1], (12, 11), "p1"
        opts.coarse_max = 20
    else:
        S = dpp.assemble(I.grf_problem(3, (8, 7, 8)))
        A, n, elem = dpp.selfp(S)[1], (8, 7, 8), "p1"
    H = mg.setup(A, len(n), n, opts, elem=elem)
    assert len(H.levels) == 3, [lv.A.shape for lv in H.levels]
    B = cycle_matrix(H)
    for seed in (31, 32):
        b = I.random_vector(A.shape[0], seed)
        x = mg.vcycle(H, b)
        assert np.linalg.norm(x - B @ b) < 1e-10 * np.linalg.norm(B @ b), (case, seed)
    # the recursion is sensitive to the cycle's structure: a cycle that adds
    # its pre-smoothed iterate to the correction of b (not of the residual)
    # differs from it wherever there is pre-smoothing
    if opts.pre(0) > 0:
        lev = H.levels[0]
        Ad = lev.A.toarray()
        Spre = cheb_error_matrix(Ad, lev.dinv, opts.pre(0), lev.lo, lev.hi)
        Bpre = (np.eye(Ad.shape[0]) - Spre) @ np.linalg.inv(Ad)
        Bc = cycle_matrix(H, 1)
        Spost = cheb_error_matrix(Ad, lev.dinv, opts.post(0), lev.lo, lev.hi)
        x0 = Bpre @ b + lev.P.toarray() @ (Bc @ (lev.P.T @ b))
        wrong = Spost @ (x0 - np.linalg.solve(Ad, b)) + np.linalg.solve(Ad, b)
        assert np.linalg.norm(wrong - B @ b) > 1e-3 * np.linalg.norm(B @ b)


def test_fieldsplit_with_exact_blocks_is_exact_inverse():
    """The full block factorisation with exact A^-1 and the exact Schur complement
    S = D - C A^-1 B is K^-1 (signs and ordering of the fieldsplit apply)."""
    S = dpp.assemble(I.grf_problem(2, 4))
    P = solver.FieldSplit(S, inner="exact_schur")
    r = I.random_vector(S.K.shape[0], 11)
    z = P.apply(r)
    assert np.linalg.norm(S.K @ z - r) < 1e-10 * np.linalg.norm(r)
    x, its, res = solver.fgmres(S.K, S.f, P.apply, rtol=1e-12)
    assert its <= 2


def test_fgmres_reaches_direct_solution():
    S = dpp.assemble(I.mms_problem(3, 6, k2=1e-2))
    x, its, res = solver.solve(S, rtol=1e-12, mg_opts=mg.MGOptions(coarse_max=40))
    xd = dpp.solve_direct(S.K, S.f)
    assert res <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert 5 <= its <= 60


# ---------------------------------------------------------------- adjoint --

def test_adjoint_sign_similarity_and_dot_test():
    """K^T = D K D (D = diag(I_u, -I_p)), so K^T lam = g is lam = D K^-1 D g."""
    S = dpp.assemble(I.grf_problem(3, 3))
    D = dpp.sign_matrix(3, S.N)
    g = I.random_vector(S.K.shape[0], 5)
    lam = solver.adjoint_solve(S, g)
    lam2 = D * dpp.solve_direct(S.K, D * g)
    assert np.linalg.norm(lam - lam2) < 1e-11 * np.linalg.norm(lam)
    x = I.random_vector(S.K.shape[0], 6)
    assert abs((S.K.T @ lam) @ x - lam @ (S.K @ x)) < 1e-11 * np.linalg.norm(lam) * np.linalg.norm(x)


def test_parameter_gradient_matches_finite_differences():
    """dJ/d ln k1_e, dJ/d ln k2_e, dJ/d beta for J = ||p1 - p1_obs||^2 against
    central differences of the oracle's own forward solves."""
    prob = I.grf_problem(3, 3)
    S = dpp.assemble(prob)
    F = dpp.fields(3, S.N)
    obs = I.random_vector(S.N, 9)

    def J_of(k1, k2, beta):
        pr = I.grf_problem(3, 3)
        pr.k1, pr.k2, pr.beta = k1, k2, beta
        Sx = dpp.assemble(pr)
        x = dpp.solve_direct(Sx.K, Sx.f)
        return np.sum((x[F["p1"]] - obs) ** 2)

    x = dpp.solve_direct(S.K, S.f)
    g = np.zeros_like(x)
    g[F["p1"]] = 2.0 * (x[F["p1"]] - obs)
    lam = solver.adjoint_solve(S, g)
    g1, g2, gb = solver.param_gradient(S, prob, x, lam)
    for j, d in enumerate(I.random_directions(3, prob.n_cells, seed0=4000)):
        eps = 1e-5
        for which, grad in ((0, g1), (1, g2)):
            kp = [prob.k1.copy(), prob.k2.copy()]
            km = [prob.k1.copy(), prob.k2.copy()]
            kp[which] = kp[which] * np.exp(eps * d)
            km[which] = km[which] * np.exp(-eps * d)
            fd = (J_of(kp[0], kp[1], prob.beta) - J_of(km[0], km[1], prob.beta)) / (2 * eps)
            assert grad @ d == pytest.approx(fd, rel=1e-5, abs=1e-9)
    eps = 1e-5
    fd = (J_of(prob.k1, prob.k2, prob.beta + eps) - J_of(prob.k1, prob.k2, prob.beta - eps)) / (2 * eps)
    assert gb == pytest.approx(fd, rel=1e-5)


# ---- velocity (flux) boundaries: section "Boundary conditions", eq. DG_GE_vBC
FLUX_FACES = {2: [[1, 1, 0, 0], [0, 0, 0, 1]], 3: [[1, 0, 0, 0, 0, 1], [0, 0, 1, 1, 0, 0]]}


def test_velocity_bc_structure():
    """Essential normal velocities: identity rows holding the data, columns
    removed (D K stays symmetric, so the adjoint identity K^T = D K D holds),
    one fixed DOF per (network, node on a velocity face, face normal)."""
    import scipy.sparse as sp
    pr = I.mms_problem(3, (4, 3, 2), k2=0.1, flux_faces=FLUX_FACES[3])
    S = dpp.assemble(pr)
    fixed, g = dpp.velocity_dofs(S.mesh, pr)
    n = pr.n
    face_nodes = {0: (n[1] + 1) * (n[2] + 1), 1: (n[0] + 1) * (n[2] + 1), 2: (n[0] + 1) * (n[1] + 1)}
    expect = sum(face_nodes[f // 2] for i in range(2) for f in range(6) if FLUX_FACES[3][i][f])
    assert fixed.sum() == expect
    Dg = sp.diags(dpp.sign_matrix(3, S.N))
    assert abs(Dg @ S.K - (Dg @ S.K).T).max() == 0.0
    rows = S.K[np.flatnonzero(fixed)]
    assert (rows != sp.csr_matrix((np.ones(fixed.sum()), (np.arange(fixed.sum()), np.flatnonzero(fixed))),
                                  shape=rows.shape)).nnz == 0
    assert np.array_equal(S.f[fixed], g[fixed])
    x = dpp.solve_direct(S.K, S.f)
    assert np.array_equal(x[fixed], g[fixed])


@pytest.mark.parametrize("dim,ns", [(2, [8, 16, 32]), (3, [4, 8, 16])])
def test_velocity_bc_mms_convergence(dim, ns):
    """With the exact normal velocities prescribed on some faces and the exact
    pressures weakly on the others, the errors still decay as h^2: a wrong
    sign in the lifting f - K g, or a weak pressure term left on a velocity
    face, breaks the rate."""
    errs = []
    for n in ns:
        pr = I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.0, flux_faces=FLUX_FACES[dim])
        S = dpp.assemble(pr)
        if S.K.shape[0] < 20000:
            x = dpp.solve_direct(S.K, S.f)
        else:  # the oracle's FGMRES with its fieldsplit built on the same K
            x = solver.solve(S, rtol=1e-12)[0]
        errs.append(post.l2_errors(S, x, lambda X: I.mms_fields(dim, X, 1.0, 0.1, 1.0, 1.0), q=4))
    hs = [1 / n for n in ns]
    for f in ("p1", "p2"):
        assert post.rates(hs, [e[f] for e in errs])[-1] > 1.9
    for f in ("u1", "u2"):
        assert post.rates(hs, [e[f] for e in errs])[-1] > 1.85


def test_velocity_bc_gradient_matches_finite_differences():
    """With velocity faces the lifted right-hand side depends on k as well;
    the adjoint gradient (lam zeroed on the prescribed DOFs) against central
    differences of the oracle's forward solves."""
    rng = np.random.default_rng(12)
    base = I.mms_problem(3, (3, 2, 3), k2=0.1, flux_faces=FLUX_FACES[3])
    base.k1 = np.exp(0.5 * rng.standard_normal(base.n_cells))
    base.k2 = 0.1 * np.exp(0.5 * rng.standard_normal(base.n_cells))
    S = dpp.assemble(base)
    F = dpp.fields(3, S.N)
    obs = I.random_vector(S.N, 19)
    w = I.random_vector(3 * S.N, 20)

    def J_of(k1, k2):
        pr = I.mms_problem(3, (3, 2, 3), k2=0.1, flux_faces=FLUX_FACES[3])
        pr.k1, pr.k2 = k1, k2
        Sx = dpp.assemble(pr)
        x = dpp.solve_direct(Sx.K, Sx.f)
        return np.sum((x[F["p1"]] - obs) ** 2) + w @ x[F["u1"]]

    x = dpp.solve_direct(S.K, S.f)
    g = np.zeros_like(x)
    g[F["p1"]] = 2.0 * (x[F["p1"]] - obs)
    g[F["u1"]] = w
    lam = solver.adjoint_solve(S, g)
    g1, g2, _ = solver.param_gradient(S, base, x, lam)
    for d in I.random_directions(2, base.n_cells, seed0=4100):
        eps = 1e-5
        for which, grad in ((0, g1), (1, g2)):
            kp = [base.k1.copy(), base.k2.copy()]
            km = [base.k1.copy(), base.k2.copy()]
            kp[which] = kp[which] * np.exp(eps * d)
            km[which] = km[which] * np.exp(-eps * d)
            fd = (J_of(*kp) - J_of(*km)) / (2 * eps)
            assert grad @ d == pytest.approx(fd, rel=1e-5, abs=1e-9)


def _pure_flux_problem(dim, n):
    return I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.0,
                         flux_faces=[[1] * (2 * dim), [1] * (2 * dim)])


def test_pure_flux_kernel_and_compatibility():
    """Velocity faces everywhere: K has the kernel p1 = p2 = const (and, as
    K^T = D K D, the same left kernel); the interpolated boundary fluxes are
    compatible only up to the discretisation error, which decays as h^2."""
    incons = []
    for n in (8, 16, 32):
        S = dpp.assemble(_pure_flux_problem(2, n))
        nv = dpp.nullspace(2, S.N)
        scale = abs(S.K).max()
        assert np.abs(S.K @ nv).max() <= 1e-14 * scale * S.N
        assert np.abs(S.K.T @ nv).max() <= 1e-14 * scale * S.N
        incons.append(abs(nv @ S.f) / np.linalg.norm(S.f))
        x = dpp.solve_pure_flux(S)
        b = dpp.consistent_rhs(S.f, 2, S.N)
        assert np.linalg.norm(b - S.K @ x) <= 1e-11 * np.linalg.norm(b)
        assert abs(dpp.pressure_mean(S.mesh, x[dpp.fields(2, S.N)["p1"]])) < 1e-12
    assert post.rates([1 / 8, 1 / 16, 1 / 32], incons).min() > 1.8


@pytest.mark.parametrize("dim,ns", [(2, [8, 16, 32]), (3, [4, 8])])
def test_pure_flux_convergence(dim, ns):
    """The normalised discrete solution (int p1 = 0) against the manufactured
    solution normalised the same way converges at h^2 in the pressures."""
    errs = []
    for n in ns:
        S = dpp.assemble(_pure_flux_problem(dim, n))
        x = dpp.solve_pure_flux(S)
        p1e = I.mms_fields(dim, S.mesh.X, 1.0, 0.1, 1.0, 1.0)[0]
        ce = dpp.pressure_mean(S.mesh, p1e)
        ex = lambda Y: (lambda t: (t[0] - ce, t[1] - ce, t[2], t[3]))(I.mms_fields(dim, Y, 1.0, 0.1, 1.0, 1.0))
        errs.append(post.l2_errors(S, x, ex, q=4))
    hs = [1 / n for n in ns]
    for f in ("p1", "p2"):
        assert post.rates(hs, [e[f] for e in errs])[-1] > 1.9
    for f in ("u1", "u2"):
        assert post.rates(hs, [e[f] for e in errs])[-1] > 1.7
