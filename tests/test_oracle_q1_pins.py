"""Pins of the oracle's Q1 discretisation on box cells (the [Q1 + Q1]^2 rows
of the element table, the HEX columns of the 3D study) against what the paper
and the mathematics fix: the printed HEX DoF counts, the textbook assembled
trilinear (bilinear) mass and stiffness stencils, exact block identities, the
linear patch test, h^2 convergence to the manufactured solutions, the mass
balance, and the nested-mesh Galerkin identity of the Q1 interpolation."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import dpp_inputs as I
from oracle import dpp, mg, post, solver

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append(line.split())
    return out


def test_dof_table_hex_matches_paper():
    for n, printed, used in _rows("dof_3d_hex_cgvms.txt"):
        n = int(n)
        if n <= 17:
            S = dpp.assemble(I.mms_problem(3, n, elem="q1"))
            ndof = S.K.shape[0]
            assert S.mesh.nc == n ** 3
        else:
            ndof = 8 * (n + 1) ** 3
        assert ndof == int(used)
        assert abs(int(printed) - int(used)) <= 1


def test_q1_pattern_is_the_full_node_box():
    m = dpp.mesh(3, (4, 4, 4), elem="q1")
    assert m.adjcnt.max() == 27 and m.adjcnt.min() == 8
    assert dpp.mesh(2, (4, 4), elem="q1").adjcnt.max() == 9
    S = dpp.assemble(I.mms_problem(3, (3, 2, 4), elem="q1"))
    assert S.K.nnz == 22 * int(S.mesh.adjcnt.sum())


def _interior_stencil(A, dim, n, h):
    """Entries A(a, a + o) of the node a at the box centre, by offset o."""
    m = [n + 1] * dim
    c = [n // 2] * dim
    a = c[0] + m[0] * (c[1] + (m[1] * c[2] if dim == 3 else 0))
    out = {}
    rng = range(-1, 2)
    offs = [(dx, dy, dz) for dz in (rng if dim == 3 else [0]) for dy in rng for dx in rng]
    for o in offs:
        b = (c[0] + o[0]) + m[0] * ((c[1] + o[1]) + (m[1] * (c[2] + o[2]) if dim == 3 else 0))
        out[o] = A[a, b]
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_textbook_trilinear_mass_and_stiffness_stencils(dim):
    """With k = 2 mu and beta = 0 the pressure block is the Q1 stiffness matrix
    and the velocity block a quarter of the Q1 mass matrix.  At an interior
    node of a uniform grid of spacing h they are the textbook stencils:
    2D stiffness 8/3 (centre) and -1/3 (the 8 neighbours), mass h^2 (16, 4, 1)/36;
    3D stiffness h (8/3, 0, -1/6, -1/12) for centre, face, edge and corner
    neighbours, mass h^3 (64, 16, 4, 1)/216."""
    n = 6
    h = 1.0 / n
    prob = I.mms_problem(dim, n, k1=2.0, k2=2.0, beta=0.0, mu=1.0, elem="q1",
                         bc_params=(1.0, 0.1, 1.0, 1.0))
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    Kpp = B["Kpp"][0].toarray()
    Kuu = B["Kuu"][0].toarray()[::dim, ::dim] * 4.0   # component 0, mass matrix
    st = _interior_stencil(Kpp, dim, n, h)
    ms = _interior_stencil(Kuu, dim, n, h)
    for o, v in st.items():
        nz = sum(1 for t in o if t != 0)
        if dim == 2:
            ref_k = 8.0 / 3.0 if nz == 0 else -1.0 / 3.0
            ref_m = h * h * {0: 16, 1: 4, 2: 1}[nz] / 36.0
        else:
            ref_k = h * {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}[nz]
            ref_m = h ** 3 * {0: 64, 1: 16, 2: 4, 3: 1}[nz] / 216.0
        assert v == pytest.approx(ref_k, abs=1e-13), (o, v, ref_k)
        assert ms[o] == pytest.approx(ref_m, rel=1e-13), (o, ms[o], ref_m)


@pytest.mark.parametrize("dim,n", [(2, (4, 3)), (3, (3, 2, 4))])
def test_q1_block_identities(dim, n):
    prob = I.grf_problem(dim, n, elem="q1")
    prob.beta = np.linspace(0.5, 1.5, prob.n_cells)
    S = dpp.assemble(prob)
    B = dpp.blocks(S)
    for i in range(2):
        assert abs(B["Kpu"][i] + B["Kup"][i].T).max() <= 1e-14
        assert abs(B["Kuu"][i] - B["Kuu"][i].T).max() <= 1e-14
        assert abs(B["Kpp"][i] - B["Kpp"][i].T).max() <= 1e-14
    assert abs(B["K12"] - B["K21"].T).max() <= 1e-15
    D = dpp.sign_matrix(dim, S.N)
    DK = D @ S.K
    assert abs(DK - DK.T).max() <= 1e-13 * abs(S.K).max()
    # pressure rows annihilate constants in the stiffness part: with beta = 0
    prob.beta = 0.0
    S0 = dpp.assemble(prob)
    B0 = dpp.blocks(S0)
    for i in range(2):
        assert np.abs(B0["Kpp"][i] @ np.ones(S0.N)).max() <= 1e-13 * abs(B0["Kpp"][i]).max()


def test_q1_velocity_pressure_blocks_carry_no_coefficient():
    """K_up, K_pu of the CG-VMS form are free of k and beta, on Q1 too."""
    a = I.grf_problem(3, (3, 4, 2), elem="q1")
    b = I.mms_problem(3, (3, 4, 2), k1=7.0, k2=0.01, beta=3.0, elem="q1")
    Ba, Bb = dpp.blocks(dpp.assemble(a)), dpp.blocks(dpp.assemble(b))
    for i in range(2):
        assert abs(Ba["Kup"][i] - Bb["Kup"][i]).max() <= 1e-15
        assert abs(Ba["Kup"][0] - Bb["Kup"][1]).max() <= 1e-15


@pytest.mark.parametrize("dim,n", [(2, (5, 3)), (3, (3, 4, 2))])
def test_q1_patch_test_linear_solution_is_exact(dim, n):
    """p1 = p2 = a.x + c, u_i = -(k_i/mu) a solves the DPP equations for any
    beta and lies in Q1; the stabilisation vanishes on it, so the discrete
    solution reproduces it (weak pressure data on every face, Q1 face
    integrals of the boundary interpolant)."""
    rng = np.random.default_rng(5)
    avec = rng.normal(size=dim)
    c = 0.7
    k1, k2, mu = 1.3, 0.4, 0.9
    prob = I.mms_problem(dim, n, k1=k1, k2=k2, beta=2.0, mu=mu, L=(1.0, 0.8, 1.2)[:dim], elem="q1")
    X = I.node_coords(dim, prob.n, prob.L)
    p = X @ avec + c
    prob.p0_1, prob.p0_2 = p.copy(), p.copy()
    S = dpp.assemble(prob)
    x = dpp.solve_direct(S.K, S.f)
    F = dpp.fields(dim, S.N)
    assert np.abs(x[F["p1"]] - p).max() <= 1e-12
    assert np.abs(x[F["p2"]] - p).max() <= 1e-12
    assert np.abs(x[F["u1"]].reshape(-1, dim) + (k1 / mu) * avec).max() <= 1e-11
    assert np.abs(x[F["u2"]].reshape(-1, dim) + (k2 / mu) * avec).max() <= 1e-11


@pytest.mark.parametrize("dim,ns", [(2, (8, 16, 32)), (3, (4, 8, 16))])
def test_q1_mms_convergence(dim, ns):
    """L2 rates of order 2 for every field (CG-VMS on Q1, as on P1)."""
    errs = []
    for n in ns:
        prob = I.mms_problem(dim, n, k1=1.0, k2=0.1, elem="q1")
        S = dpp.assemble(prob)
        if S.K.shape[0] <= 30000:
            x = dpp.solve_direct(S.K, S.f)
        else:  # the oracle's own FGMRES, far below the discretisation error
            x, its, res = solver.solve(S, rtol=1e-11, maxiter=400)
            assert res <= 1e-11
        errs.append(post.l2_errors(S, x, lambda X: I.mms_fields(dim, X, 1.0, 0.1, 1.0, 1.0), q=4))
    hs = [1.0 / n for n in ns]
    for f, lo in (("p1", 1.9), ("p2", 1.9), ("u1", 1.85), ("u2", 1.85)):
        assert post.rates(hs, [e[f] for e in errs])[-1] > lo, (f, errs)


@pytest.mark.parametrize("dim,n,L", [(2, (5, 3), (1.0, 0.7)), (3, (3, 2, 4), (1.0, 0.6, 0.8))])
def test_q1_l2_errors_pinned(dim, n, L):
    """The error integral on box cells (post.l2_errors with Q1): zero on the
    nodal interpolant of multilinear exact fields; for linear exact fields
    (which Q1 reproduces) and random nodal data, the squared error is the sum
    over cells of e^T M e with the textbook Q1 mass matrix, the tensor product
    of the one-dimensional (h/6)[[2, 1], [1, 2]] (built here from the corner
    coordinates, so a wrong basis, weight, point map or cell volume fails
    it); a constant pressure offset c gives |c| |Omega|^(1/2)."""
    prob = I.mms_problem(dim, n, L=L, elem="q1")
    S = dpp.assemble(prob)
    msh = S.mesh
    N = msh.N
    F = dpp.fields(dim, N)
    h = np.array([L[a] / n[a] for a in range(dim)])

    def multilinear(X):
        t = np.prod(X + 0.3, axis=1)
        return (t + X[:, 0], 2.0 * t - 0.5, np.outer(t, [1.0, -2.0, 0.5][:dim]) + 0.3,
                np.outer(t - X[:, -1], [-0.7, 0.2, 1.1][:dim]))

    def nodal(fn):
        p1, p2, u1, u2 = fn(msh.X)
        x = np.zeros(S.K.shape[0])
        x[F["p1"]], x[F["p2"]] = p1, p2
        x[F["u1"]], x[F["u2"]] = u1.reshape(-1), u2.reshape(-1)
        return x

    e = post.l2_errors(S, nodal(multilinear), multilinear, q=3)
    assert max(e.values()) < 1e-13, e
    xc = nodal(multilinear)
    xc[F["p2"]] += 0.37
    e = post.l2_errors(S, xc, multilinear, q=3)
    assert abs(e["p2"] - 0.37 * np.sqrt(np.prod(L))) < 1e-13 and e["p1"] < 1e-13

    a = np.array([0.4, -1.3, 0.8][:dim])

    def linear(X):
        s_ = X @ a
        return (s_ + 1.0, 2.0 * s_ - 0.5, np.outer(s_, [1.0, -2.0, 0.5][:dim]) + 0.3,
                np.outer(s_, [-0.7, 0.2, 1.1][:dim]))

    xr = I.random_vector(S.K.shape[0], 23)
    d = xr - nodal(linear)
    ref = dict(u1=0.0, p1=0.0, u2=0.0, p2=0.0)
    for cell in msh.cells:
        V = msh.X[cell]
        same = np.abs(V[:, None, :] - V[None, :, :]) < 1e-12 * h   # [v, w, axis]
        M = np.prod(np.where(same, h / 3.0, h / 6.0), axis=-1)
        for f in ("p1", "p2"):
            ev = d[F[f]][cell]
            ref[f] += ev @ M @ ev
        for f in ("u1", "u2"):
            ev = d[F[f]].reshape(N, dim)[cell]
            ref[f] += np.einsum("vc,vw,wc->", ev, M, ev)
    got = post.l2_errors(S, xr, linear, q=2)
    for f in ("u1", "p1", "u2", "p2"):
        assert abs(got[f] - np.sqrt(ref[f])) < 1e-12 * np.sqrt(ref[f]), (f, got[f], np.sqrt(ref[f]))


@pytest.mark.parametrize("faces", [False, True])
def test_q1_parameter_gradient_matches_finite_differences(faces):
    """dJ/d ln k1_e, dJ/d ln k2_e and dJ/d beta on box cells, J = ||p1 - obs||^2,
    against central differences of the oracle's own Q1 forward solves (with and
    without velocity faces)."""
    ff = [[1, 0, 0, 1, 0, 0], [0, 0, 1, 0, 0, 1]] if faces else None
    rng = np.random.default_rng(5)

    def problem():
        return I.mms_problem(3, (3, 2, 3), k1=1.0, k2=0.1, beta=0.7, mu=1.2, elem="q1", flux_faces=ff)

    prob = problem()
    prob.k1 = 10 ** rng.uniform(-1, 1, prob.n_cells)
    prob.k2 = 10 ** rng.uniform(-2, 0, prob.n_cells)
    S = dpp.assemble(prob)
    F = dpp.fields(3, S.N)
    obs = I.random_vector(S.N, 19)

    def J_of(k1, k2, beta):
        pr = problem()
        pr.k1, pr.k2, pr.beta = k1, k2, beta
        Sx = dpp.assemble(pr)
        xx = dpp.solve_direct(Sx.K, Sx.f)
        return np.sum((xx[F["p1"]] - obs) ** 2)

    x = dpp.solve_direct(S.K, S.f)
    g = np.zeros_like(x)
    g[F["p1"]] = 2.0 * (x[F["p1"]] - obs)
    lam = solver.adjoint_solve(S, g)
    g1, g2, gb = solver.param_gradient(S, prob, x, lam)
    assert g1.shape == (prob.n_cells,)
    eps = 1e-5
    for d in I.random_directions(2, prob.n_cells, seed0=4100):
        for which, grad in ((0, g1), (1, g2)):
            kp = [prob.k1.copy(), prob.k2.copy()]
            km = [prob.k1.copy(), prob.k2.copy()]
            kp[which] = kp[which] * np.exp(eps * d)
            km[which] = km[which] * np.exp(-eps * d)
            fd = (J_of(kp[0], kp[1], prob.beta) - J_of(km[0], km[1], prob.beta)) / (2 * eps)
            assert grad @ d == pytest.approx(fd, rel=1e-5, abs=1e-9)
    fd = (J_of(prob.k1, prob.k2, prob.beta + eps) - J_of(prob.k1, prob.k2, prob.beta - eps)) / (2 * eps)
    assert gb == pytest.approx(fd, rel=1e-5)


def test_q1_mass_balance():
    prob = I.grf_problem(3, 6, elem="q1")
    S = dpp.assemble(prob)
    x = dpp.solve_direct(S.K, S.f)
    f1, f2, i1, i2 = post.balance(S, x)
    assert abs(f1 + f2) <= 1e-11 * max(abs(f1), 1.0)
    assert abs(f1 + (prob.beta / prob.mu) * (i1 - i2)) <= 1e-10 * max(abs(f1), 1.0)


def test_q1_interpolation_reproduces_trilinear_functions():
    for dim, n in ((2, (6, 5)), (3, (4, 5, 3))):
        P = mg.interpolation_q1(dim, n)
        nc = mg.coarse_cells(n)
        Xf = I.node_coords(dim, n)
        # coarse node positions in fine index space (the last one at n when n is odd)
        pos = [np.array([2 * c if 2 * c <= n[a] else n[a] for c in range(nc[a] + 1)], float) / n[a]
               for a in range(dim)]
        grids = np.meshgrid(*pos, indexing="ij")
        Xc = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids], 1)
        rng = np.random.default_rng(1)
        coef = rng.normal(size=2 ** dim)

        def f(X):
            out = np.zeros(len(X))
            for v in range(2 ** dim):
                t = np.ones(len(X))
                for a in range(dim):
                    if (v >> a) & 1:
                        t = t * X[:, a]
                out += coef[v] * t
            return out
        assert np.abs(P @ f(Xc) - f(Xf)).max() <= 1e-13


def test_q1_galerkin_equals_rediscretisation_on_nested_meshes():
    """Conforming nested Q1 spaces: P^T A_h P is the stiffness matrix of the
    coarse mesh (pressure block with k = 2 mu, beta = 0)."""
    for dim, n in ((2, (8, 6)), (3, (4, 4, 6))):
        fine = dpp.blocks(dpp.assemble(I.mms_problem(dim, n, k1=2.0, k2=2.0, beta=0.0, elem="q1",
                                                     bc_params=(1.0, 0.1, 1.0, 1.0))))
        nc = mg.coarse_cells(n)
        coarse = dpp.blocks(dpp.assemble(I.mms_problem(dim, nc, k1=2.0, k2=2.0, beta=0.0, elem="q1",
                                                     bc_params=(1.0, 0.1, 1.0, 1.0))))
        P = mg.interpolation_q1(dim, n)
        G = (P.T @ fine["Kpp"][0] @ P).toarray()
        assert np.abs(G - coarse["Kpp"][0].toarray()).max() <= 1e-13


def test_q1_fieldsplit_and_fgmres_reach_the_direct_solution():
    prob = I.grf_problem(3, 6, elem="q1")
    S = dpp.assemble(prob)
    xd = dpp.solve_direct(S.K, S.f)
    F = solver.FieldSplit(S, inner="exact_selfp", velocity="exact")
    x, its, res = solver.fgmres(S.K, S.f, F.apply, rtol=1e-12)
    assert res <= 1e-12 and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    x, its, res = solver.solve(S, rtol=1e-12, mg_opts=mg.MGOptions(coarse_max=30))
    assert res <= 1e-12 and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_q1_pure_flux_solution_and_pressure_mean():
    """Velocity faces everywhere on Q1 boxes: the bordered solve returns a
    solution of K x = f (consistent part) with int p1 = 0, and the Q1 pressure
    mean is exact on trilinear functions."""
    prob = I.mms_problem(3, (3, 2, 4), k1=1.0, k2=0.1, flux_faces=[[1] * 6, [1] * 6], elem="q1")
    S = dpp.assemble(prob)
    X = S.mesh.X
    # int over the unit box of x y z = 1/8 (trilinear, reproduced by Q1)
    assert dpp.pressure_mean(S.mesh, X[:, 0] * X[:, 1] * X[:, 2]) == pytest.approx(0.125, abs=1e-14)
    x = dpp.solve_pure_flux(S)
    F = dpp.fields(3, S.N)
    assert abs(dpp.pressure_mean(S.mesh, x[F["p1"]])) <= 1e-12 * np.abs(x[F["p1"]]).max()
    fc = dpp.consistent_rhs(S.f, 3, S.N)
    assert np.linalg.norm(S.K @ x - fc) <= 1e-10 * np.linalg.norm(fc)
