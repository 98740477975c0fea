"""Q1 box cells (the [Q1 + Q1]^2 CG-VMS rows of the element table, the HEX and
QUAD columns of the studies) on the GPU path against the oracle through the
C ABI: assembly (CSR and f), operator products, selfp, the multigrid
hierarchy with the trilinear transfers and every level-kernel shape, the
fieldsplit apply, FP64 and mixed-precision solves, velocity faces, graph
replay, the full-size 64^3 workload by the oracle's residual, and the calls
that are P1 only.  Bars as in test_gpu_parity."""
import numpy as np
import pytest
import scipy.sparse as sp

import dpp_inputs as I
from oracle import dpp as odpp
from oracle import mg as omg
from oracle import solver as osolver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def lib():
    import paper_1808_08328_amd as dpp
    return dpp


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _ragged2d():
    q = I.mms_problem(2, (9, 6), k1=1.0, k2=0.1, beta=2.0, mu=1.3, L=(1.0, 0.7), elem="q1")
    q.k1 = I.hex_to_cells(10 ** I.grf_log10((9, 6), 2, 5, 0.0, 1.0), 2, "q1")
    q.k2 = q.k1 * 0.05
    q.body = np.array([0.4, -0.3])
    return q


def _ragged3d():
    q = I.mms_problem(3, (5, 3, 4), k1=1.0, k2=0.1, beta=1.0, mu=0.8, L=(1.0, 0.6, 0.8), elem="q1")
    q.k1 = I.hex_to_cells(10 ** I.grf_log10((5, 3, 4), 3, 7, 0.0, 1.0), 3, "q1")
    q.k2 = I.hex_to_cells(10 ** I.grf_log10((5, 3, 4), 3, 8, -2.0, 1.0), 3, "q1")
    q.beta = np.linspace(0.5, 1.5, q.n_cells)
    q.body = np.array([0.3, -0.2, 0.1])
    return q


CASES = {
    "2d_ragged_body": _ragged2d,
    "3d_ragged_body": _ragged3d,
    "3d_8_mms": lambda: I.mms_problem(3, 8, k1=1.0, k2=1e-2, elem="q1"),
    "3d_thin_1x3x2": lambda: I.mms_problem(3, (1, 3, 2), k2=0.1, elem="q1"),
    "2d_thin_3x1": lambda: I.mms_problem(2, (3, 1), k2=0.2, elem="q1"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_q1_assembly_and_products_match_oracle(case):
    print("q1 case", case, flush=True)
    prob = CASES[case]()
    S = odpp.assemble(prob)
    P = lib().assemble_problem(prob)
    assert P.n_dof == S.K.shape[0] and P.nnz == S.K.nnz
    rp, ci, vv = P.export_csr()
    assert np.array_equal(H(rp), S.K.indptr)
    assert np.array_equal(H(ci), S.K.indices)
    assert np.abs(H(vv) - S.K.data).max() <= 1e-13 * np.abs(S.K.data).max()
    f = H(P.rhs())
    assert np.abs(f - S.f).max() <= 1e-13 * np.abs(S.f).max()
    x = I.random_vector(P.n_dof, 1)
    assert relmax(H(P.spmv(T(x))), S.K @ x) <= 1e-13
    B = odpp.blocks(S)
    xp = I.random_vector(P.n_nodes, 2)
    xu = I.random_vector(P.dim * P.n_nodes, 3)
    for i in range(2):
        assert relmax(H(P.spmv(T(xp), which=1 + i)), B["Kup"][i] @ xp) <= 1e-13
        assert relmax(H(P.spmv(T(xu), which=3 + i)), B["Kpu"][i] @ xu) <= 1e-13


@pytest.mark.parametrize("case,cmax", [("2d_ragged_body", 10), ("3d_ragged_body", 8), ("3d_8_mms", 40)])
def test_q1_hierarchy_cycle_and_fieldsplit_match_oracle(case, cmax):
    prob = CASES[case]()
    S = odpp.assemble(prob)
    P = lib().assemble_problem(prob)
    pc = P.setup_precond(coarse_max=cmax)
    info = pc.info()
    Sp = odpp.selfp(S)
    Hs = [omg.setup(Sp[i], prob.dim, prob.n, omg.MGOptions(coarse_max=cmax), elem="q1") for i in range(2)]
    assert info["levels"] == len(Hs[0].levels) >= 2
    for i in range(2):
        for l, lev in enumerate(Hs[i].levels):
            x = I.random_vector(lev.A.shape[0], 10 + l)
            assert relmax(H(pc.level_spmv(l, i, T(x))), lev.A @ x) <= 1e-13, (i, l)
            if l < len(Hs[i].levels) - 1:
                assert info["hi"][l][i] == pytest.approx(lev.hi, rel=1e-10)
    N = P.n_nodes
    b = I.random_vector(2 * N, 21)
    xg = H(pc.vcycle(T(b)))
    for i in range(2):
        assert relmax(xg[i * N:(i + 1) * N], omg.vcycle(Hs[i], b[i * N:(i + 1) * N])) <= 1e-11
    F = osolver.FieldSplit(S, omg.MGOptions(coarse_max=cmax))
    r = I.random_vector(P.n_dof, 22)
    assert relmax(H(pc.apply(T(r))), F.apply(r)) <= 1e-11


@pytest.mark.parametrize("case,cmax", [("2d_ragged_body", 10), ("3d_8_mms", 10), ("3d_ragged_body", 8)])
def test_q1_every_level_kernel_shape_matches_oracle(case, cmax):
    """All lanes-per-row / symmetric-storage variants on the 125-point (25 in
    2D) Q1 level stencils; 3d_8_mms has an odd node count on every level, and
    3d_ragged_body a level with two nodes along y and z, where stored offsets
    such as (-2, -2, 1) have a negative linear offset (the mirror reads of the
    symmetric storage must stay masked there)."""
    prob = CASES[case]()
    S = odpp.assemble(prob)
    P = lib().assemble_problem(prob)
    pc = P.setup_precond(coarse_max=cmax)
    Hs = [omg.setup(sp_, prob.dim, prob.n, omg.MGOptions(coarse_max=cmax), elem="q1")
          for sp_ in odpp.selfp(S)]
    nlev = pc.info()["levels"]
    assert nlev >= 3
    N = P.n_nodes
    b = I.random_vector(2 * N, 5)
    ref = np.concatenate([omg.vcycle(Hs[i], b[i * N:(i + 1) * N]) for i in range(2)])
    for lanes in (0, 1, 2, 4, 8):
        for sym in (0, 1):
            for l in range(nlev - 1):
                pc.set_shape(l, lanes, sym)
            x = I.random_vector(N, 6)
            for i in range(2):
                assert relmax(H(pc.level_spmv(0, i, T(x))), Hs[i].levels[0].A @ x) <= 1e-13
            assert relmax(H(pc.vcycle(T(b))), ref) <= 1e-11, (lanes, sym)


@pytest.mark.parametrize("case", list(CASES))
def test_q1_fp64_solve_matches_oracle_direct_solve(case):
    prob = CASES[case]()
    S = odpp.assemble(prob)
    xo = odpp.solve_direct(S.K, S.f)
    P = lib().assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    # the boxes one cell thick have cond(K) ~ 1e3 (measured: 1.4e3 at 1x3x2),
    # so the residual bar that gives 1e-10 per field is 1e-14 there
    rtol = 1e-14 if P.n_dof < 2000 else 1e-12
    x, st = P.solve(pc, rtol=rtol, maxiter=600)
    x = H(x)
    assert st.converged == 1 and st.rel_residual <= rtol
    F = odpp.fields(prob.dim, S.N)
    for f in ("u1", "p1", "u2", "p2"):
        assert np.linalg.norm(x[F[f]] - xo[F[f]]) <= 1e-10 * np.linalg.norm(xo[F[f]]), f
    assert np.linalg.norm(S.f - S.K @ x) <= 1.05 * rtol * np.linalg.norm(S.f)


@pytest.mark.parametrize("precision", [1, 2])
def test_q1_mixed_precision_matches_oracle(precision):
    prob = I.grf_problem(3, 8, elem="q1")
    S = odpp.assemble(prob)
    xo = odpp.solve_direct(S.K, S.f)
    P = lib().assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    x, st = P.solve(pc, rtol=1e-10, precision=precision, maxiter=600)
    x = H(x)
    assert st.converged == 1
    F = odpp.fields(3, S.N)
    for f in ("u1", "p1", "u2", "p2"):
        assert np.linalg.norm(x[F[f]] - xo[F[f]]) <= 1e-7 * np.linalg.norm(xo[F[f]]), f


def test_q1_graph_replay_matches_eager_solve():
    prob = I.mms_problem(3, 10, k1=1.0, k2=1e-2, elem="q1")
    P = lib().assemble_problem(prob)
    pc = P.setup_precond(coarse_max=60)
    xe, se = P.solve(pc, rtol=1e-10)
    for rep in range(2):
        xg, sg = P.solve(pc, rtol=1e-10, use_graph=1)
        assert torch.equal(xg, xe) and sg.iters == se.iters, rep
        y = P.spmv(xg)
        torch.cuda.synchronize()
        del y


@pytest.mark.parametrize("faces", [[[1, 0, 0, 1, 0, 0], [0, 1, 1, 0, 0, 1]], [[1] * 6, [1] * 6]])
def test_q1_velocity_faces_match_oracle(faces):
    """Velocity faces on Q1 boxes (essential u.n by elimination), including
    every face of both networks (pure flux: consistent right-hand side,
    int p1 = 0)."""
    prob = I.mms_problem(3, (4, 3, 5), k1=1.0, k2=0.1, beta=1.0, mu=0.8, L=(1.0, 0.6, 0.8),
                         flux_faces=faces, elem="q1")
    S = odpp.assemble(prob)
    P = lib().assemble_problem(prob)
    rp, ci, vv = P.export_csr()
    Kg = sp.csr_matrix((H(vv), H(ci), H(rp)), shape=S.K.shape)
    assert abs(Kg - S.K).max() <= 1e-13 * np.abs(S.K.data).max()
    assert relmax(H(P.rhs()), S.f) <= 1e-13
    x = I.random_vector(P.n_dof, 1)
    assert relmax(H(P.spmv(T(x))), S.K @ x) <= 1e-13
    pc = P.setup_precond(coarse_max=30)
    F = osolver.FieldSplit(S, omg.MGOptions(coarse_max=30))
    r = I.random_vector(P.n_dof, 22)
    assert relmax(H(pc.apply(T(r))), F.apply(r)) <= 1e-11
    # cond(K) of these small boxes is ~1e3: solve to 1e-14 for the 1e-10 bar
    xs, st = P.solve(pc, rtol=1e-14, maxiter=600)
    assert st.converged
    xo = odpp.solve_pure_flux(S) if odpp.pure_flux(prob) else odpp.solve_direct(S.K, S.f)
    Fd = odpp.fields(3, S.N)
    xg = H(xs)
    for f in ("u1", "p1", "u2", "p2"):
        e = np.linalg.norm(xg[Fd[f]] - xo[Fd[f]]) / np.linalg.norm(xo[Fd[f]])
        print(f, "%.2e" % e, flush=True)
        assert e <= 1e-10, f


@pytest.mark.timeout(900)
def test_q1_full_size_solve_oracle_residual():
    """The 64^3 Q1 workload (2,197,000 DOF) in the benchmark's launch
    configuration: the oracle's own FP64 K applied to the GPU solution at
    1e-8, and 2000 sampled rows of K."""
    import time
    t0 = time.time()

    def step(msg):
        print("full-size Q1 64^3: %s (%.1f s)" % (msg, time.time() - t0), flush=True)

    step("start")
    prob = I.make_config("h2_3d64_q1")
    P = lib().assemble_problem(prob)
    step("assembled")
    pc = P.setup_precond()
    step("preconditioner set up")
    x, st = P.solve(pc)
    step("solved in %d iterations" % st.iters)
    assert st.converged == 1
    S = odpp.assemble(prob)
    step("oracle assembled")
    r = S.f - odpp.spmv(S.K, H(x))
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(S.f)
    rp, ci, vv = P.export_csr()
    step("exported")
    rows = np.random.default_rng(0).integers(0, P.n_dof, 2000)
    rph, cih, vvh = H(rp), H(ci), H(vv)
    scale = np.abs(S.K.data).max()
    for rr in rows:
        a, b = rph[rr], rph[rr + 1]
        assert np.array_equal(cih[a:b], S.K.indices[S.K.indptr[rr]:S.K.indptr[rr + 1]])
        assert np.abs(vvh[a:b] - S.K.data[S.K.indptr[rr]:S.K.indptr[rr + 1]]).max() <= 1e-13 * scale


@pytest.mark.parametrize("faces", [False, True])
def test_q1_adjoint_and_gradient_match_oracle(faces):
    """Adjoint solve and per-box parameter gradient on Q1 box cells against the
    oracle's LU of K^T and its box-cell gradient (pinned to finite
    differences), with and without velocity faces."""
    dpp = lib()
    rng = np.random.default_rng(7)
    ff = [[1, 0, 0, 1, 0, 0], [0, 0, 1, 0, 0, 1]] if faces else None
    prob = I.mms_problem(3, (5, 4, 6), k1=1.0, k2=0.1, beta=0.7, mu=1.2, elem="q1", flux_faces=ff)
    prob.k1 = 10 ** rng.uniform(-1, 1, prob.n_cells)
    prob.k2 = 10 ** rng.uniform(-2, 0, prob.n_cells)
    print("q1 gradient case faces", faces, flush=True)
    S = odpp.assemble(prob)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    x, st = P.solve(pc, rtol=1e-12)
    assert st.converged
    F = odpp.fields(3, S.N)
    obs = I.random_vector(S.N, 33)
    xh = H(x)
    g = np.zeros(P.n_dof)
    g[F["p1"]] = 2 * (xh[F["p1"]] - obs)
    lam, st = P.solve_adjoint(pc, torch.as_tensor(g, device="cuda"), rtol=1e-12)
    lo = osolver.adjoint_solve(S, g)
    assert np.linalg.norm(H(lam) - lo) <= 1e-10 * np.linalg.norm(lo)
    g1, g2, gb = P.param_grad(x, lam)
    r1, r2, rb = osolver.param_gradient(S, prob, xh, H(lam))
    assert H(g1).shape == (prob.n_cells,)
    for got, ref in ((H(g1), r1), (H(g2), r2)):
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    assert H(gb)[0] == pytest.approx(rb, rel=1e-10)


def test_q1_p1_only_calls_are_refused():
    dpp = lib()
    prob = I.mms_problem(3, 3, elem="q1")
    with pytest.raises(dpp.DppError) as e:
        dpp.assemble_batch([prob, prob])
    assert e.value.status == 7
