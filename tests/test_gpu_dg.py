"""GPU parity of the DG-VMS path (discontinuous P1 on the Kuhn simplices)
against the oracle (`oracle/dg.py`), through the C ABI: the right-hand side,
every entry of K, and the K product, at 1e-13."""
import numpy as np
import pytest
import scipy.sparse as sp

import dpp_inputs as I
from oracle import dg as odg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def random_problem(dim, n, seed, beta_cells=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    prob = I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.3, elem="dg")
    nc = prob.n_cells
    prob.k1 = 10 ** rng.uniform(-1, 1, nc)
    prob.k2 = 10 ** rng.uniform(-2, 0, nc)
    if beta_cells:
        prob.beta = 10 ** rng.uniform(-1, 0.5, nc)
    prob.body = rng.normal(size=(nc, dim))
    return prob


CASES = {
    "2d_ragged": (2, (5, 3), False),
    "2d_thin": (2, (1, 4), True),
    "3d_ragged": (3, (3, 2, 4), True),
    "3d_cube": (3, 3, False),
    "3d_thin": (3, (1, 2, 1), False),
    "2d_single_box": (2, (1, 1), True),
    "3d_single_box": (3, (1, 1, 1), True),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_dg_assembly_and_product_match_oracle(case):
    import paper_1808_08328_amd as dpp
    dim, n, bc = CASES[case]
    print("dg case", case, flush=True)
    prob = random_problem(dim, n, 7, bc)
    S = odg.assemble(prob)
    P = dpp.assemble_problem(prob)
    assert P.n_dof == S.K.shape[0] == prob.n_dof
    assert P.n_nodes == S.S
    f = H(P.rhs())
    assert np.abs(f - S.f).max() <= 1e-13 * np.abs(S.f).max()
    rowptr, cols, vals = P.export_csr()
    Kg = sp.csr_matrix((H(vals), H(cols), H(rowptr)), shape=S.K.shape)
    scale = np.abs(S.K).max()
    assert abs(Kg - S.K).max() <= 1e-13 * scale
    x = I.random_vector(P.n_dof, 3)
    y = H(P.spmv(torch.as_tensor(x, device="cuda")))
    ref = S.K @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_dg_refuses_what_it_does_not_implement():
    import paper_1808_08328_amd as dpp
    prob = random_problem(2, 4, 1)
    P = dpp.assemble_problem(prob)
    x = torch.zeros(P.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(dpp.DppError) as e:
        P.spmv(x, which=1)
    assert e.value.status == 7


PC_CASES = {"2d_ragged": (2, (9, 6), 30), "3d_ragged": (3, (4, 3, 5), 20), "3d_cube": (3, 4, 40),
            "2d_default_coarse": (2, (50, 45), 0)}


@pytest.mark.parametrize("case", sorted(PC_CASES))
def test_dg_fieldsplit_matches_oracle(case):
    """The DG fieldsplit apply (block-Jacobi Chebyshev velocity solve,
    two-level pressure blocks over the nodal CG-VMS hierarchy, Chebyshev on
    S_q) against the oracle's definition, at the cycles' 1e-11; coarse_max 0
    takes the default coarsest level of each side (the 2D nodal cycle's own)."""
    import paper_1808_08328_amd as dpp
    from oracle import mg as omg
    dim, n, cmax = PC_CASES[case]
    print("dg precond case", case, flush=True)
    prob = random_problem(dim, n, 13, True)
    S = odg.assemble(prob)
    Fo = odg.FieldSplitDG(S, prob, omg.MGOptions(coarse_max=cmax))
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=cmax)
    r = I.random_vector(P.n_dof, 5)
    z = H(pc.apply(torch.as_tensor(r, device="cuda")))
    zo = Fo.apply(r)
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max()


SOLVE_CASES = {"2d_ragged": (2, (12, 7)), "2d_mms": (2, 16), "3d_ragged": (3, (4, 3, 5)), "3d_mms": (3, 4),
               "3d_ragged_single_box": (3, (1, 1, 1))}


@pytest.mark.parametrize("case", sorted(SOLVE_CASES))
def test_dg_fp64_solve_matches_oracle_direct_solve(case):
    import paper_1808_08328_amd as dpp
    from oracle import dpp as odpp
    dim, n = SOLVE_CASES[case]
    print("dg solve case", case, flush=True)
    prob = (random_problem(dim, n, 17, True) if "ragged" in case
            else I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.0, elem="dg"))
    S = odg.assemble(prob)
    xo = odpp.solve_direct(S.K, S.f)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    x, st = P.solve(pc, rtol=1e-12)
    assert st.converged == 1
    xg = H(x)
    F = odg.fields(dim, S.S)
    for f in ("u1", "p1", "u2", "p2"):
        err = np.linalg.norm(xg[F[f]] - xo[F[f]]) / np.linalg.norm(xo[F[f]])
        assert err <= 1e-10, (f, err, st.iters)
    print("iterations", st.iters, flush=True)


def test_dg_refuses_iterative_refinement():
    import paper_1808_08328_amd as dpp
    P = dpp.assemble_problem(random_problem(2, 6, 2))
    pc = P.setup_precond(coarse_max=30)
    with pytest.raises(dpp.DppError) as e:
        P.solve(pc, precision=1)
    assert e.value.status == 7


@pytest.mark.parametrize("case", sorted(SOLVE_CASES))
def test_dg_fp32_preconditioner_solve_matches_oracle(case):
    """precision 2: FP64 flexible GMRES around the fieldsplit run in FP32
    (block inverses, diagonals and work vectors rounded once, the nodal cycle
    on its FP32 levels); solved to 1e-10, every field within 1e-7 of the
    oracle's direct solution, in about as many iterations as in FP64."""
    import paper_1808_08328_amd as dpp
    from oracle import dpp as odpp
    dim, n = SOLVE_CASES[case]
    print("dg fp32-preconditioner case", case, flush=True)
    prob = (random_problem(dim, n, 17, True) if "ragged" in case
            else I.mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.0, elem="dg"))
    S = odg.assemble(prob)
    xo = odpp.solve_direct(S.K, S.f)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    x64, st64 = P.solve(pc, rtol=1e-10)
    x, st = P.solve(pc, rtol=1e-10, precision=2)
    assert st.converged == 1 and st.iters <= st64.iters + 3, (st.iters, st64.iters)
    xg = H(x)
    F = odg.fields(dim, S.S)
    for f in ("u1", "p1", "u2", "p2"):
        err = np.linalg.norm(xg[F[f]] - xo[F[f]]) / np.linalg.norm(xo[F[f]])
        assert err <= 1e-7, (f, err)
    # the FP64 path is unchanged by the FP32 copies
    x64b, _ = P.solve(pc, rtol=1e-10)
    assert np.array_equal(H(x64b), H(x64))


@pytest.mark.parametrize("precision", [0, 2])
def test_dg_graph_replay_matches_eager_solve(precision):
    """Arnoldi steps replayed from captured hipGraphs (the DG fieldsplit and the
    nodal cycle inside them) give the eager solve bit for bit, with eager work
    between the replays."""
    import paper_1808_08328_amd as dpp
    P = dpp.assemble_problem(random_problem(3, (3, 4, 2), 31, True))
    pc = P.setup_precond(coarse_max=40)
    xe, se = P.solve(pc, rtol=1e-10, precision=precision)
    for rep in range(2):
        xg, sg = P.solve(pc, rtol=1e-10, precision=precision, use_graph=1)
        assert torch.equal(xg, xe) and sg.iters == se.iters, rep
        y = P.spmv(xg)
        torch.cuda.synchronize()
        del y


@pytest.mark.parametrize("case", ["2d_ragged", "3d_ragged"])
def test_dg_adjoint_matches_oracle(case):
    """K^T lambda = g through D K D on the DG blocks, against the oracle's
    sparse LU of K^T, for g = 2 (p1 - p_obs) (a least-squares misfit)."""
    import paper_1808_08328_amd as dpp
    from oracle import solver as osolver
    dim, n = SOLVE_CASES[case]
    print("dg adjoint case", case, flush=True)
    prob = random_problem(dim, n, 23, True)
    S = odg.assemble(prob)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    x, st = P.solve(pc, rtol=1e-12)
    assert st.converged == 1
    F = odg.fields(dim, S.S)
    xh = H(x)
    g = np.zeros(P.n_dof)
    g[F["p1"]] = 2 * (xh[F["p1"]] - I.random_vector(S.S, 29))
    lam, st = P.solve_adjoint(pc, torch.as_tensor(g, device="cuda"), rtol=1e-12)
    assert st.converged == 1
    lo = osolver.adjoint_solve(S, g)
    assert np.linalg.norm(H(lam) - lo) <= 1e-10 * np.linalg.norm(lo)
    with pytest.raises(dpp.DppError) as e:
        P.param_grad(x, lam)
    assert e.value.status == 7


@pytest.mark.timeout(400)
@pytest.mark.parametrize("workload", ["g1_2d160_dg", "g2_3d20_dg"])
def test_dg_full_size_solve_oracle_residual(workload):
    """The largest DG rows of the h-size study (921,600 and 1,536,000 DOF) in
    the benchmark's launch configuration: the oracle's own FP64 K applied to
    the GPU solution at 1e-8, and 2000 sampled rows of K against the oracle's."""
    import time

    import paper_1808_08328_amd as dpp
    from oracle import dpp as odpp
    t0 = time.time()

    def step(msg):
        print("full-size DG %s: %s (%.1f s)" % (workload, msg, time.time() - t0), flush=True)

    step("start")
    prob = I.make_config(workload)
    P = dpp.assemble_problem(prob)
    step("assembled")
    pc = P.setup_precond()
    step("preconditioner set up")
    x, st = P.solve(pc)
    step("solved in %d iterations" % st.iters)
    assert st.converged == 1
    xg = H(x)
    rows = np.random.default_rng(0).integers(0, P.n_dof, 2000)
    rp, ci, vv = (H(t) for t in P.export_csr())
    del pc, P
    torch.cuda.empty_cache()
    step("exported")
    S = odg.assemble(prob)
    step("oracle assembled")
    r = S.f - odpp.spmv(S.K, xg)
    rel = np.linalg.norm(r) / np.linalg.norm(S.f)
    step("oracle residual %.3e" % rel)
    assert rel <= 1.05e-8
    # the export lists every entry of the coupled blocks, the oracle only the
    # entries its assembly touched: compare row values, absent = 0
    scale = np.abs(S.K.data).max()
    for rr in rows:
        a, b = rp[rr], rp[rr + 1]
        lo, hi = S.K.indptr[rr], S.K.indptr[rr + 1]
        g = dict(zip(ci[a:b].tolist(), vv[a:b].tolist()))
        assert len(g) == b - a
        o = dict(zip(S.K.indices[lo:hi].tolist(), S.K.data[lo:hi].tolist()))
        assert set(o) <= set(g), rr
        assert max(abs(g[c] - o.get(c, 0.0)) for c in g) <= 1e-13 * scale, rr


@pytest.mark.parametrize("dim,n", [(2, (9, 6)), (3, (3, 4, 2))])
def test_dg_l2_errors_match_oracle(dim, n):
    """dpp_mms_l2_errors on a DG solution (fields on the vertex slots) and on
    the DG interpolant of the exact fields, against the oracle's integral of
    the same rule, at 1e-12."""
    import paper_1808_08328_amd as dpp
    prob = I.mms_problem(dim, n, k1=1.0, k2=0.2, beta=1.0, mu=0.9, elem="dg")
    mms = prob.meta["mms"]
    S = odg.assemble(prob)
    P = dpp.assemble_problem(prob)
    x, st = P.solve(P.setup_precond(coarse_max=40), rtol=1e-10)
    assert st.converged == 1
    field = {"p1": 0, "p2": 1, "u1": 2, "u2": 3}
    exact = {f: (lambda X, i=i: np.asarray(I.mms_fields(dim, X, *mms)[i]).reshape(X.shape[0], -1))
             for f, i in field.items()}
    Fs = odg.fields(dim, S.S)
    X = odg.slot_coords(S.mesh)
    xi = np.zeros(P.n_dof)
    for f, i in field.items():
        xi[Fs[f]] = np.asarray(I.mms_fields(dim, X, *mms)[i]).ravel()
    for xv in (H(x), xi):
        for q in (2, 4):
            eg = P.mms_l2_errors(torch.as_tensor(xv, device="cuda"), mms, q=q)
            eo = odg.l2_errors(S, xv, exact, q=q, relative=False)
            for f in ("u1", "p1", "u2", "p2"):
                assert abs(eg[f] - eo[f]) <= 1e-12 * eo[f], (q, f, eg[f], eo[f])


def test_dg_solve_time_cycle_degrees_reach_the_nodal_cycle():
    """Cycle degrees given to the solve act as if given to the setup: on
    DG-VMS problems they reach the nodal cycle of the pressure solve as well
    as the smoothing on the slots (same iterations, same solution)."""
    import paper_1808_08328_amd as dpp
    prob = random_problem(3, (3, 3, 4), 11)
    P = dpp.assemble_problem(prob)
    o = dict(cheb_post_fine=3, cheb_post_coarse=2)
    xa, sa = P.solve(P.setup_precond(coarse_max=30, **o), rtol=1e-10)
    pc = P.setup_precond(coarse_max=30)
    x0, s0 = P.solve(pc, rtol=1e-10)
    xb, sb = P.solve(pc, rtol=1e-10, **o)
    assert sa.converged and sb.converged and s0.converged
    assert sa.iters == sb.iters
    a, b = H(xa), H(xb)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
    # and the degrees matter: the default cycle takes a different path
    assert s0.iters != sa.iters or np.abs(H(x0) - a).max() > 1e-13 * np.abs(a).max()
