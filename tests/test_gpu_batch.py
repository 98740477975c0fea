"""GPU parity of the batched multi-instance solve against the oracle and the
single-instance path (bars as in test_gpu_parity)."""
import numpy as np
import pytest

import dpp_inputs as I
from oracle import dpp as odpp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def uneven_2d(count=8, seed=77):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(rng.integers(4, 41))
        # eta = sqrt(beta (k1 + k2) / (k1 k2)) stays below about 10, so the
        # manufactured solution's exp(eta y) layer stays representable
        beta = float(10 ** rng.uniform(-1, 0.5))
        ratio = float(10 ** rng.uniform(-1.5, 0))
        out.append(I.mms_problem(2, n if i % 3 else (n, n // 2 + 3), k1=1.0, k2=ratio, beta=beta))
    return out


@pytest.mark.parametrize("cycle", [None, (2, 2, 1, 2)])
def test_batch_operator_and_preconditioner_match_single_path(cycle):
    import paper_1808_08328_amd as dpp
    probs = uneven_2d()
    names = ("cheb_pre_fine", "cheb_post_fine", "cheb_pre_coarse", "cheb_post_coarse")
    kw = dict(zip(names, cycle)) if cycle else {}
    B = dpp.assemble_batch(probs, coarse_max=30, **kw)
    x = torch.as_tensor(I.random_vector(B.n_dof, 3), device="cuda")
    yb = [H(v) for v in B.split(B.spmv(x))]
    zb = [H(v) for v in B.split(B.precond_apply(x))]
    xs = B.split(x)
    for i, pr in enumerate(probs):
        P = dpp.assemble_problem(pr)
        pc = P.setup_precond(coarse_max=30, **kw)
        ys = H(P.spmv(xs[i].contiguous()))
        assert np.abs(yb[i] - ys).max() <= 1e-13 * np.abs(ys).max(), ("spmv", i)
        zs = H(pc.apply(xs[i].contiguous()))
        assert np.abs(zb[i] - zs).max() <= 1e-11 * np.abs(zs).max(), ("precond", i)


def test_batch_matches_oracle_and_single_solves():
    import paper_1808_08328_amd as dpp
    probs = uneven_2d()
    print("batch sizes", [p.n for p in probs], flush=True)
    B = dpp.assemble_batch(probs, coarse_max=30)
    assert len(B.lanes()) >= 2
    x, st = B.solve(rtol=1e-12)
    assert all(s.converged for s in st)
    xs = [H(v) for v in B.split(x)]
    for i, pr in enumerate(probs):
        S = odpp.assemble(pr)
        xo = odpp.solve_direct(S.K, S.f)
        F = odpp.fields(2, S.N)
        for f in ("u1", "p1", "u2", "p2"):
            assert np.linalg.norm(xs[i][F[f]] - xo[F[f]]) <= 1e-10 * np.linalg.norm(xo[F[f]]), (i, f)
        # same preconditioner definition as the single-instance path: same iteration count
        P = dpp.assemble_problem(pr)
        pc = P.setup_precond(coarse_max=30)
        _, s1 = P.solve(pc, rtol=1e-12)
        assert abs(s1.iters - st[i].iters) <= 1, (i, s1.iters, st[i].iters)


def test_batch_graph_replay_is_bit_identical():
    import paper_1808_08328_amd as dpp
    probs = uneven_2d(6, seed=5)
    B = dpp.assemble_batch(probs, coarse_max=30)
    x1, s1 = B.solve(rtol=1e-10)
    x2, s2 = B.solve(rtol=1e-10, use_graph=1)
    x3, s3 = B.solve(rtol=1e-10, use_graph=1)  # replays the cached graphs
    assert torch.equal(x1, x2) and torch.equal(x2, x3)
    assert [s.iters for s in s1] == [s.iters for s in s2] == [s.iters for s in s3]


@pytest.mark.parametrize("cycle", [None, (2, 2, 1, 2)])
def test_batch_fp32_preconditioner_and_3d(cycle):
    import paper_1808_08328_amd as dpp
    probs = [I.grf_problem(3, 5), I.mms_problem(3, (6, 4, 5), k2=1e-2), I.grf_problem(3, 7)]
    names = ("cheb_pre_fine", "cheb_post_fine", "cheb_pre_coarse", "cheb_post_coarse")
    B = dpp.assemble_batch(probs, coarse_max=40, **(dict(zip(names, cycle)) if cycle else {}))
    for precision in (0, 1, 2):
        x, st = B.solve(rtol=1e-10, precision=precision)
        assert all(s.converged for s in st)
        for i, pr in enumerate(probs):
            S = odpp.assemble(pr)
            xo = odpp.solve_direct(S.K, S.f)
            xi = H(B.split(x)[i])
            assert np.linalg.norm(xi - xo) <= 1e-7 * np.linalg.norm(xo), (precision, i)


def test_batch_masks_converged_instances_and_reports_unconverged():
    import paper_1808_08328_amd as dpp
    probs = [I.mms_problem(2, 4), I.mms_problem(2, 30, k2=1e-3)]
    B = dpp.assemble_batch(probs, coarse_max=30)
    with pytest.raises(dpp.DppError) as e:
        B.solve(rtol=1e-10, maxiter=3)
    assert e.value.status == 4
    x, st = B.solve(rtol=1e-10, maxiter=3, allow_unconverged=True)
    assert st[1].converged == 0 and st[1].iters == 3


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_velocity_faces_match_single_path_and_oracle(dim):
    """Instances with and without velocity faces in one batch: masked products
    and preconditioner as in the single-instance path, solutions as the
    oracle's."""
    import paper_1808_08328_amd as dpp
    if dim == 2:
        probs = [I.mms_problem(2, 9, k2=0.3, flux_faces=[[1, 1, 0, 0], [0, 0, 1, 0]]),
                 I.mms_problem(2, (12, 7), k2=0.1),
                 I.mms_problem(2, 10, k2=0.2, beta=2.0, flux_faces=[[0, 0, 0, 1], [1, 0, 0, 0]]),
                 I.mms_problem(2, 8, k2=0.1, flux_faces=[[1, 1, 1, 1], [0, 0, 0, 0]])]
    else:
        probs = [I.mms_problem(3, (4, 3, 4), k2=0.1, flux_faces=[[1, 0, 0, 0, 0, 1], [0, 0, 1, 1, 0, 0]]),
                 I.mms_problem(3, 5, k2=0.1),
                 I.mms_problem(3, (3, 5, 4), k2=0.05, flux_faces=[[0, 1, 1, 0, 0, 0], [1, 1, 0, 0, 0, 0]])]
    B = dpp.assemble_batch(probs, coarse_max=30)
    x = torch.as_tensor(I.random_vector(B.n_dof, 3), device="cuda")
    yb = [H(v) for v in B.split(B.spmv(x))]
    zb = [H(v) for v in B.split(B.precond_apply(x))]
    xs = B.split(x)
    for i, pr in enumerate(probs):
        P = dpp.assemble_problem(pr)
        pc = P.setup_precond(coarse_max=30)
        ys = H(P.spmv(xs[i].contiguous()))
        assert np.abs(yb[i] - ys).max() <= 1e-13 * np.abs(ys).max(), ("spmv", i)
        zs = H(pc.apply(xs[i].contiguous()))
        assert np.abs(zb[i] - zs).max() <= 1e-11 * np.abs(zs).max(), ("precond", i)
    xsol, st = B.solve(rtol=1e-13)
    assert all(s.converged for s in st)
    for i, pr in enumerate(probs):
        S = odpp.assemble(pr)
        xo = odpp.solve_direct(S.K, S.f)
        xi = H(B.split(xsol)[i])
        F = odpp.fields(dim, S.N)
        for f in ("u1", "p1", "u2", "p2"):
            assert np.linalg.norm(xi[F[f]] - xo[F[f]]) <= 1e-10 * np.linalg.norm(xo[F[f]]), (i, f)


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_pure_flux_instances_match_oracle(dim):
    """Pure-flux instances (velocity faces everywhere, singular K) in a batch
    with regular ones: each takes the consistent part of its f and returns
    int p1 = 0, as the oracle's bordered solve; FP64 and FP32 preconditioner."""
    import paper_1808_08328_amd as dpp
    full = [[1] * (2 * dim), [1] * (2 * dim)]
    if dim == 2:
        probs = [I.mms_problem(2, 8, k2=0.1, flux_faces=full),
                 I.mms_problem(2, (9, 6), k2=0.2, beta=2.0),
                 I.mms_problem(2, (7, 10), k2=0.3, beta=0.5, mu=1.3, flux_faces=full)]
    else:
        probs = [I.mms_problem(3, (4, 3, 5), k2=0.1, mu=0.8, flux_faces=full),
                 I.mms_problem(3, 4, k2=0.1)]
    B = dpp.assemble_batch(probs, coarse_max=30)
    refs = []
    for pr in probs:
        S = odpp.assemble(pr)
        refs.append((S, odpp.solve_pure_flux(S) if odpp.pure_flux(pr) else odpp.solve_direct(S.K, S.f)))
    for precision, tol in ((0, 1e-9), (1, 1e-9), (2, 1e-9)):
        xsol, st = B.solve(rtol=1e-13, precision=precision)
        assert all(s.converged for s in st), precision
        for i, (S, xo) in enumerate(refs):
            xi = H(B.split(xsol)[i])
            F = odpp.fields(dim, S.N)
            if odpp.pure_flux(probs[i]):
                assert abs(odpp.pressure_mean(S.mesh, xi[F["p1"]])) <= 1e-12 * np.abs(xi[F["p1"]]).max()
            for f in ("u1", "p1", "u2", "p2"):
                assert np.linalg.norm(xi[F[f]] - xo[F[f]]) <= tol * np.linalg.norm(xo[F[f]]), (precision, i, f)


def test_full_size_batch_oracle_residuals():
    """The benchmark's batch at full size (64 uneven 2D instances, 32^2..256^2
    cells, 9,131,268 DOF) in the benchmark's launch configuration (hipGraph
    replay of the Arnoldi steps; FP64, iterative refinement with FP32 inner
    solves, and the FP32 preconditioner): every
    instance's solution against the oracle's own K and f of that instance, and
    the batched K product against the oracle's K on a random vector."""
    import paper_1808_08328_amd as dpp
    print("full-size batch c4_batch64", flush=True)
    probs = I.batch_configs(64, seed=2024)
    B = dpp.assemble_batch(probs)
    assert B.n_dof == 9131268
    x = torch.as_tensor(I.random_vector(B.n_dof, 21), device="cuda")
    yb = [H(v) for v in B.split(B.spmv(x))]
    xs = [H(v) for v in B.split(x)]
    sols = {}
    for precision in (0, 1, 2):
        xsol, st = B.solve(rtol=1e-8, precision=precision, use_graph=1)
        assert all(s.converged for s in st), precision
        sols[precision] = [H(v) for v in B.split(xsol)]
    for i, pr in enumerate(probs):
        S = odpp.assemble(pr)
        ref = S.K @ xs[i]
        assert np.abs(yb[i] - ref).max() <= 1e-13 * np.abs(ref).max(), ("spmv", i)
        fn = np.linalg.norm(S.f)
        for precision in (0, 1, 2):
            r = S.f - S.K @ sols[precision][i]
            assert np.linalg.norm(r) <= 1.05e-8 * fn, (precision, i, np.linalg.norm(r) / fn)
