"""GPU checks of the tolerance contract's remaining configurations and of the
library's handle and argument behaviour, through the C ABI:

- plain FP64 solves at rtol 1e-12 against the oracle's own flexible GMRES at
  1e-12, per field at 1e-10, on a 32^3 log-normal box and on the full 64^3
  manufactured-solution workload;
- the torch.autograd.Function around the forward and adjoint solves, against
  dpp_param_grad bit for bit and against central differences;
- a rejected solve leaves the preconditioner handle usable and unchanged;
- the adjoint solve reuses its scratch vector (two calls agree bit for bit);
- negative per-cell beta and an uncoupled pure-flux box are refused.
"""
import ctypes as C

import numpy as np
import pytest

import dpp_inputs as I
from oracle import dpp as odpp
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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["c3_3d32_grf", "c2_3d64"])
def test_fp64_fields_vs_oracle_fgmres(name):
    """Both sides at rtol 1e-12 (true residual): each field of the GPU solution
    within 1e-10 of the oracle's.  The oracle is its own FP64 assembly,
    fieldsplit and flexible GMRES (its OpenMP CSR product as the operator)."""
    print("fp64 fields vs oracle", name, flush=True)
    prob = I.grf_problem(3, 32) if name == "c3_3d32_grf" else I.make_config(name)
    P = lib().assemble_problem(prob)
    pc = P.setup_precond()
    x, st = P.solve(pc, rtol=1e-12, maxiter=400)
    assert st.converged == 1 and st.rel_residual <= 1e-12
    xg = H(x)
    del pc, P
    torch.cuda.empty_cache()
    S = odpp.assemble(prob)
    F = osolver.FieldSplit(S)
    xo, its, res = osolver.fgmres(S.K, S.f, F.apply, 30, 1e-12, 400,
                                  matvec=lambda v: odpp.spmv(S.K, v))
    assert res <= 1e-12
    assert np.linalg.norm(S.f - odpp.spmv(S.K, xg)) <= 1.05e-12 * np.linalg.norm(S.f)
    fs = odpp.fields(3, S.N)
    for f in ("u1", "p1", "u2", "p2"):
        e = np.linalg.norm(xg[fs[f]] - xo[fs[f]]) / np.linalg.norm(xo[fs[f]])
        print("  %s %.2e" % (f, e), flush=True)
        assert e <= 1e-10, f


def test_autograd_function_matches_param_grad_and_finite_differences():
    """DppSolve (forward: assemble + setup + solve; backward: adjoint solve +
    parameter gradient) on a 3D n = 8 log-normal box with
    J = ||p1 - p_obs||^2: torch.autograd.backward gives dpp_param_grad's
    values bit for bit, and central differences on three directions."""
    dpp = lib()
    base = I.grf_problem(3, 8)
    F = odpp.fields(3, base.n_nodes)
    spec = dict(dim=3, n=base.n, p0_1=T(base.p0_1), p0_2=T(base.p0_2), mu=base.mu)
    opts = dict(rtol=1e-12, coarse_max=40)
    p_obs = T(I.random_vector(base.n_nodes, 51))

    lk1 = T(np.log(base.k1)).requires_grad_(True)
    lk2 = T(np.log(base.k2)).requires_grad_(True)
    beta = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    x = dpp.DppSolve.apply(lk1, lk2, beta, spec, opts)
    J = ((x[F["p1"]] - p_obs) ** 2).sum()
    torch.autograd.backward(J)

    # the same through the C ABI directly
    k1, k2 = torch.exp(lk1.detach()), torch.exp(lk2.detach())
    P = dpp.assemble(3, base.n, k1, k2, spec["p0_1"], spec["p0_2"], beta=1.0, mu=base.mu)
    pc = P.setup_precond(coarse_max=40)
    x2, _ = P.solve(pc, rtol=1e-12)
    assert torch.equal(x2, x.detach())
    g = torch.zeros_like(x2)
    g[F["p1"]] = 2.0 * (x2[F["p1"]] - p_obs)
    lam, _ = P.solve_adjoint(pc, g, rtol=1e-12)
    g1, g2, gb = P.param_grad(x2, lam)
    assert torch.equal(lk1.grad, g1) and torch.equal(lk2.grad, g2)
    assert beta.grad.shape == beta.shape and torch.equal(beta.grad, gb.reshape(()))

    def Jof(a1, a2, b):
        with torch.no_grad():
            xx = dpp.DppSolve.apply(a1, a2, torch.tensor(b, dtype=torch.float64, device="cuda"),
                                    spec, opts)
            return float(((xx[F["p1"]] - p_obs) ** 2).sum())

    th1, th2 = lk1.detach(), lk2.detach()
    # step 1e-3 ||theta||_inf (the directions have unit norm): small enough for
    # the O(eps^2) truncation, large enough for the rtol 1e-12 solves
    eps = 1e-3 * float(max(th1.abs().max(), th2.abs().max()))
    fds, ads = [], []
    for j, d in enumerate(I.random_directions(3, base.n_cells, seed0=4100)):
        dt = T(d)
        a1, a2 = (dt, 0 * dt) if j != 1 else (0 * dt, dt)
        fd = (Jof(th1 + eps * a1, th2 + eps * a2, 1.0) - Jof(th1 - eps * a1, th2 - eps * a2, 1.0)) / (2 * eps)
        ad = float((lk1.grad * a1).sum() + (lk2.grad * a2).sum())
        fds.append(fd)
        ads.append(ad)
        print("direction %d: autograd %.10e fd %.10e" % (j, ad, fd), flush=True)
    scale = max(abs(v) for v in fds)
    assert max(abs(a - f) for a, f in zip(ads, fds)) <= 1e-6 * scale
    hb = 1e-3
    fdb = (4 * (Jof(th1, th2, 1 + hb) - Jof(th1, th2, 1 - hb)) / (2 * hb)
           - (Jof(th1, th2, 1 + 2 * hb) - Jof(th1, th2, 1 - 2 * hb)) / (4 * hb)) / 3
    print("beta: autograd %.10e fd %.10e" % (float(beta.grad), fdb), flush=True)
    assert abs(float(beta.grad) - fdb) <= 1e-6 * abs(fdb)


def test_autograd_function_rejects_what_it_does_not_differentiate():
    dpp = lib()
    base = I.mms_problem(3, 2)
    spec = dict(dim=3, n=base.n, p0_1=T(base.p0_1), p0_2=T(base.p0_2))
    lk = T(np.zeros(base.n_cells))
    with pytest.raises(ValueError):
        dpp.DppSolve.apply(lk, lk, torch.ones(2, dtype=torch.float64, device="cuda"), spec, None)
    with pytest.raises(ValueError):
        dpp.DppSolve.apply(lk, lk, torch.tensor(1.0, dtype=torch.float64, device="cuda"),
                           {**spec, "body": T(np.ones(3 * base.n_cells))}, None)


def test_rejected_solve_leaves_the_preconditioner_unchanged():
    """A solve refused for its smoothing degrees must not change the handle:
    the fieldsplit apply gives the same z afterwards, and a solve with the
    handle's own options (NULL opts through the C ABI) still converges."""
    dpp = lib()
    prob = I.mms_problem(3, 6, k2=1e-2)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    r = T(I.random_vector(P.n_dof, 3))
    z0 = pc.apply(r)
    x0, s0 = P.solve(pc)
    for bad in (dict(cheb_post_fine=0), dict(cheb_degree=0), dict(cheb_post_coarse=9),
                dict(cheb_pre_fine=-2)):
        with pytest.raises(dpp.DppError) as e:
            P.solve(pc, **bad)
        assert e.value.status == 1, bad
        assert torch.equal(pc.apply(r), z0), bad
    L = dpp.lib()
    x = torch.zeros(P.n_dof, dtype=torch.float64, device="cuda")
    st = dpp.SolveStats()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.dpp_solve(P.handle, pc.handle, None, None, C.c_void_p(x.data_ptr()), C.byref(st), s) == 0
    assert st.converged == 1 and st.iters == s0.iters
    assert torch.equal(x, x0)


def test_adjoint_solves_repeat_bit_for_bit():
    """The adjoint's D g vector is kept on the preconditioner: two adjoint
    solves with different g in a row, then the first again."""
    dpp = lib()
    prob = I.grf_problem(3, 5)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    g1 = T(I.random_vector(P.n_dof, 61))
    g2 = T(I.random_vector(P.n_dof, 62))
    l1, _ = P.solve_adjoint(pc, g1, rtol=1e-12)
    l2, _ = P.solve_adjoint(pc, g2, rtol=1e-12)
    l1b, _ = P.solve_adjoint(pc, g1, rtol=1e-12)
    assert torch.equal(l1, l1b) and not torch.equal(l1, l2)
    S = odpp.assemble(prob)
    lo = osolver.adjoint_solve(S, H(g2))
    assert np.linalg.norm(H(l2) - lo) <= 1e-10 * np.linalg.norm(lo)


def test_coefficient_checks():
    dpp = lib()
    prob = I.mms_problem(2, 4)
    with pytest.raises(dpp.DppError) as e:
        bc = np.ones(prob.n_cells)
        bc[5] = -0.5
        dpp.assemble(2, prob.n, T(prob.k1), T(prob.k2), T(prob.p0_1), T(prob.p0_2),
                     beta_cells=T(bc))
    assert e.value.status == 5
    pure = I.mms_problem(2, 4, flux_faces=[[1] * 4, [1] * 4])
    pure.beta = 0.0
    with pytest.raises(dpp.DppError) as e:
        dpp.assemble_problem(pure)
    assert e.value.status == 7
    pure.beta = np.zeros(pure.n_cells)
    with pytest.raises(dpp.DppError) as e:
        dpp.assemble_problem(pure)
    assert e.value.status == 7
    pure.beta = np.where(np.arange(pure.n_cells) % 2 == 0, 0.7, 0.0)
    P = dpp.assemble_problem(pure)  # coupled in half of the cells: accepted
    x, st = P.solve(P.setup_precond(), rtol=1e-10)
    assert st.converged == 1
