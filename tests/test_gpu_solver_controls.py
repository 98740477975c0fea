"""GPU checks of the solver controls through the C ABI: the stagnation stop
(forced from the host with a stagnation ratio no cycle can meet, so every
kernel runs and exits normally), fixed kernel schedules, the inner iteration
limit of mixed precision and the setup time in the statistics."""
import numpy as np
import pytest

import dpp_inputs as I
from oracle import dpp as odpp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_forced_stagnation_stops_with_the_last_iterate(precision):
    """With stag_ratio tiny every finished cycle counts as stalled: the solve
    stops after stag_cycles cycles with DPP_ERR_STAGNATED, x holds the last
    iterate (the residual the statistics report) and the default settings
    solve the same system."""
    import paper_1808_08328_amd as dpp
    prob = I.grf_problem(3, 6)
    print("stagnation case 3D n=6 precision", precision, flush=True)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    opts = dict(rtol=1e-12, restart=2, precision=precision, stag_cycles=2, stag_ratio=1e-300,
                inner_rtol=0.5)
    with pytest.raises(dpp.DppError) as e:
        P.solve(pc, **opts)
    assert e.value.status == 8
    x, st = P.solve(pc, allow_unconverged=True, **opts)
    assert st.converged == 0
    if precision == 1:
        assert st.refinements == 2
    else:
        assert st.restarts == 2 and st.iters == 4
    S = odpp.assemble(prob)
    xh = H(x)
    rel = np.linalg.norm(S.f - S.K @ xh) / np.linalg.norm(S.f)
    assert 1e-12 < rel < 1.0 and abs(rel - st.rel_residual) <= 1e-6 * rel
    # the same system without the forced test (an inner tolerance of 0.5 would
    # only halve the residual per refinement sweep: the default one here)
    x2, st2 = P.solve(pc, rtol=1e-10, restart=2, precision=precision)
    assert st2.converged == 1


def test_forced_stagnation_in_a_batch():
    import paper_1808_08328_amd as dpp
    probs = [I.mms_problem(2, 12, k2=0.1), I.mms_problem(2, (9, 14), k2=0.2)]
    B = dpp.assemble_batch(probs, coarse_max=30)
    for precision in (0, 1):
        opts = dict(rtol=1e-12, restart=2, precision=precision, stag_cycles=1, stag_ratio=1e-300,
                    inner_rtol=0.5)
        with pytest.raises(dpp.DppError) as e:
            B.solve(**opts)
        assert e.value.status == 8, precision
        x, st = B.solve(allow_unconverged=True, **opts)
        assert not any(s.converged for s in st)
        x, st = B.solve(rtol=1e-10, restart=2, precision=precision)
        assert all(s.converged for s in st), precision


@pytest.mark.parametrize("schedule", [0, 5, 9])
def test_fixed_schedule_on_every_level(schedule):
    import paper_1808_08328_amd as dpp
    prob = I.grf_problem(3, 12)
    P = dpp.assemble_problem(prob)
    pa = P.setup_precond(coarse_max=40)
    pf = P.setup_precond(coarse_max=40, schedule=schedule)
    lanes = [0, 1, 2, 4, 8][schedule % 5]
    for lvl in range(pf.info()["levels"] - 1):
        assert pf.shape(lvl) == (lanes, 1 if schedule >= 5 else 0)
    r = torch.as_tensor(I.random_vector(P.n_dof, 9), device="cuda")
    za, zf = H(pa.apply(r)), H(pf.apply(r))
    assert np.abs(za - zf).max() <= 1e-11 * np.abs(za).max()
    x, st = P.solve(pf, rtol=1e-10)
    assert st.converged == 1 and st.ms_setup > 0.0
    with pytest.raises(dpp.DppError):
        P.setup_precond(schedule=10)


def test_inner_iteration_limit_of_mixed_precision():
    import paper_1808_08328_amd as dpp
    prob = I.grf_problem(3, 10)
    P = dpp.assemble_problem(prob)
    pc = P.setup_precond(coarse_max=40)
    _, s_free = P.solve(pc, rtol=1e-10, precision=1)
    _, s_lim = P.solve(pc, rtol=1e-10, precision=1, inner_maxiter=2)
    assert s_free.converged == s_lim.converged == 1
    # at most two inner iterations per sweep
    assert s_lim.iters <= 2 * s_lim.refinements and s_lim.refinements > s_free.refinements
