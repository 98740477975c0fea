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
