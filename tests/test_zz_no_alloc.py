"""The allocation-free entry point dpp_mms_l2_errors_noalloc against
dpp_mms_l2_errors, through the C ABI: two calls in a row on one GPU, the
second on a smaller box (the fixed scratch keeps the first call's contents),
in 3D and 2D and at the largest quadrature order; out-of-range orders are
argument errors."""
import ctypes as C

import numpy as np
import pytest

import dpp_inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(dpp, prob):
    P = dpp.assemble_problem(prob)
    x, st = P.solve(P.setup_precond(), rtol=1e-10)
    assert st.converged == 1
    return P, x


def _errors(L, name, P, x, mms, q):
    m = (C.c_double * 4)(*[float(v) for v in mms])
    e = (C.c_double * 4)()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = getattr(L, name)(P.handle, C.c_void_p(x.data_ptr()), m, int(q), e, s)
    return st, np.array(e[:])


def _lib():
    import paper_1808_08328_amd as dpp
    L = dpp.lib()
    f = L.dpp_mms_l2_errors_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int,
                  C.POINTER(C.c_double), C.c_void_p]
    return dpp, L


# 48^3 and 600^2 have more simplices than the 2048 workgroups of 256 threads
# cover, so the grid-stride loop takes several per thread there
@pytest.mark.parametrize("dim,sizes,q", [(3, (48, 6), 4), (2, (600, 10), 3), (3, (12, 3), 16)])
def test_noalloc_matches_allocating_entry_point(dim, sizes, q):
    dpp, L = _lib()
    mms = (1.0, 0.1, 1.0, 1.0)
    for n in sizes:  # the second call is on a smaller box
        print("noalloc case dim %d n %d q %d" % (dim, n, q), flush=True)
        P, x = _solve(dpp, I.mms_problem(dim, n, k1=mms[0], k2=mms[1], beta=mms[2], mu=mms[3]))
        st0, ref = _errors(L, "dpp_mms_l2_errors", P, x, mms, q)
        st1, got = _errors(L, "dpp_mms_l2_errors_noalloc", P, x, mms, q)
        assert st0 == 0 and st1 == 0
        assert np.all(ref > 0)
        # the same integral, partial sums grouped differently
        assert np.abs(got - ref).max() <= 1e-12 * ref.max(), (got, ref)


def test_noalloc_rejects_orders_beyond_the_scratch():
    dpp, L = _lib()
    P, x = _solve(dpp, I.mms_problem(2, 4))
    for q in (0, 17):
        st, _ = _errors(L, "dpp_mms_l2_errors_noalloc", P, x, (1.0, 0.1, 1.0, 1.0), q)
        assert st == 1
