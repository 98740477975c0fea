"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports
every symbol that include/dpp.h declares; the option defaults are sane."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpp.h")
LIB = os.path.join(ROOT, "paper_1808_08328_amd", "libdpp.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("dpp_assemble", "dpp_setup_precond", "dpp_solve", "dpp_solve_adjoint",
                 "dpp_param_grad", "dpp_spmv", "dpp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    lib = C.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options():
    import paper_1808_08328_amd as dpp
    o = dpp.default_opts()
    assert o.restart == 30 and o.rtol == 1e-8 and o.precision == 0
    assert o.cheb_degree == 2 and o.coarse_max == 0
    assert o.inner_maxiter == 0 and o.schedule == -1
    assert o.stag_cycles == 3 and o.stag_ratio == 0.999
    with pytest.raises(TypeError):
        dpp.default_opts(nonsense=1)


def test_null_arguments_are_rejected_without_a_gpu():
    import paper_1808_08328_amd as dpp
    L = dpp.lib()
    h = C.c_void_p()
    st = L.dpp_assemble(None, None, None, C.byref(h))
    assert st == 1  # DPP_ERR_ARG
    assert b"null" in L.dpp_last_error()
    st = L.dpp_solve(None, None, None, None, None, None, None)
    assert st == 1


def test_oversized_boxes_are_rejected_without_a_gpu():
    """Boxes with 2^31 or more unknowns (the stencil kernels index with 32-bit
    integers) and boxes beyond 4096 cells per axis are argument errors,
    reported before any device work."""
    import paper_1808_08328_amd as dpp
    from paper_1808_08328_amd._binding import _Box, _Params
    L = dpp.lib()
    dummy = (C.c_double * 4)()
    prm = _Params(mu=1.0, k1=C.cast(dummy, C.c_void_p), k2=C.cast(dummy, C.c_void_p), beta=1.0,
                  p0_1=C.cast(dummy, C.c_void_p), p0_2=C.cast(dummy, C.c_void_p))
    h = C.c_void_p()
    for n, msg in (((1024, 1024, 1024), b"2^31"), ((4097, 2, 2), b"4096")):
        box = _Box(dim=3, n=(C.c_int * 3)(*n), L=(C.c_double * 3)(1.0, 1.0, 1.0))
        st = L.dpp_assemble(C.byref(box), C.byref(prm), None, C.byref(h))
        assert st == 1, n
        assert msg in L.dpp_last_error(), (n, L.dpp_last_error())
