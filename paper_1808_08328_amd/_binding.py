"""ctypes marshalling for libdpp.so (names follow the C ABI without the dpp_ prefix)."""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libdpp.so")
_lib = None

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_NOT_CONVERGED",
          5: "ERR_NUMERIC", 6: "ERR_BREAKDOWN", 7: "ERR_UNSUPPORTED", 8: "ERR_STAGNATED"}


class DppError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Box(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("elem", C.c_int)]


ELEM = {"p1": 0, "q1": 1, "dg": 2}


class _Params(C.Structure):
    _fields_ = [("mu", C.c_double), ("k1", C.c_void_p), ("k2", C.c_void_p), ("beta", C.c_double),
                ("beta_cells", C.c_void_p), ("body", C.c_void_p), ("p0_1", C.c_void_p),
                ("p0_2", C.c_void_p), ("face_bc", C.c_void_p), ("u_bc_1", C.c_void_p),
                ("u_bc_2", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxiter", C.c_int), ("rtol", C.c_double),
                ("precision", C.c_int), ("inner_rtol", C.c_double), ("max_refine", C.c_int),
                ("coarse_max", C.c_int), ("cheb_degree", C.c_int), ("cheb_lo_frac", C.c_double),
                ("cheb_hi_factor", C.c_double), ("power_iters", C.c_int), ("use_graph", C.c_int),
                ("cheb_pre_fine", C.c_int), ("cheb_post_fine", C.c_int),
                ("cheb_pre_coarse", C.c_int), ("cheb_post_coarse", C.c_int),
                ("inner_maxiter", C.c_int), ("schedule", C.c_int), ("stag_cycles", C.c_int),
                ("stag_ratio", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("refinements", C.c_int),
                ("converged", C.c_int), ("rel_residual", C.c_double), ("ms_solve", C.c_double),
                ("ms_setup", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    """Load libdpp.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise RuntimeError("libdpp.so is not built (run __graft_entry__.build()); "
                           "there is no fallback path")
    L = C.CDLL(lib_path)
    P, I64 = C.c_void_p, C.POINTER(C.c_int64)
    sig = {
        "dpp_default_opts": (None, [C.POINTER(_Opts)]),
        "dpp_last_error": (C.c_char_p, []),
        "dpp_assemble": (C.c_int, [C.POINTER(_Box), C.POINTER(_Params), P, C.POINTER(P)]),
        "dpp_problem_sizes": (C.c_int, [P, I64, I64, I64, I64]),
        "dpp_rhs": (C.c_int, [P, P, P]),
        "dpp_export_csr": (C.c_int, [P, P, P, P, P]),
        "dpp_spmv": (C.c_int, [P, C.c_int, P, P, P]),
        "dpp_setup_precond": (C.c_int, [P, C.POINTER(_Opts), P, C.POINTER(P)]),
        "dpp_precond_info": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)]),
        "dpp_precond_apply": (C.c_int, [P, P, P, P]),
        "dpp_precond_shape": (C.c_int, [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "dpp_precond_set_shape": (C.c_int, [P, C.c_int, C.c_int, C.c_int]),
        "dpp_vcycle": (C.c_int, [P, P, P, P]),
        "dpp_level_spmv": (C.c_int, [P, C.c_int, C.c_int, P, P, P]),
        "dpp_solve": (C.c_int, [P, P, C.POINTER(_Opts), P, P, C.POINTER(SolveStats), P]),
        "dpp_solve_adjoint": (C.c_int, [P, P, C.POINTER(_Opts), P, P, C.POINTER(SolveStats), P]),
        "dpp_param_grad": (C.c_int, [P, P, P, P, P, P, P]),
        "dpp_mms_l2_errors": (C.c_int, [P, P, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), P]),
        "dpp_simplex_rule": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "dpp_profile_enable": (C.c_int, [C.c_int]),
        "dpp_profile_read": (C.c_int, [C.c_int, I64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "dpp_assemble_batch": (C.c_int, [C.c_int, C.POINTER(_Box), C.POINTER(_Params),
                                         C.POINTER(_Opts), P, C.POINTER(P)]),
        "dpp_batch_sizes": (C.c_int, [P, I64, I64]),
        "dpp_batch_lanes": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "dpp_solve_batch": (C.c_int, [P, C.POINTER(_Opts), P, C.POINTER(SolveStats), P]),
        "dpp_batch_spmv": (C.c_int, [P, P, P, P]),
        "dpp_batch_precond_apply": (C.c_int, [P, P, P, P]),
        "dpp_destroy_batch": (None, [P]),
        "dpp_destroy_problem": (None, [P]),
        "dpp_destroy_precond": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st, allow=()):
    if st != 0 and st not in allow:
        raise DppError(st, lib().dpp_last_error().decode())
    return st


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


PROFILE_FAMILIES = ["spmv_K", "cheb_S_l0", "resid_S_l0", "schur_rhs", "schur_vel", "coarse_levels",
                    "vector_l0", "arnoldi", "batch_spmv_K", "batch_cheb_S_l0", "batch_schur",
                    "batch_levels", "batch_arnoldi", "dg_vel", "dg_pres", "dg_transfer"]


def profile_enable(on=True):
    """dpp_profile_enable: time kernel families with HIP events (clears records)."""
    _check(lib().dpp_profile_enable(1 if on else 0))


def profile_read():
    """dpp_profile_read for every family -> {name: (launches, total_ms, total_bytes)}."""
    out = {}
    for i, name in enumerate(PROFILE_FAMILIES):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().dpp_profile_read(i, C.byref(n), C.byref(ms), C.byref(by)))
        out[name] = (n.value, ms.value, by.value)
    return out


def default_opts(**kw):
    o = _Opts()
    lib().dpp_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown solver option %r" % k)
        setattr(o, k, v)
    return o


class Precond:
    def __init__(self, problem, handle, opts):
        self.problem, self.handle, self.opts = problem, handle, opts

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpp_destroy_precond(self.handle)
            self.handle = None

    def info(self):
        nl = C.c_int()
        ln = (C.c_int * 48)()
        hi = (C.c_double * 32)()
        _check(lib().dpp_precond_info(self.handle, C.byref(nl), ln, hi))
        return dict(levels=nl.value,
                    level_n=[tuple(ln[3 * l:3 * l + 3]) for l in range(nl.value)],
                    hi=[(hi[2 * l], hi[2 * l + 1]) for l in range(nl.value)])

    def shape(self, level):
        lanes, sym = C.c_int(), C.c_int()
        _check(lib().dpp_precond_shape(self.handle, level, C.byref(lanes), C.byref(sym)))
        return lanes.value, sym.value

    def set_shape(self, level, lanes, sym):
        _check(lib().dpp_precond_set_shape(self.handle, level, lanes, sym))

    def apply(self, r, stream=None):
        z = torch.empty_like(r)
        _check(lib().dpp_precond_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def vcycle(self, b, stream=None):
        x = torch.empty_like(b)
        _check(lib().dpp_vcycle(self.handle, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def level_spmv(self, level, net, x, stream=None):
        y = torch.empty_like(x)
        _check(lib().dpp_level_spmv(self.handle, level, net, _ptr(x), _ptr(y), _stream(stream)))
        return y


class Problem:
    """An assembled DPP system (handle over dpp_problem)."""

    def __init__(self, handle, dim, n, beta_per_cell=False, elem="p1"):
        self.handle, self.dim, self.n, self.elem = handle, dim, tuple(n), elem
        self.beta_per_cell = beta_per_cell
        nd, nn, nc, nz = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().dpp_problem_sizes(handle, C.byref(nd), C.byref(nn), C.byref(nc), C.byref(nz)))
        self.n_dof, self.n_nodes, self.n_cells, self.nnz = nd.value, nn.value, nc.value, nz.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpp_destroy_problem(self.handle)
            self.handle = None

    def rhs(self, stream=None):
        f = torch.empty(self.n_dof, dtype=torch.float64, device="cuda")
        _check(lib().dpp_rhs(self.handle, _ptr(f), _stream(stream)))
        return f

    def export_csr(self, stream=None):
        rp = torch.empty(self.n_dof + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        vv = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(lib().dpp_export_csr(self.handle, _ptr(rp), _ptr(ci), _ptr(vv), _stream(stream)))
        return rp, ci, vv

    def fields(self, x):
        """Views of u1, p1, u2, p2 in a vector laid out as [u1 | p1 | u2 | p2]."""
        N, d = self.n_nodes, self.dim
        cuts = [0, d * N, (d + 1) * N, (2 * d + 1) * N, 2 * (d + 1) * N]
        return {f: x[cuts[i]:cuts[i + 1]] for i, f in enumerate(("u1", "p1", "u2", "p2"))}

    def spmv(self, x, which=0, stream=None):
        N, d = self.n_nodes, self.dim
        out = {0: self.n_dof, 1: d * N, 2: d * N, 3: N, 4: N}[which]
        y = torch.empty(out, dtype=torch.float64, device=x.device)
        _check(lib().dpp_spmv(self.handle, which, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def setup_precond(self, stream=None, **opts):
        o = default_opts(**opts)
        h = C.c_void_p()
        _check(lib().dpp_setup_precond(self.handle, C.byref(o), _stream(stream), C.byref(h)))
        return Precond(self, h, o)

    def solve(self, pc, rhs=None, x0=None, stream=None, allow_unconverged=False, **opts):
        o = default_opts(**{**{k: getattr(pc.opts, k) for k, _ in _Opts._fields_}, **opts})
        x = torch.zeros(self.n_dof, dtype=torch.float64, device="cuda") if x0 is None else x0.clone()
        st = SolveStats()
        _check(lib().dpp_solve(self.handle, pc.handle, C.byref(o), _ptr(rhs), _ptr(x), C.byref(st),
                               _stream(stream)), allow=(4, 8) if allow_unconverged else ())
        return x, st

    def solve_adjoint(self, pc, g, stream=None, **opts):
        o = default_opts(**{**{k: getattr(pc.opts, k) for k, _ in _Opts._fields_}, **opts})
        lam = torch.empty(self.n_dof, dtype=torch.float64, device="cuda")
        st = SolveStats()
        _check(lib().dpp_solve_adjoint(self.handle, pc.handle, C.byref(o), _ptr(g), _ptr(lam),
                                       C.byref(st), _stream(stream)))
        return lam, st

    def param_grad(self, x, lam, stream=None):
        """Returns (dJ/dln k1 [n_cells], dJ/dln k2 [n_cells], dJ/dbeta [1] or [n_cells])."""
        g1 = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        g2 = torch.empty_like(g1)
        gb = torch.empty(self.n_cells if self.beta_per_cell else 1, dtype=torch.float64,
                         device="cuda")
        _check(lib().dpp_param_grad(self.handle, _ptr(x), _ptr(lam), _ptr(g1), _ptr(g2), _ptr(gb),
                                    _stream(stream)))
        return g1, g2, gb

    def mms_l2_errors(self, x, mms, q=4, stream=None):
        """dpp_mms_l2_errors: {'u1', 'p1', 'u2', 'p2'} L2 errors of x against the
        manufactured solution with mms = (k1, k2, beta, mu)."""
        m = (C.c_double * 4)(*[float(v) for v in mms])
        e = (C.c_double * 4)()
        _check(lib().dpp_mms_l2_errors(self.handle, _ptr(x), m, int(q), e, _stream(stream)))
        return dict(zip(("u1", "p1", "u2", "p2"), list(e)))



def simplex_rule(dim, q):
    """dpp_simplex_rule (host only): barycentric points [q^dim, dim+1] and
    weights [q^dim] of the conical-product Gauss rule."""
    import numpy as np
    nq = q ** dim
    lam = (C.c_double * (nq * (dim + 1)))()
    w = (C.c_double * nq)()
    _check(lib().dpp_simplex_rule(int(dim), int(q), lam, w))
    return np.array(lam[:]).reshape(nq, dim + 1), np.array(w[:])

def assemble(dim, n, k1, k2, p0_1, p0_2, beta=1.0, mu=1.0, L=None, body=None, beta_cells=None,
             face_bc=None, u_bc_1=None, u_bc_2=None, stream=None, elem="p1"):
    """dpp_assemble on device tensors (float64, contiguous); face_bc is a host
    int8 array [2, 2*dim] (velocity faces) or None; elem "p1" (Kuhn simplices)
    or "q1" (box cells)."""
    lib()
    box = _Box()
    box.dim = dim
    box.elem = ELEM[elem]
    for a in range(3):
        box.n[a] = int(n[a]) if a < dim else 0
        box.L[a] = float(L[a]) if (L is not None and a < dim) else (1.0 if a < dim else 0.0)
    p = _Params()
    p.mu = float(mu)
    p.k1, p.k2 = _ptr(k1), _ptr(k2)
    p.beta = float(beta)
    p.beta_cells = _ptr(beta_cells)
    p.body = _ptr(body)
    p.p0_1, p.p0_2 = _ptr(p0_1), _ptr(p0_2)
    fb = None
    if face_bc is not None:
        import numpy as np
        fb = np.ascontiguousarray(np.asarray(face_bc, dtype=np.int8).reshape(2, 2 * dim))
        p.face_bc = fb.ctypes.data_as(C.c_void_p)
    else:
        p.face_bc = None
    p.u_bc_1, p.u_bc_2 = _ptr(u_bc_1), _ptr(u_bc_2)
    h = C.c_void_p()
    _check(lib().dpp_assemble(C.byref(box), C.byref(p), _stream(stream), C.byref(h)))
    return Problem(h, dim, n, beta_per_cell=beta_cells is not None, elem=elem)


def assemble_problem(prob, device="cuda", stream=None):
    """Assemble a ``dpp_inputs.Problem`` (host arrays are copied to the device)."""
    dv = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)
    beta = prob.beta
    beta_cells = None
    if hasattr(beta, "__len__"):
        beta_cells, beta = dv(beta), 0.0
    body = None if prob.body is None else dv(
        (torch.as_tensor(prob.body, dtype=torch.float64) * prob.gamma).expand(prob.n_cells, prob.dim)
        .contiguous())
    fb = getattr(prob, "face_bc", None)
    ub = [None if getattr(prob, k, None) is None else dv(getattr(prob, k)).reshape(-1)
          for k in ("u_bc_1", "u_bc_2")]
    return assemble(prob.dim, prob.n, dv(prob.k1), dv(prob.k2), dv(prob.p0_1), dv(prob.p0_2),
                    beta=float(beta), mu=prob.mu, L=prob.L, body=body, beta_cells=beta_cells,
                    face_bc=fb, u_bc_1=ub[0], u_bc_2=ub[1], stream=stream,
                    elem=getattr(prob, "elem", "p1"))


class Batch:
    """Many independent instances solved together (handle over dpp_batch)."""

    def __init__(self, handle, nb, dim, keep):
        self.handle, self.nb, self.dim, self._keep = handle, nb, dim, keep
        tot = C.c_int64()
        offs = (C.c_int64 * (nb + 1))()
        _check(lib().dpp_batch_sizes(handle, C.byref(tot), offs))
        self.n_dof = tot.value
        self.offsets = [offs[i] for i in range(nb + 1)]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpp_destroy_batch(self.handle)
            self.handle = None

    def lanes(self):
        nl = C.c_int()
        ln = (C.c_int * 16)()
        _check(lib().dpp_batch_lanes(self.handle, C.byref(nl), ln))
        return [ln[i] for i in range(nl.value)]

    def solve(self, x0=None, stream=None, allow_unconverged=False, **opts):
        o = default_opts(**opts)
        x = torch.zeros(self.n_dof, dtype=torch.float64, device="cuda") if x0 is None else x0.clone()
        st = (SolveStats * self.nb)()
        _check(lib().dpp_solve_batch(self.handle, C.byref(o), _ptr(x), st, _stream(stream)),
               allow=(4, 8) if allow_unconverged else ())
        return x, [st[i] for i in range(self.nb)]

    def spmv(self, x, stream=None):
        y = torch.empty_like(x)
        _check(lib().dpp_batch_spmv(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def precond_apply(self, r, stream=None):
        z = torch.empty_like(r)
        _check(lib().dpp_batch_precond_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def split(self, x):
        return [x[self.offsets[i]:self.offsets[i + 1]] for i in range(self.nb)]


def assemble_batch(problems, stream=None, **opts):
    """dpp_assemble_batch over a list of ``dpp_inputs.Problem`` (one dimension)."""
    lib()
    nb = len(problems)
    boxes = (_Box * nb)()
    params = (_Params * nb)()
    keep = []
    dv = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to("cuda")
    for i, pr in enumerate(problems):
        boxes[i].dim = pr.dim
        boxes[i].elem = ELEM[getattr(pr, "elem", "p1")]
        for a in range(3):
            boxes[i].n[a] = int(pr.n[a]) if a < pr.dim else 0
            boxes[i].L[a] = float(pr.L[a]) if a < pr.dim else 0.0
        arrs = [dv(pr.k1), dv(pr.k2), dv(pr.p0_1), dv(pr.p0_2)]
        p = params[i]
        p.mu = float(pr.mu)
        p.k1, p.k2, p.p0_1, p.p0_2 = (_ptr(t) for t in arrs)
        p.beta = float(pr.beta)
        p.beta_cells = None
        p.body = None
        p.face_bc = p.u_bc_1 = p.u_bc_2 = None
        if getattr(pr, "face_bc", None) is not None:
            import numpy as np
            fb = np.ascontiguousarray(np.asarray(pr.face_bc, dtype=np.int8).reshape(2, 2 * pr.dim))
            ub = [None if getattr(pr, k, None) is None else dv(getattr(pr, k)).reshape(-1)
                  for k in ("u_bc_1", "u_bc_2")]
            arrs += [fb] + [u for u in ub if u is not None]
            p.face_bc = fb.ctypes.data_as(C.c_void_p)
            p.u_bc_1, p.u_bc_2 = _ptr(ub[0]), _ptr(ub[1])
        keep.append(arrs)
    o = default_opts(**opts)
    h = C.c_void_p()
    _check(lib().dpp_assemble_batch(nb, boxes, params, C.byref(o), _stream(stream), C.byref(h)))
    return Batch(h, nb, problems[0].dim, keep)


class DppSolve(torch.autograd.Function):
    """x = K(theta)^-1 f with theta = (ln k1 per cell, ln k2 per cell, beta).

    forward: dpp_assemble + dpp_setup_precond + dpp_solve; backward:
    dpp_solve_adjoint (K^T lambda = dJ/dx) + dpp_param_grad.  Boundary data
    are held fixed (df/dtheta = 0).  beta is one scalar (a tensor of one
    element; its gradient has the same shape).  spec: dim, n, p0_1, p0_2
    (device tensors), optional mu and L; body forces and velocity faces are
    not differentiated here and are rejected."""

    @staticmethod
    def forward(ctx, logk1, logk2, beta, spec, opts):
        bad = [k for k in ("body", "beta_cells", "face_bc", "u_bc_1", "u_bc_2")
               if spec.get(k) is not None]
        if bad:
            raise ValueError("DppSolve does not support %s" % ", ".join(bad))
        if not torch.is_tensor(beta) or beta.numel() != 1:
            raise ValueError("beta must be a tensor holding one scalar")
        prob = assemble(spec["dim"], spec["n"], torch.exp(logk1).contiguous(),
                        torch.exp(logk2).contiguous(), spec["p0_1"], spec["p0_2"],
                        beta=float(beta.reshape(())), mu=spec.get("mu", 1.0), L=spec.get("L"))
        pc = prob.setup_precond(**(opts or {}))
        x, _ = prob.solve(pc, **(opts or {}))
        ctx.prob, ctx.pc, ctx.opts, ctx.beta_shape = prob, pc, opts, beta.shape
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam, _ = ctx.prob.solve_adjoint(ctx.pc, gx.contiguous(), **(ctx.opts or {}))
        g1, g2, gb = ctx.prob.param_grad(x, lam)
        return g1, g2, gb.reshape(ctx.beta_shape), None, None
