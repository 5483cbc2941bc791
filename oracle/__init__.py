"""Plain FP64 CPU oracle (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C loops,
FP64, no fusion) through ctypes and shares no code with the HIP library.

Arrays are numpy float64, C-contiguous, shape (n, n) or (n, n, n) with the
x index fastest (last axis).  Every routine documents the passage of the
paper it follows in ``oracle.c``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

BC_DIRICHLET0 = 0
BC_PERIODIC = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_d = ctypes.c_int
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_p = ctypes.c_void_p


def lib():
    """Load liboracle.so, compiling it first only if it is not built."""
    global _lib
    if _lib is None:
        _lib = _load("liboracle.so")
    return _lib


_lib_omp = None


def lib_timing():
    """The host-timing build (liboracle_omp.so: -O3, OpenMP over the solve's cell
    loops); used only to time the oracle for the benchmark's CPU baseline."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _load("liboracle_omp.so")
    return _lib_omp


def _load(name):
    path = os.path.join(_HERE, name)
    if not os.path.exists(path):
        _build.build()
    L = ctypes.CDLL(path)
    sig = {
        "or_apply_A": [_d, _i64, _f64, _d, _p, _p],
        "or_residual": [_d, _i64, _f64, _d, _p, _p, _p],
        "or_rel_res": [_d, _i64, _f64, _d, _p, _p],
        "or_jacobi": [_d, _i64, _f64, _d, _f64, _p, _p, _p],
        "or_restrict": [_d, _i64, _p, _p],
        "or_prolong_add": [_d, _i64, _d, _p, _p],
        "or_coarse_solve": [_d, _i64, _f64, _d, _p, _p],
        "or_vcycle": [_d, _i64, _f64, _d, _d, _d, _f64, _i64, _p, _p],
        "or_mg_solve": [_d, _i64, _f64, _d, _p, _p, _f64, _d, _d, _f64, _d, _d, _d, _i64,
                        _p, _p, _p, _d],
        "or_ad_scalar_step": [_d, _i64, _f64, _d, _p, _p, _f64, _f64],
        "or_divergence": [_d, _i64, _f64, _p, _p],
        "or_gradient": [_d, _i64, _f64, _p, _p],
        "or_ns_momentum": [_d, _i64, _f64, _f64, _f64, _p, _p],
        "or_ns_step": [_d, _i64, _f64, _p, _p, _p, _p, _f64, _f64, _f64, _d, _d, _f64, _d, _d,
                       _i64, _p, _p],
        "or_prolong_const_add": [_d, _i64, _p, _p],
        "or_sawtooth": [_d, _i64, _f64, _d, _f64, _d, _d, _i64, _p, _p],
        "or_saw_solve": [_d, _i64, _f64, _d, _p, _p, _f64, _f64, _d, _d, _d, _d, _i64, _p, _p, _p, _d],
        "or_ad_apply": [_p, _i64, _f64, _p, _p],
        "or_ad_explicit_step": [_d, _i64, _f64, _d, _d, _p, _p, _f64, _f64],
        "or_nsc_derivative": [_d, _i64, _f64, _d, _d, _p, _p],
        "or_nsc_momentum": [_d, _i64, _f64, _d, _f64, _f64, _p, _p],
        "or_nsc_project": [_d, _i64, _f64, _d, _f64, _p, _p, _f64, _d, _p, _p],
        "or_nsc_step": [_d, _i64, _f64, _d, _f64, _f64, _p, _p, _f64, _d, _p],
        "or_ad_explicit_rate": [_d, _i64, _f64, _d, _d, _p, _p, _f64, _p],
        "or_ad_jacobi": [_p, _i64, _f64, _f64, _p, _p, _p],
        "or_ad_vcycle": [_p, _i64, _f64, _d, _d, _f64, _i64, _p, _p],
        "or_ad_sawtooth": [_p, _i64, _f64, _f64, _d, _d, _i64, _p, _p],
        "or_ad_solve": [_p, _i64, _f64, _p, _p, _f64, _d, _d, _d, _f64, _d, _d, _d, _i64, _p, _p, _p, _p, _d],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _f64 if name == "or_rel_res" else (None if name in (
            "or_apply_A", "or_residual", "or_jacobi", "or_restrict", "or_prolong_add",
            "or_divergence", "or_gradient", "or_ns_momentum", "or_prolong_const_add", "or_ad_apply",
            "or_ad_jacobi", "or_nsc_derivative", "or_nsc_momentum") else ctypes.c_int)
    L.or_threads.argtypes = [_d]
    L.or_threads.restype = ctypes.c_int
    return L


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid(a):
    d = a.ndim
    n = a.shape[0]
    assert d in (2, 3) and all(s == n for s in a.shape), a.shape
    return d, n


def _ptr_array(arrs):
    t = (ctypes.c_void_p * 3)(*[(_ptr(a) if a is not None else None) for a in arrs]
                              + [None] * (3 - len(arrs)))
    return ctypes.cast(t, ctypes.c_void_p), t


def apply_A(x, h, bc):
    x = _arr(x)
    d, n = _grid(x)
    y = np.empty_like(x)
    lib().or_apply_A(d, n, h, bc, _ptr(x), _ptr(y))
    return y


def residual(f, x, h, bc):
    f, x = _arr(f), _arr(x)
    d, n = _grid(x)
    r = np.empty_like(x)
    lib().or_residual(d, n, h, bc, _ptr(f), _ptr(x), _ptr(r))
    return r


def rel_res(f, x, h, bc):
    f, x = _arr(f), _arr(x)
    d, n = _grid(x)
    return lib().or_rel_res(d, n, h, bc, _ptr(f), _ptr(x))


def jacobi(f, x, h, bc, omega=2.0 / 3.0):
    f, x = _arr(f), _arr(x)
    d, n = _grid(x)
    y = np.empty_like(x)
    lib().or_jacobi(d, n, h, bc, omega, _ptr(f), _ptr(x), _ptr(y))
    return y


def restrict(r):
    r = _arr(r)
    d, n = _grid(r)
    fc = np.empty((n // 2,) * d)
    lib().or_restrict(d, n, _ptr(r), _ptr(fc))
    return fc


def prolong_add(e, x, bc):
    """Returns x + P e (x is not modified)."""
    e, x = _arr(e), _arr(x).copy()
    d, nc = _grid(e)
    assert x.shape == (2 * nc,) * d
    lib().or_prolong_add(d, nc, bc, _ptr(e), _ptr(x))
    return x


def coarse_solve(f, x, h, bc):
    """Returns x + A^{-1}(f - A x) (dense Cholesky)."""
    f, x = _arr(f), _arr(x).copy()
    d, n = _grid(x)
    st = lib().or_coarse_solve(d, n, h, bc, _ptr(f), _ptr(x))
    if st != 0:
        raise RuntimeError("coarse solve failed: %d" % st)
    return x


def vcycle(f, x, h, bc, nu1=2, nu2=2, omega=2.0 / 3.0, n_coarsest=4):
    """Returns the iterate after one V(nu1, nu2) cycle from x."""
    f, x = _arr(f), _arr(x).copy()
    d, n = _grid(x)
    st = lib().or_vcycle(d, n, h, bc, nu1, nu2, omega, n_coarsest, _ptr(f), _ptr(x))
    if st != 0:
        raise RuntimeError("vcycle failed: %d" % st)
    return x


def prolong_const_add(e, x):
    """Returns x + (the paper's copying prolongation of e) (x is not modified)."""
    e, x = _arr(e), _arr(x).copy()
    d, nc = _grid(e)
    assert x.shape == (2 * nc,) * d
    lib().or_prolong_const_add(d, nc, _ptr(e), _ptr(x))
    return x


def sawtooth(f, x, h, bc, alpha=1.0, nu=1, prolong_const=True, n_coarsest=4):
    """Returns the iterate after one sawtooth cycle (Appendix B) from x."""
    f, x = _arr(f), _arr(x).copy()
    d, n = _grid(x)
    lib().or_sawtooth(d, n, h, bc, alpha, nu, int(prolong_const), n_coarsest, _ptr(f), _ptr(x))
    return x


def saw_solve(f, h, bc, tol=1e-10, alpha=1.0, nu=1, prolong_const=True, max_cycles=200, fixed_cycles=0,
              n_coarsest=4):
    f = _arr(f)
    d, n = _grid(f)
    x = np.zeros_like(f)
    cyc = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(256)
    st = lib().or_saw_solve(d, n, h, bc, _ptr(f), _ptr(x), tol, alpha, nu, int(prolong_const), max_cycles,
                            fixed_cycles, n_coarsest, ctypes.byref(cyc), ctypes.byref(rr), _ptr(hist), 256)
    if st == -1:
        raise ValueError("oracle saw_solve: invalid arguments")
    return SolveResult(x, st, cyc.value, rr.value, hist[: min(cyc.value + 1, 256)])


class AdOp(ctypes.Structure):
    """The implicit advection-diffusion operator I + dt (a . D) + nu dt (-Laplacian)
    (scheme 0 upwind, 1 central)."""
    _fields_ = [("d", ctypes.c_int), ("bc", ctypes.c_int), ("scheme", ctypes.c_int), ("dt", ctypes.c_double),
                ("nu", ctypes.c_double), ("a", ctypes.c_double * 3)]


def ad_op(d, bc, dt, nu, a, scheme=0):
    aa = list(a) + [0.0] * (3 - len(a))
    return AdOp(d, bc, scheme, dt, nu, (ctypes.c_double * 3)(*aa))


def ad_apply(op, x, h):
    x = _arr(x)
    d, n = _grid(x)
    y = np.empty_like(x)
    lib().or_ad_apply(ctypes.byref(op), n, h, _ptr(x), _ptr(y))
    return y


def ad_jacobi(op, f, x, h, omega=2.0 / 3.0):
    f, x = _arr(f), _arr(x)
    d, n = _grid(x)
    y = np.empty_like(x)
    lib().or_ad_jacobi(ctypes.byref(op), n, h, omega, _ptr(f), _ptr(x), _ptr(y))
    return y


def ad_vcycle(op, f, x, h, nu1=2, nu2=2, omega=2.0 / 3.0, n_coarsest=4):
    f, x = _arr(f), _arr(x).copy()
    d, n = _grid(x)
    st = lib().or_ad_vcycle(ctypes.byref(op), n, h, nu1, nu2, omega, n_coarsest, _ptr(f), _ptr(x))
    if st != 0:
        raise RuntimeError("ad vcycle failed: %d" % st)
    return x


def ad_sawtooth(op, f, x, h, alpha=1.0, nu=1, prolong_const=True, n_coarsest=4):
    f, x = _arr(f), _arr(x).copy()
    d, n = _grid(x)
    lib().or_ad_sawtooth(ctypes.byref(op), n, h, alpha, nu, int(prolong_const), n_coarsest, _ptr(f), _ptr(x))
    return x


def ad_solve(op, f, h, tol=1e-10, cycle=0, nu1=2, nu2=2, omega=2.0 / 3.0, prolong_const=False, max_cycles=200,
             fixed_cycles=0, n_coarsest=4):
    f = _arr(f)
    d, n = _grid(f)
    x = np.zeros_like(f)
    cyc = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist, l1 = np.zeros(512), np.zeros(512)
    st = lib().or_ad_solve(ctypes.byref(op), n, h, _ptr(f), _ptr(x), tol, cycle, nu1, nu2, omega, int(prolong_const),
                           max_cycles, fixed_cycles, n_coarsest, ctypes.byref(cyc), ctypes.byref(rr), _ptr(hist),
                           _ptr(l1), 512)
    if st == -1:
        raise ValueError("oracle ad_solve: invalid arguments")
    res = SolveResult(x, st, cyc.value, rr.value, hist[: min(cyc.value + 1, 512)])
    res.l1diff = l1[: min(cyc.value, 512)]
    return res


class SolveResult:
    def __init__(self, x, status, cycles, rel_res, hist):
        self.x, self.status, self.cycles, self.rel_res, self.hist = x, status, cycles, rel_res, hist


def mg_solve(f, h, bc, tol=1e-10, nu1=2, nu2=2, omega=2.0 / 3.0, max_cycles=200,
             fixed_cycles=0, x0=None, n_coarsest=4, threads=0):
    """Multigrid solve (or_mg_solve).  threads > 0 runs the host-timing build with
    that many OpenMP threads instead of the test build."""
    f = _arr(f)
    d, n = _grid(f)
    x = np.zeros_like(f) if x0 is None else _arr(x0).copy()
    cyc = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(256)
    L = lib()
    if threads > 0:
        L = lib_timing()
        L.or_threads(threads)
    st = L.or_mg_solve(d, n, h, bc, _ptr(f), _ptr(x), tol, nu1, nu2, omega, max_cycles,
                           fixed_cycles, 0 if x0 is None else 1, n_coarsest,
                           ctypes.byref(cyc), ctypes.byref(rr), _ptr(hist), 256)
    if st == -1:
        raise ValueError("oracle mg_solve: invalid arguments")
    return SolveResult(x, st, cyc.value, rr.value, hist[: min(cyc.value + 1, 256)])


BC_NEUMANN = 2
SCHEME_CENTRAL, SCHEME_UPWIND, SCHEME_FE = 0, 1, 2


def ad_explicit_step(T, h, bc, dt, nu, a=None, scheme=SCHEME_CENTRAL):
    """One predictor-corrector step with the chosen filter family; returns the new T."""
    T = _arr(T).copy()
    d, n = _grid(T)
    keep = ap = None
    if a is not None:
        a = [_arr(c) for c in a]
        ap, keep = _ptr_array(a)
    if lib().or_ad_explicit_step(d, n, h, bc, scheme, _ptr(T), ap, dt, nu) != 0:
        raise ValueError("oracle ad_explicit_step: invalid arguments")
    del keep
    return T


def ad_explicit_rate(T, h, bc, nu, a=None, scheme=SCHEME_CENTRAL):
    """The rate R(T) = a . D T + nu (diffusion filter * T) of the explicit step."""
    T = _arr(T)
    d, n = _grid(T)
    keep = ap = None
    if a is not None:
        a = [_arr(c) for c in a]
        ap, keep = _ptr_array(a)
    R = np.empty_like(T)
    if lib().or_ad_explicit_rate(d, n, h, bc, scheme, _ptr(T), ap, nu, _ptr(R)) != 0:
        raise ValueError("oracle ad_explicit_rate: invalid arguments")
    del keep
    return R


def nsc_derivative(f, h, e, scheme=SCHEME_FE):
    """D_e f of the collocated step (periodic): the scheme's first-derivative filter."""
    f = _arr(f)
    d, n = _grid(f)
    g = np.empty_like(f)
    lib().or_nsc_derivative(d, n, h, scheme, e, _ptr(f), _ptr(g))
    return g


def _qptrs(q):
    q = [_arr(c).copy() for c in q]
    return q, _ptr_array(q)


def nsc_momentum(q, p, h, dt, nu, scheme=SCHEME_FE):
    """Momentum predictor-corrector of the collocated step; returns q*."""
    q, (qp, keep) = _qptrs(q)
    p = _arr(p)
    d, n = _grid(p)
    lib().or_nsc_momentum(d, n, h, scheme, dt, nu, qp, _ptr(p))
    del keep
    return q


def nsc_project(q, p, h, dt, scheme=SCHEME_FE, tol=1e-12, fixed_cycles=0):
    """Pressure and velocity corrections of the collocated step; returns (q, p, dp, cycles)."""
    q, (qp, keep) = _qptrs(q)
    p = _arr(p).copy()
    d, n = _grid(p)
    dp = np.empty_like(p)
    cyc = ctypes.c_int(0)
    st = lib().or_nsc_project(d, n, h, scheme, dt, qp, _ptr(p), tol, fixed_cycles, ctypes.byref(cyc), _ptr(dp))
    del keep
    if st not in (0, -2):
        raise ValueError("oracle nsc_project failed: %d" % st)
    return q, p, dp, cyc.value


def nsc_step(q, p, h, dt, nu, scheme=SCHEME_FE, tol=1e-12, fixed_cycles=0):
    """One collocated projection step; returns (q, p, cycles)."""
    q, (qp, keep) = _qptrs(q)
    p = _arr(p).copy()
    d, n = _grid(p)
    cyc = ctypes.c_int(0)
    st = lib().or_nsc_step(d, n, h, scheme, dt, nu, qp, _ptr(p), tol, fixed_cycles, ctypes.byref(cyc))
    del keep
    if st not in (0, -2):
        raise ValueError("oracle nsc_step failed: %d" % st)
    return q, p, cyc.value


def ad_scalar_step(T, h, bc, dt, nu, a=None):
    """One predictor-corrector advection-diffusion step; returns the new T."""
    T = _arr(T).copy()
    d, n = _grid(T)
    keep = None
    ap = None
    if a is not None:
        a = [_arr(c) for c in a]
        ap, keep = _ptr_array(a)
    lib().or_ad_scalar_step(d, n, h, bc, _ptr(T), ap, dt, nu)
    del keep
    return T


def divergence(q, h):
    q = [_arr(c) for c in q]
    d, n = _grid(q[0])
    div = np.empty_like(q[0])
    qp, keep = _ptr_array(q)
    lib().or_divergence(d, n, h, qp, _ptr(div))
    return div


def gradient(p, h):
    p = _arr(p)
    d, n = _grid(p)
    g = [np.empty_like(p) for _ in range(d)]
    gp, keep = _ptr_array(g)
    lib().or_gradient(d, n, h, _ptr(p), gp)
    return g


def ns_momentum(q, p, h, dt, nu):
    """Predictor-corrector momentum stages; returns q* (list of arrays)."""
    q = [_arr(c).copy() for c in q]
    p = _arr(p)
    d, n = _grid(p)
    qp, keep = _ptr_array(q)
    lib().or_ns_momentum(d, n, h, dt, nu, qp, _ptr(p))
    return q


def ns_step(q, p, h, dt, nu, tol=1e-10, nu1=2, nu2=2, omega=2.0 / 3.0, max_cycles=200,
            fixed_cycles=0, n_coarsest=4):
    """One projection step; returns (q_new list, p_new, cycles, rel_res, status)."""
    q = [_arr(c).copy() for c in q]
    p = _arr(p).copy()
    d, n = _grid(p)
    w = q[2] if d == 3 else None
    cyc = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = lib().or_ns_step(d, n, h, _ptr(q[0]), _ptr(q[1]), _ptr(w) if w is not None else None,
                          _ptr(p), dt, nu, tol, nu1, nu2, omega, max_cycles, fixed_cycles,
                          n_coarsest, ctypes.byref(cyc), ctypes.byref(rr))
    return q, p, cyc.value, rr.value, st
