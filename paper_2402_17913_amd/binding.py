"""ctypes binding of libneuphys.so (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: tensors must already be on the GPU, contiguous and of
the dtype the entry point expects.  If the library is not built, importing
the binding raises immediately -- there is no fallback.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libneuphys.so")

NP_OK, NP_EINVAL, NP_ENOCONV, NP_ENAN, NP_EHIP, NP_ENOMEM = 0, -1, -2, -3, -4, -5
BC_DIRICHLET0, BC_PERIODIC = 0, 1
FP64, FP32, BF16 = 0, 1, 2
_STATUS = {0: "NP_OK", -1: "NP_EINVAL", -2: "NP_ENOCONV", -3: "NP_ENAN", -4: "NP_EHIP", -5: "NP_ENOMEM"}


class NpDims(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3)]


class NpMgOpts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("fixed_cycles", ctypes.c_int),
                ("smooth_prec", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("stream", ctypes.c_void_p), ("cycle", ctypes.c_int),
                ("prolong", ctypes.c_int), ("cnn_cgc", ctypes.c_int)]


class NpMgStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("used_fallback", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("rho_est", ctypes.c_double), ("hist", ctypes.c_double * 256), ("cgc_accepted", ctypes.c_int)]

    def as_dict(self):
        n = min(256, max(self.outer_iters, self.cycles) + 1)
        return dict(cycles=self.cycles, outer_iters=self.outer_iters,
                    used_fallback=self.used_fallback, rel_res=self.rel_res,
                    rho_est=self.rho_est, hist=list(self.hist[:n]), cgc_accepted=self.cgc_accepted)


class NpAdOp(ctypes.Structure):
    """Backward-Euler advection-diffusion operator (scheme 0 upwind, 1 central)."""
    _fields_ = [("dt", ctypes.c_double), ("nu", ctypes.c_double), ("a", ctypes.c_double * 3),
                ("scheme", ctypes.c_int)]


def ad_op(dt, nu, a, scheme=0):
    aa = list(a) + [0.0] * (3 - len(a))
    return NpAdOp(dt, nu, (ctypes.c_double * 3)(*aa), scheme)


class NeuphysError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s -> %s: %s" % (fn, _STATUS.get(status, status), msg))
        self.status = status


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_SIGS = {
    "np_default_opts": (None, [ctypes.POINTER(NpMgOpts)]),
    "np_last_error": (ctypes.c_char_p, []),
    "np_release_all": (None, []),
    "mg_poisson_solve": (_I, [NpDims, _D, _I, _P, _P, _D, ctypes.POINTER(NpMgOpts),
                              ctypes.POINTER(NpMgStats)]),
    "mg_poisson_solve_noalloc": (_I, [NpDims, _D, _I, _P, _P, _D, ctypes.POINTER(NpMgOpts),
                                      ctypes.POINTER(NpMgStats)]),
    "ns_projection_step": (_I, [NpDims, _D, _P, _P, _P, _P, _D, _D, _I, _D,
                                ctypes.POINTER(NpMgOpts), ctypes.POINTER(NpMgStats)]),
    "np_ad_scalar_step": (_I, [NpDims, _D, _P, _P, _D, _D, _I, ctypes.POINTER(NpMgOpts)]),
    "np_op_apply": (_I, [NpDims, _D, _I, _P, _P, _P]),
    "np_op_jacobi": (_I, [NpDims, _D, _I, _D, _P, _P, _P, _P]),
    "np_op_resid_restrict": (_I, [NpDims, _D, _I, _P, _P, _P, _P]),
    "np_op_prolong_add": (_I, [NpDims, _I, _P, _P, _P]),
    "np_op_vcycle": (_I, [NpDims, _D, _I, _P, _P, ctypes.POINTER(NpMgOpts)]),
    "np_op_resid_norm": (_I, [NpDims, _D, _I, _P, _P, ctypes.POINTER(_D), _P]),
    "np_prof_enable": (None, [_I]),
    "np_prof_read": (_I, [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "np_set_tuning": (_I, [ctypes.c_char_p, _I]),
    "mg_poisson_solve_batched": (_I, [_I, ctypes.POINTER(NpDims), ctypes.POINTER(_D), _I, _P, _P, _D,
                                      ctypes.POINTER(NpMgOpts), ctypes.POINTER(NpMgStats)]),
    "np_last_autotune": (_I, [ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "np_last_batched_settings": (_I, [ctypes.POINTER(_I)] * 6),
    "ns_projection_step_io": (_I, [NpDims, _D, _P, _P, _P, _P, _D, _D, _I, _D, ctypes.POINTER(NpMgOpts),
                                   ctypes.POINTER(NpMgStats), _P, _P]),
    "np_cnn_create": (_I, [_I, _I, ctypes.POINTER(_P)]),
    "np_cnn_destroy": (None, [_P]),
    "np_cnn_num_params": (ctypes.c_int64, [_P]),
    "np_cnn_set_params": (_I, [_P, _P, ctypes.c_int64]),
    "np_cnn_get_params": (_I, [_P, _P, ctypes.c_int64]),
    "np_cnn_get_grads": (_I, [_P, _P, ctypes.c_int64]),
    "np_cnn_forward": (_I, [_P, _P, _P, _P]),
    "np_cnn_gradients": (_I, [_P, _I, _P, _P, ctypes.POINTER(_D), _P]),
    "np_cnn_train_step": (_I, [_P, _I, _P, _P, ctypes.c_float, ctypes.POINTER(_D), _P]),
    "np_cnn_prepare": (_I, [_P, NpDims, _P, _P, _P, _P, ctypes.POINTER(_D), _P]),
    "np_cnn_attach": (_I, [_P]),
    "np_cnn_save": (_I, [_P, ctypes.c_char_p]),
    "np_cnn_open": (_I, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "np_cnn_load": (_I, [ctypes.c_char_p]),
    "np_cnn_init": (_I, [_P, ctypes.c_uint64]),
    "np_cnn_train": (_I, [ctypes.POINTER(NpDims), _I, _I, _P, _P, ctypes.c_char_p, ctypes.c_char_p,
                          ctypes.POINTER(_D)]),
    "np_get_tuning": (_I, [ctypes.c_char_p]),
    "np_prof_level": (_I, [NpDims, _D, _I, _I, _I, _P, _P, _P, _I, _P, ctypes.POINTER(_D)]),
    "np_op_level": (_I, [NpDims, _D, _I, _I, _I, _P, _P, _P, _P, _P]),
    "np_ad_implicit_solve": (_I, [NpDims, _D, _I, ctypes.POINTER(NpAdOp), _P, _P, _D, ctypes.POINTER(NpMgOpts),
                                  ctypes.POINTER(NpMgStats), ctypes.POINTER(_D)]),
    "np_ad_apply": (_I, [NpDims, _D, _I, ctypes.POINTER(NpAdOp), _P, _P, _P]),
    "np_ad_explicit_step": (_I, [NpDims, _D, _P, _P, _D, _D, _I, _I, ctypes.POINTER(NpMgOpts)]),
    "ns_collocated_step": (_I, [NpDims, _D, _P, _P, _P, _P, _D, _D, _I, _D, ctypes.POINTER(NpMgOpts),
                                ctypes.POINTER(NpMgStats)]),
    "np_nsc_divergence": (_I, [NpDims, _D, _P, _P, _P, _I, _P, _P]),
    "np_ad_prof_level": (_I, [NpDims, _D, _I, ctypes.POINTER(NpAdOp), _I, _P, _P, _P, _I, _P, ctypes.POINTER(_D)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libneuphys.so is not built (expected at %s); run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def _check(fn, st):
    if st != NP_OK:
        raise NeuphysError(fn, st, lib.np_last_error().decode())


def _dims(t):
    if t.dim() not in (2, 3):
        raise ValueError("fields must be 2D or 3D tensors")
    n = list(reversed(t.shape)) + [1] * (3 - t.dim())
    return NpDims(t.dim(), (ctypes.c_int64 * 3)(*n))


def _dev(t, dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype):
        raise ValueError("expected a contiguous %s CUDA tensor" % dtype)
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


CYCLE_V, CYCLE_SAWTOOTH = 0, 1
PROLONG_LINEAR, PROLONG_COPY = 0, 1


def make_opts(nu1=2, nu2=2, omega=2.0 / 3.0, max_cycles=200, fixed_cycles=0, smooth_prec=FP64,
              inner_cycles=0, warm_start=0, cycle=CYCLE_V, prolong=PROLONG_LINEAR, cnn_cgc=0):
    o = NpMgOpts()
    lib.np_default_opts(ctypes.byref(o))
    o.nu1, o.nu2, o.omega = nu1, nu2, omega
    o.max_cycles, o.fixed_cycles = max_cycles, fixed_cycles
    o.smooth_prec, o.inner_cycles, o.warm_start = smooth_prec, inner_cycles, warm_start
    o.cycle, o.prolong, o.cnn_cgc = cycle, prolong, cnn_cgc
    o.stream = _stream()
    return o


def mg_poisson_solve(rhs, x, h, bc, tol=1e-10, check=True, **opts):
    """Solves A x = rhs in place in x; returns (status, stats dict)."""
    o = make_opts(**opts)
    st = NpMgStats()
    s = lib.mg_poisson_solve(_dims(rhs), h, bc, _dev(rhs), _dev(x), tol, ctypes.byref(o),
                             ctypes.byref(st))
    if check:
        _check("mg_poisson_solve", s)
    return s, st.as_dict()


def mg_poisson_solve_noalloc(rhs, x, h, bc, tol=1e-10, check=True, **opts):
    """mg_poisson_solve in the library's static workspace (no device allocation);
    returns (status, stats dict)."""
    o = make_opts(**opts)
    st = NpMgStats()
    s = lib.mg_poisson_solve_noalloc(_dims(rhs), h, bc, _dev(rhs), _dev(x), tol, ctypes.byref(o),
                                     ctypes.byref(st))
    if check:
        _check("mg_poisson_solve_noalloc", s)
    return s, st.as_dict()


def mg_poisson_solve_batched(rhs, x, h, bc=BC_DIRICHLET0, tol=1e-10, check=True, **opts):
    """Solves rhs[p] -> x[p] for every p (lists of 2D CUDA tensors); returns
    (status, list of stats dicts)."""
    n = len(rhs)
    if len(x) != n or len(h) != n:
        raise ValueError("rhs, x and h must have the same length")
    dims = (NpDims * n)(*[_dims(t) for t in rhs])
    hs = (ctypes.c_double * n)(*h)
    rp = (ctypes.c_void_p * n)(*[_dev(t).value for t in rhs])
    xp = (ctypes.c_void_p * n)(*[_dev(t).value for t in x])
    o = make_opts(**opts)
    st = (NpMgStats * n)()
    s = lib.mg_poisson_solve_batched(n, dims, hs, bc, ctypes.cast(rp, ctypes.c_void_p),
                                     ctypes.cast(xp, ctypes.c_void_p), tol, ctypes.byref(o), st)
    if check:
        _check("mg_poisson_solve_batched", s)
    return s, [st[i].as_dict() for i in range(n)]


def np_last_autotune():
    inner = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    lib.np_last_autotune(ctypes.byref(inner), ctypes.byref(ms))
    return inner.value, ms.value


BATCHED_SOURCES = {0: "caller", 1: "tuned", 2: "process cache", 3: "file cache"}


def np_last_batched_settings():
    """Settings of this thread's last batched solve: dict(inner_cycles, nu1, nu2,
    row_marching, workgroups, source) with source one of BATCHED_SOURCES."""
    v = [ctypes.c_int(0) for _ in range(6)]
    lib.np_last_batched_settings(*[ctypes.byref(x) for x in v])
    names = ("inner_cycles", "nu1", "nu2", "row_marching", "workgroups", "source")
    out = {k: x.value for k, x in zip(names, v)}
    out["source"] = BATCHED_SOURCES[out["source"]]
    return out


def ns_projection_step(u, v, w, p, h, dt, nu, bc=BC_PERIODIC, tol=1e-10, check=True, **opts):
    o = make_opts(**opts)
    st = NpMgStats()
    s = lib.ns_projection_step(_dims(p), h, _dev(u), _dev(v), _dev(w), _dev(p), dt, nu, bc, tol,
                               ctypes.byref(o), ctypes.byref(st))
    if check:
        _check("ns_projection_step", s)
    return s, st.as_dict()


def ns_collocated_step(u, v, w, p, h, dt, nu, scheme=2, tol=1e-10, check=True, **opts):
    """Collocated projection step with the paper's filter families, in place; returns
    (status, stats dict)."""
    o = make_opts(**opts)
    st = NpMgStats()
    s = lib.ns_collocated_step(_dims(p), h, _dev(u), _dev(v), _dev(w), _dev(p), dt, nu, scheme, tol,
                               ctypes.byref(o), ctypes.byref(st))
    if check:
        _check("ns_collocated_step", s)
    return s, st.as_dict()


def np_nsc_divergence(u, v, w, div, h, scheme=2):
    """div = D.q with the collocated step's first-derivative filter (periodic)."""
    _check("np_nsc_divergence", lib.np_nsc_divergence(_dims(u), h, _dev(u), _dev(v), _dev(w), scheme, _dev(div),
                                                      _stream()))


def ns_projection_step_io(u, v, w, p, h, dt, nu, rhs_out=None, dp_out=None, bc=BC_PERIODIC, tol=1e-10,
                          check=True, **opts):
    """Projection step that also returns (into rhs_out, dp_out) the pressure-correction
    right-hand side and increment it solved for."""
    o = make_opts(**opts)
    st = NpMgStats()
    s = lib.ns_projection_step_io(_dims(p), h, _dev(u), _dev(v), _dev(w), _dev(p), dt, nu, bc, tol,
                                  ctypes.byref(o), ctypes.byref(st), _dev(rhs_out), _dev(dp_out))
    if check:
        _check("ns_projection_step_io", s)
    return s, st.as_dict()


class Cnn:
    """Handle of a learned warm-start network (np_cnn_*)."""

    def __init__(self, n_in=None, levels=None, path=None):
        self.h = ctypes.c_void_p(None)
        if path is not None:
            import struct
            with open(path, "rb") as fp:
                head = fp.read(15)
            levels, n_in = struct.unpack("<ii", head[7:15])
            _check("np_cnn_open", lib.np_cnn_open(path.encode(), ctypes.byref(self.h)))
        else:
            _check("np_cnn_create", lib.np_cnn_create(n_in, levels, ctypes.byref(self.h)))
        self.n_in, self.levels = n_in, levels
        self.n = lib.np_cnn_num_params(self.h)

    def close(self):
        if self.h:
            lib.np_cnn_destroy(self.h)
            self.h = ctypes.c_void_p(None)

    def set_params(self, vec):
        import numpy as np
        a = np.ascontiguousarray(vec, dtype=np.float32)
        _check("np_cnn_set_params", lib.np_cnn_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size))

    def get_params(self):
        import numpy as np
        a = np.empty(self.n, dtype=np.float32)
        _check("np_cnn_get_params", lib.np_cnn_get_params(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size))
        return a

    def get_grads(self):
        import numpy as np
        a = np.empty(self.n, dtype=np.float32)
        _check("np_cnn_get_grads", lib.np_cnn_get_grads(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size))
        return a

    def forward(self, x, y):
        _check("np_cnn_forward", lib.np_cnn_forward(self.h, _dev(x, torch.float32), _dev(y, torch.float32),
                                                    _stream()))

    def _ptrs(self, ts):
        arr = (ctypes.c_void_p * len(ts))(*[_dev(t, torch.float32).value for t in ts])
        return arr

    def gradients(self, xs, ts):
        loss = ctypes.c_double(0.0)
        a, b = self._ptrs(xs), self._ptrs(ts)
        _check("np_cnn_gradients", lib.np_cnn_gradients(self.h, len(xs), ctypes.cast(a, ctypes.c_void_p),
                                                        ctypes.cast(b, ctypes.c_void_p), ctypes.byref(loss),
                                                        _stream()))
        return loss.value

    def train_step(self, xs, ts, lr):
        loss = ctypes.c_double(0.0)
        a, b = self._ptrs(xs), self._ptrs(ts)
        _check("np_cnn_train_step", lib.np_cnn_train_step(self.h, len(xs), ctypes.cast(a, ctypes.c_void_p),
                                                          ctypes.cast(b, ctypes.c_void_p), lr,
                                                          ctypes.byref(loss), _stream()))
        return loss.value

    def prepare(self, f, p, x_in, target):
        sc = ctypes.c_double(0.0)
        _check("np_cnn_prepare", lib.np_cnn_prepare(self.h, _dims(f), _dev(f), _dev(p), _dev(x_in, torch.float32),
                                                    _dev(target, torch.float32) if target is not None else None,
                                                    ctypes.byref(sc), _stream()))
        return sc.value

    def attach(self):
        lib.np_cnn_attach(self.h)

    @staticmethod
    def detach():
        lib.np_cnn_attach(None)

    def save(self, path):
        _check("np_cnn_save", lib.np_cnn_save(self.h, path.encode()))

    def init(self, seed=0):
        _check("np_cnn_init", lib.np_cnn_init(self.h, ctypes.c_uint64(seed)))


def np_cnn_load(path):
    """Loads a weight file into a library-owned network used by warm_start=1
    (None detaches it)."""
    _check("np_cnn_load", lib.np_cnn_load(path.encode() if path is not None else None))


def np_cnn_train(rhs, p, weights_out, cfg=None, bc=BC_PERIODIC):
    """Trains a network on device FP64 (rhs, p) pairs (lists of 3D tensors) and
    writes it to weights_out; returns the per-epoch mean loss."""
    import json
    n = len(rhs)
    if len(p) != n:
        raise ValueError("rhs and p must have the same length")
    cfg = dict(cfg or {})
    js = json.dumps(cfg)
    dims = (NpDims * n)(*[_dims(t) for t in rhs])
    rp = (ctypes.c_void_p * n)(*[_dev(t).value for t in rhs])
    pp = (ctypes.c_void_p * n)(*[_dev(t).value for t in p])
    epochs = int(cfg.get("epochs", 10))
    hist = (ctypes.c_double * max(epochs, 1))()
    _check("np_cnn_train", lib.np_cnn_train(dims, bc, n, ctypes.cast(rp, ctypes.c_void_p),
                                            ctypes.cast(pp, ctypes.c_void_p), js.encode(),
                                            weights_out.encode(), hist))
    return list(hist)[:epochs]


BC_NEUMANN = 2
SCHEME_CENTRAL, SCHEME_UPWIND, SCHEME_FE = 0, 1, 2


def np_ad_explicit_step(T, h, dt, nu, bc, a=None, scheme=SCHEME_CENTRAL):
    """One predictor-corrector advection-diffusion step in place, with the chosen filter
    family (central, upwind, finite element); a: list of collocated velocity tensors."""
    ap = None
    if a is not None:
        ap = (ctypes.c_void_p * 3)(*[_dev(c).value for c in a] + [None] * (3 - len(a)))
    o = make_opts()
    _check("np_ad_explicit_step", lib.np_ad_explicit_step(_dims(T), h, _dev(T),
                                                          ctypes.cast(ap, ctypes.c_void_p) if ap else None, dt,
                                                          nu, bc, scheme, ctypes.byref(o)))


def np_ad_scalar_step(T, h, dt, nu, bc, a=None):
    arr = None
    if a is not None:
        arr = (ctypes.c_void_p * 3)(*[_dev(c).value for c in a] + [None] * (3 - len(a)))
    o = make_opts()
    s = lib.np_ad_scalar_step(_dims(T), h, _dev(T), ctypes.cast(arr, ctypes.c_void_p) if arr else None,
                              dt, nu, bc, ctypes.byref(o))
    _check("np_ad_scalar_step", s)


def np_ad_implicit_solve(rhs, x, h, bc, op, tol=1e-10, check=True, l1=False, **opts):
    """Solves the backward-Euler advection-diffusion system A x = rhs in place in x
    (op from ad_op); returns (status, stats dict), with stats["l1_change"] the
    per-cycle L1 change of the iterate when l1 is set."""
    o = make_opts(**opts)
    st = NpMgStats()
    buf = (ctypes.c_double * 256)() if l1 else None
    s = lib.np_ad_implicit_solve(_dims(rhs), h, bc, ctypes.byref(op), _dev(rhs), _dev(x), tol, ctypes.byref(o),
                                 ctypes.byref(st), buf)
    if check:
        _check("np_ad_implicit_solve", s)
    d = st.as_dict()
    if l1:
        d["l1_change"] = list(buf[:min(256, st.cycles)])
    return s, d


def np_ad_apply(x, y, h, bc, op):
    _check("np_ad_apply", lib.np_ad_apply(_dims(x), h, bc, ctypes.byref(op), _dev(x), _dev(y), _stream()))


def np_ad_prof_level(kind, f, x, y, h, bc, op, reps=50):
    """Average duration (ms) of `reps` back-to-back launches of the advection-diffusion
    solver's level kernel `kind` (PROF_LEVEL_SWEEP/RESTRICT/PROLONG) on this grid."""
    out = ctypes.c_double(0.0)
    _check("np_ad_prof_level", lib.np_ad_prof_level(_dims(x), h, bc, ctypes.byref(op), kind,
                                                    _dev(f) if f is not None else None, _dev(x), _dev(y), reps,
                                                    _stream(), ctypes.byref(out)))
    return out.value


def np_op_apply(x, y, h, bc):
    _check("np_op_apply", lib.np_op_apply(_dims(x), h, bc, _dev(x), _dev(y), _stream()))


def np_op_jacobi(f, x_in, x_out, h, bc, omega=2.0 / 3.0):
    _check("np_op_jacobi", lib.np_op_jacobi(_dims(x_in), h, bc, omega, _dev(f), _dev(x_in),
                                            _dev(x_out), _stream()))


def np_op_resid_restrict(f, x, fc, h, bc):
    _check("np_op_resid_restrict", lib.np_op_resid_restrict(_dims(x), h, bc, _dev(f), _dev(x),
                                                            _dev(fc), _stream()))


def np_op_prolong_add(ec, x, bc):
    _check("np_op_prolong_add", lib.np_op_prolong_add(_dims(x), bc, _dev(ec), _dev(x), _stream()))


def np_op_vcycle(f, x, h, bc, **opts):
    o = make_opts(**opts)
    _check("np_op_vcycle", lib.np_op_vcycle(_dims(x), h, bc, _dev(f), _dev(x), ctypes.byref(o)))


def np_op_resid_norm(f, x, h, bc):
    out = ctypes.c_double(0.0)
    _check("np_op_resid_norm", lib.np_op_resid_norm(_dims(x), h, bc, _dev(f), _dev(x),
                                                    ctypes.byref(out), _stream()))
    return out.value


PROF_DOWN, PROF_DOWN_ZERO, PROF_UP, PROF_JACOBI = 1, 2, 4, 8
PROF_RESTRICT, PROF_PROLONG, PROF_REFINE, PROF_SWEEP_ZERO = 16, 32, 64, 128


def np_prof_enable(mask):
    lib.np_prof_enable(int(mask))


def np_set_tuning(key, value):
    _check("np_set_tuning", lib.np_set_tuning(key.encode(), int(value)))


def np_get_tuning(key):
    return lib.np_get_tuning(key.encode())


def np_prof_read():
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    _check("np_prof_read", lib.np_prof_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def np_release_all():
    lib.np_release_all()


PROF_LEVEL_SWEEP, PROF_LEVEL_RESTRICT, PROF_LEVEL_PROLONG = 0, 1, 2


LEVEL_ZERO2, LEVEL_RESTRICT, LEVEL_DOWN0, LEVEL_PSWEEP_SWEEP, LEVEL_UP2, LEVEL_UP2Z, LEVEL_SWEEP2Z, LEVEL_DOWN0Z, LEVEL_DOWN2Z = range(9)


def np_op_level(kind, f, x, xout, c, h, bc, prec):
    """One 3D level step (np_op_level kind LEVEL_*) on tensors of the precision
    (float64, float32, or int16 holding BF16 bit patterns); xout / c may be None
    where the kind does not use them."""
    dt = {FP64: torch.float64, FP32: torch.float32, BF16: torch.int16}[prec]
    _check("np_op_level", lib.np_op_level(_dims(x), h, bc, prec, kind, _dev(f, dt), _dev(x, dt),
                                          _dev(xout, dt) if xout is not None else None,
                                          _dev(c, dt) if c is not None else None, _stream()))


def np_prof_level(kind, f, x, y, h, bc, prec, reps=50):
    """Mean duration (ms) of `reps` back-to-back launches of a solver level kernel on
    the current stream: kind 0 y = sweep(x), 1 y = R (f - A x) (y coarse), 2 x += P y
    (y coarse; f may be None).  Tensors of the precision: float64, float32, or int16
    holding BF16 bit patterns."""
    dt = {FP64: torch.float64, FP32: torch.float32, BF16: torch.int16}[prec]
    out = ctypes.c_double(0.0)
    _check("np_prof_level", lib.np_prof_level(_dims(x), h, bc, prec, kind, _dev(f, dt) if f is not None else None,
                                              _dev(x, dt), _dev(y, dt), reps, _stream(), ctypes.byref(out)))
    return out.value
