"""Host-side checks of the C ABI: the library loads and exports every symbol the
header declares (no GPU needed, nothing is computed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "neuphys.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for", "while", "return")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("mg_poisson_solve", "ns_projection_step", "mg_poisson_solve_batched", "np_cnn_train",
              "np_cnn_load", "np_ad_scalar_step", "np_last_error", "np_release_all", "np_default_opts"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2402_17913_amd", "libneuphys.so")
    if not os.path.exists(path):
        import sys
        sys.path.insert(0, ROOT)
        from paper_2402_17913_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_opts_and_last_error_without_gpu():
    path = os.path.join(ROOT, "paper_2402_17913_amd", "libneuphys.so")
    import sys
    sys.path.insert(0, ROOT)
    lib = ctypes.CDLL(path)
    from paper_2402_17913_amd.binding import NpMgOpts  # the one mirror of np_mg_opts
    o = NpMgOpts()
    lib.np_default_opts(ctypes.byref(o))
    assert (o.nu1, o.nu2, o.max_cycles) == (2, 2, 200) and abs(o.omega - 2 / 3) < 1e-15
    assert (o.warm_start, o.cycle, o.prolong) == (0, 0, 0)
    lib.np_last_error.restype = ctypes.c_char_p
    assert lib.np_last_error() == b""


def test_cnn_train_rejects_bad_configuration():
    """Argument and configuration errors are reported before any device work."""
    import ctypes
    from paper_2402_17913_amd import binding as B
    dims = (B.NpDims * 1)(B.NpDims(3, (ctypes.c_int64 * 3)(32, 32, 32)))
    fake = (ctypes.c_void_p * 1)(ctypes.c_void_p(16))
    for cfg, bc in ((b'{"n_in": 16, "depth": 2}', B.BC_PERIODIC), (b'{"n_in": 16', B.BC_PERIODIC),
                    (b'[1]', B.BC_PERIODIC), (b'{"epochs": 0}', B.BC_PERIODIC), (b'{}', B.BC_DIRICHLET0)):
        st = B.lib.np_cnn_train(dims, bc, 1, ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                                cfg, b"/nonexistent/w.npcnn", None)
        assert st == B.NP_EINVAL, cfg
        assert B.lib.np_last_error() not in (None, b"")
