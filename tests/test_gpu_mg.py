"""GPU parity of the multigrid path against the FP64 oracle (run on an MI355X).

FP64 bar: relative difference max|gpu - oracle| / max|oracle| <= 1e-12 for the
same number of cycles (operators alone: <= 1e-13).  Mixed precision and
tolerance-stopped solves are judged by the oracle's own residual evaluator.
"""
import numpy as np
import pytest

from paper_2402_17913_amd import inputs

pytestmark = pytest.mark.gpu
DIR, PER = 0, 1


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_17913_amd import binding
    return binding


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def say(*a):
    print(*a, flush=True)


SHAPES = [(2, 4), (2, 8), (2, 64), (2, 256), (3, 4), (3, 8), (3, 32), (3, 64)]


# ------------------------------------------------------------- single operators
@pytest.mark.parametrize("d,n", SHAPES)
@pytest.mark.parametrize("bc", [DIR, PER])
def test_apply_and_jacobi(B, orc, d, n, bc):
    say("apply/jacobi", d, n, bc)
    rng = np.random.default_rng(100 + n * d + bc)
    h = 1.0 / n
    x, f = rng.standard_normal((n,) * d), rng.standard_normal((n,) * d)
    y = dev(np.zeros_like(x))
    B.np_op_apply(dev(x), y, h, bc)
    assert rel(host(y), orc.apply_A(x, h, bc)) < 1e-13
    xo = dev(np.zeros_like(x))
    B.np_op_jacobi(dev(f), dev(x), xo, h, bc)
    assert rel(host(xo), orc.jacobi(f, x, h, bc)) < 1e-13


@pytest.mark.parametrize("d,n", [s for s in SHAPES if s[1] >= 8])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_restrict_and_prolong(B, orc, d, n, bc):
    say("restrict/prolong", d, n, bc)
    rng = np.random.default_rng(200 + n * d + bc)
    h = 1.0 / n
    x, f = rng.standard_normal((n,) * d), rng.standard_normal((n,) * d)
    fc = dev(np.zeros((n // 2,) * d))
    B.np_op_resid_restrict(dev(f), dev(x), fc, h, bc)
    assert rel(host(fc), orc.restrict(orc.residual(f, x, h, bc))) < 1e-13
    ec = rng.standard_normal((n // 2,) * d)
    xg = dev(x)
    B.np_op_prolong_add(dev(ec), xg, bc)
    assert rel(host(xg), orc.prolong_add(ec, x, bc)) < 1e-14


@pytest.mark.parametrize("d,n", [(2, 4), (2, 16), (2, 128), (2, 512), (3, 4), (3, 16), (3, 32),
                                 (3, 64), (3, 128)])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_one_vcycle(B, orc, d, n, bc):
    say("vcycle", d, n, bc)
    rng = np.random.default_rng(300 + n * d + bc)
    h = 1.0 / n
    x, f = rng.standard_normal((n,) * d), rng.standard_normal((n,) * d)
    if bc == PER:
        f -= f.mean()
    xg = dev(x)
    B.np_op_vcycle(dev(f), xg, h, bc)
    assert rel(host(xg), orc.vcycle(f, x, h, bc)) < 1e-12


@pytest.mark.parametrize("knobs", [dict(fused=1), dict(graphs=0), dict(fused=1, bz3=2, bz2=2),
                                   dict(fused=1, fmin2=4, fmin3=4), dict(tail=0), dict(fused=1, tail=0),
                                   dict(zero2=0), dict(sweep3=0, zero2=0), dict(fused=1, fmax2=64, fmax3=32)])
def test_kernel_variants_agree(B, orc, knobs):
    """Fused level kernels (also with the smallest marching chunks, down to 4^d, and
    on a range of levels only), direct launches, the per-level kernels without the
    one-workgroup tail, separate sweeps from a zero iterate and the direct 3D
    kernels all give the oracle's cycles."""
    old = {k: B.np_get_tuning(k) for k in knobs}
    try:
        for k, v in knobs.items():
            B.np_set_tuning(k, v)
        for d, n, bc in [(2, 64, DIR), (2, 256, PER), (3, 32, PER), (3, 64, DIR), (3, 128, PER)]:
            say("variant", knobs, d, n, bc)
            rng = np.random.default_rng(n + d)
            h = 1.0 / n
            x, f = rng.standard_normal((n,) * d), rng.standard_normal((n,) * d)
            if bc == PER:
                f -= f.mean()
            xg = dev(x)
            B.np_op_vcycle(dev(f), xg, h, bc)
            assert rel(host(xg), orc.vcycle(f, x, h, bc)) < 1e-12
            ref = orc.mg_solve(f, h, bc, fixed_cycles=3)
            xg = dev(np.zeros_like(f))
            st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, fixed_cycles=3)
            assert stats["cycles"] == 3 and rel(host(xg), ref.x) < 1e-12
    finally:
        for k, v in old.items():
            B.np_set_tuning(k, v)


@pytest.mark.parametrize("bc", [DIR, PER])
def test_sweep3_matches_direct_sweep(B, orc, bc):
    """The z-marching 3D sweep (levels of n >= 128) and the direct sweep give the
    same solves on every precision path (FP64 to 1e-13 after fixed cycles, the
    mixed paths to their rounding with the same cycle counts), and the FP64 result
    matches the oracle."""
    n = 128
    rng = np.random.default_rng(77 + bc)
    f = rng.standard_normal((n, n, n))
    if bc == PER:
        f -= f.mean()
    h = 1.0 / n
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("sweep3", v)
            for prec in (B.FP64, B.FP32, B.BF16):
                say("sweep3", v, bc, prec)
                xg = dev(np.zeros_like(f))
                kw = dict(fixed_cycles=4) if prec == B.FP64 else {}
                st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, smooth_prec=prec, **kw)
                out[(v, prec)] = (host(xg), stats)
    finally:
        B.np_set_tuning("sweep3", 1)
    ref = orc.mg_solve(f, h, bc, fixed_cycles=4)
    assert rel(out[(1, B.FP64)][0], ref.x) < 1e-12
    assert rel(out[(1, B.FP64)][0], out[(0, B.FP64)][0]) < 1e-13
    for prec in (B.FP32, B.BF16):
        a, sa = out[(1, prec)]
        b, sb = out[(0, prec)]
        assert sa["cycles"] == sb["cycles"] and sa["outer_iters"] == sb["outer_iters"]
        assert orc.rel_res(f, a, h, bc) <= 1e-10
        assert rel(a, b) < 1e-8


@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("nu2", [2, 1])
@pytest.mark.parametrize("d,n", [(3, 128), (2, 512)])
def test_prolong_sweep_fusion_bit_identical(B, orc, bc, nu2, d, n):
    """Prolongation + correction and the first post-sweep in one kernel (3D: z-marching,
    levels 128^3, 64^3, 32^3; 2D: per cell, every level above the tail) give the solves
    of the two-kernel path bit for bit, on every precision path, with one and two
    post-sweeps; the FP64 result matches the oracle."""
    rng = np.random.default_rng(131 + bc + d)
    f = rng.standard_normal((n,) * d)
    if bc == PER:
        f -= f.mean()
    h = 1.0 / n
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("psweep", v)
            for prec in (B.FP64, B.FP32, B.BF16):
                say("psweep", v, d, n, bc, nu2, prec)
                xg = dev(np.zeros_like(f))
                kw = dict(fixed_cycles=3) if prec == B.FP64 else {}
                st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, smooth_prec=prec, nu1=2, nu2=nu2, **kw)
                out[(v, prec)] = (host(xg), stats)
    finally:
        B.np_set_tuning("psweep", 1)
    for prec in (B.FP64, B.FP32, B.BF16):
        a, sa = out[(1, prec)]
        b, sb = out[(0, prec)]
        assert sa["cycles"] == sb["cycles"], prec
        assert np.array_equal(a, b), (prec, rel(a, b))
    ref = orc.mg_solve(f, h, bc, fixed_cycles=3, nu1=2, nu2=nu2)
    assert rel(out[(1, B.FP64)][0], ref.x) < 1e-12


@pytest.mark.parametrize("bc", [DIR, PER])
def test_refinement_two_cells_per_thread_bit_identical(B, orc, bc):
    """The 3D refinement step with two cells per thread (16-byte FP64 accesses) gives
    the one-cell form's mixed-precision solves bit for bit, with the same cycle and
    refinement counts, and they meet the tolerance by the oracle's residual."""
    n = 128
    rng = np.random.default_rng(171 + bc)
    f = rng.standard_normal((n, n, n))
    if bc == PER:
        f -= f.mean()
    h = 1.0 / n
    out = {}
    try:
        for v in (1, 2):
            B.np_set_tuning("ir_cpt", v)
            for prec in (B.FP32, B.BF16):
                say("ir_cpt", v, bc, prec)
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, smooth_prec=prec)
                out[(v, prec)] = (host(xg), stats["cycles"], stats["outer_iters"])
    finally:
        B.np_set_tuning("ir_cpt", 2)
    for prec in (B.FP32, B.BF16):
        a, b = out[(1, prec)], out[(2, prec)]
        assert a[1:] == b[1:], prec
        assert np.array_equal(a[0], b[0]), prec
        assert orc.rel_res(f, b[0], h, bc) <= 1e-10


@pytest.mark.parametrize("bc", [DIR, PER])
def test_mixed_zero_start_reads_no_iterate(B, orc, bc):
    """A 3D mixed solve from a zero guess (z-marching levels) never reads the caller's x:
    its first residual is f, rounded in the norm's pass, and its first update writes
    x = 0 + e.  From an x full of NaNs it gives the solve of the path that zeroes x first
    (the one-cell refinement kernel) bit for bit, with the same counts; a solve stopped
    before any cycle (max_cycles 0, or tol >= 1) returns the zero iterate."""
    n = 128
    rng = np.random.default_rng(613 + bc)
    f = rng.standard_normal((n, n, n))
    if bc == PER:
        f -= f.mean()
    h = 1.0 / n
    nan = np.full_like(f, np.nan)
    out = {}
    try:
        for v in (1, 2):
            B.np_set_tuning("ir_cpt", v)
            for prec in (B.FP32, B.BF16):
                say("zero start", v, bc, prec)
                xg = dev(nan)
                st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, smooth_prec=prec)
                out[(v, prec)] = (host(xg), stats["cycles"], stats["outer_iters"])
    finally:
        B.np_set_tuning("ir_cpt", 2)
    for prec in (B.FP32, B.BF16):
        a, b = out[(1, prec)], out[(2, prec)]
        assert a[1:] == b[1:], prec
        assert np.array_equal(a[0], b[0]), prec
        assert orc.rel_res(f, b[0], h, bc) <= 1e-10
        for kw in (dict(max_cycles=0), dict(tol=1.0)):
            xg = dev(nan)
            B.mg_poisson_solve(dev(f), xg, h, bc, smooth_prec=prec, check=False, **kw)
            assert np.array_equal(host(xg), np.zeros_like(f)), (prec, kw)


@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("n", [128, 256, 1024])
def test_blk2_same_solves(B, orc, bc, n):
    """2D levels of 128^2 .. 1024^2 on one block kernel per leg (knob blk2) against the
    per-cell kernels: FP64 fixed cycles and FP64, FP32- and BF16-mixed solves to the
    tolerance give the same iterates bit for bit in the same cycles, within 1e-12 of the
    oracle's V-cycles (FP64) and meeting the tolerance by its residual."""
    rng = np.random.default_rng(701 + n + bc)
    f = rng.standard_normal((n, n))
    if bc == PER:
        f -= f.mean()
    h = 1.0 / n
    fg = dev(f)
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("blk2", v)
            say("blk2", v, n, bc)
            xg = dev(np.zeros_like(f))
            B.mg_poisson_solve(fg, xg, h, bc, fixed_cycles=3)
            out[(v, "fixed")] = host(xg)
            for p in (B.FP64, B.FP32, B.BF16):
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(fg, xg, h, bc, smooth_prec=p)
                out[(v, p)] = (host(xg), stats["cycles"])
    finally:
        B.np_set_tuning("blk2", 1)
    assert np.array_equal(out[(1, "fixed")], out[(0, "fixed")])
    for p in (B.FP64, B.FP32, B.BF16):
        assert out[(1, p)][1] == out[(0, p)][1], p
        assert np.array_equal(out[(1, p)][0], out[(0, p)][0]), p
        assert orc.rel_res(f, out[(1, p)][0], h, bc) <= 1e-10
    if n <= 256:
        ref = orc.mg_solve(f, h, bc, fixed_cycles=3)
        assert rel(out[(1, "fixed")], ref.x) < 1e-12


@pytest.mark.parametrize("knob,on,off", [("greps", 8, 1), ("tailck", 1, 0), ("zbar", 1, 2), ("d2cpt", 2, 1)])
@pytest.mark.parametrize("shape", [(128, 128), (64, 64, 64), (256, 256, 256)])
def test_launch_grouping_same_solves(B, orc, shape, knob, on, off):
    """Cycles replayed as graphs of up to 8 (knob greps) against one graph per cycle, the
    convergence check run by the one-workgroup tail kernel (knob tailck) against its own
    launch, the 3D zero-start down-leg pass with one barrier per plane step (knob zbar)
    against two, and the FP64 nonzero down-leg pass on two cells per thread (knob d2cpt)
    against one: FP64 solves to the tolerance and for fixed cycles, FP32- and BF16-mixed
    solves from a zero and from a nonzero guess, the sawtooth cycle and the
    advection-diffusion V-cycle give the same iterates and histories bit for bit; the
    tolerance-stopped results meet the tolerance by the oracle's residual."""
    n, d = shape[0], len(shape)
    bc = DIR if d == 3 else PER
    rng = np.random.default_rng(811 + n + d)
    f = rng.standard_normal(shape)
    if bc == PER:
        f -= f.mean()
    x0 = 1e-3 * rng.standard_normal(shape)
    h = 1.0 / n
    fg = dev(f)
    op = B.ad_op(1.0, 0.1, [1.0] * d, 0)
    out = {}

    def run(tag, fn, start):
        xg = dev(start)
        _, stats = fn(xg)
        out[tag] = (host(xg), stats["cycles"], stats["outer_iters"], stats["hist"])

    prev = B.np_get_tuning(knob)
    try:
        for v in (on, off):
            B.np_set_tuning(knob, v)
            say(knob, v, shape, bc)
            z = np.zeros_like(f)
            run((v, "fixed"), lambda xg: B.mg_poisson_solve(fg, xg, h, bc, fixed_cycles=11), z)
            run((v, "saw"), lambda xg: B.mg_poisson_solve(fg, xg, h, bc, cycle=B.CYCLE_SAWTOOTH, nu1=0,
                                                          fixed_cycles=6), z)
            run((v, "ad"), lambda xg: B.np_ad_implicit_solve(fg, xg, 1.0, bc, op), z)
            for p in (B.FP64, B.FP32, B.BF16):
                run((v, p, 0), lambda xg: B.mg_poisson_solve(fg, xg, h, bc, smooth_prec=p), z)
                run((v, p, 2), lambda xg: B.mg_poisson_solve(fg, xg, h, bc, smooth_prec=p, warm_start=2), x0)
    finally:
        B.np_set_tuning(knob, prev)
    for k in [key for key in out if key[0] == on]:
        a, b = out[k], out[(off,) + k[1:]]
        assert np.array_equal(a[0], b[0]), k
        assert a[1:3] == b[1:3], k
        if knob == "d2cpt":
            # other tiles: the check's partial sums group the residual differently, to rounding
            assert np.allclose(a[3], b[3], rtol=1e-12, atol=0.0), k
        else:
            assert a[3] == b[3], k
        if len(k) == 3:
            assert orc.rel_res(f, a[0], h, bc) <= 1e-10, k


@pytest.mark.parametrize("bc", [DIR, PER])
def test_prof_level_runs_the_solver_kernels(B, orc, bc):
    """The timing hook launches the solver's level kernels (FP64, 128^3, the z-marching
    kernels): the sweep's output is one oracle Jacobi sweep, the restriction's is the
    oracle's restricted residual, and reps + 1 prolongations add reps + 1 times the
    oracle's P y; every call reports a positive duration."""
    n = 128
    rng = np.random.default_rng(5 + bc)
    f, x = rng.standard_normal((n, n, n)), rng.standard_normal((n, n, n))
    yc = rng.standard_normal((n // 2,) * 3)
    h = 1.0 / n
    y = dev(np.zeros_like(x))
    assert B.np_prof_level(B.PROF_LEVEL_SWEEP, dev(f), dev(x), y, h, bc, B.FP64, reps=3) > 0
    assert rel(host(y), orc.jacobi(f, x, h, bc)) < 1e-13
    c = dev(np.zeros_like(yc))
    assert B.np_prof_level(B.PROF_LEVEL_RESTRICT, dev(f), dev(x), c, h, bc, B.FP64, reps=3) > 0
    assert rel(host(c), orc.restrict(orc.residual(f, x, h, bc))) < 1e-13
    xg = dev(x)
    assert B.np_prof_level(B.PROF_LEVEL_PROLONG, None, xg, dev(yc), h, bc, B.FP64, reps=3) > 0
    ref = x + 4 * (orc.prolong_add(yc, np.zeros_like(x), bc))
    assert rel(host(xg), ref) < 1e-13


@pytest.mark.parametrize("bc", [DIR, PER])
def test_bf16_pair_kernels(B, orc, bc):
    """BF16 storage on the z-marching kernels (two cells per thread): the sweep equals
    the direct sweep bit for bit; restriction and prolongation match the FP64 oracle on
    the BF16-rounded inputs to BF16 rounding of their terms."""
    import torch
    n = 128
    h = 1.0 / n
    rng = np.random.default_rng(21 + bc)

    def b16(a):
        return torch.from_numpy(a).to(torch.bfloat16).cuda()

    def val(t):
        return t.float().cpu().numpy().astype(np.float64)

    f, x = b16(rng.standard_normal((n, n, n))), b16(rng.standard_normal((n, n, n)))
    yc = b16(rng.standard_normal((n // 2,) * 3))
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("sweep3", v)
            y = torch.zeros_like(x)
            B.np_prof_level(B.PROF_LEVEL_SWEEP, f.view(torch.int16), x.view(torch.int16), y.view(torch.int16), h, bc,
                            B.BF16, reps=1)
            c = torch.zeros_like(yc)
            B.np_prof_level(B.PROF_LEVEL_RESTRICT, f.view(torch.int16), x.view(torch.int16), c.view(torch.int16), h,
                            bc, B.BF16, reps=1)
            xp = x.clone()
            B.np_prof_level(B.PROF_LEVEL_PROLONG, None, xp.view(torch.int16), yc.view(torch.int16), h, bc, B.BF16,
                            reps=1)
            out[v] = (val(y), val(c), val(xp))
    finally:
        B.np_set_tuning("sweep3", 1)
    fv, xv, ycv = val(f), val(x), val(yc)
    assert np.array_equal(out[1][0], out[0][0])
    scale = np.max(np.abs(fv)) + 12 * np.max(np.abs(xv)) / h ** 2
    ref_c = orc.restrict(orc.residual(fv, xv, h, bc))
    ref_p = xv + 2 * orc.prolong_add(ycv, np.zeros_like(xv), bc)  # warm-up launch + one timed launch
    for v in (1, 0):
        assert np.max(np.abs(out[v][1] - ref_c)) <= 8e-3 * scale
        assert np.max(np.abs(out[v][2] - ref_p)) <= 8e-3 * (np.max(np.abs(xv)) + 2 * np.max(np.abs(ycv)))


def test_tuning_knobs_validate(B):
    with pytest.raises(B.NeuphysError):
        B.np_set_tuning("no_such_knob", 1)
    with pytest.raises(B.NeuphysError):
        B.np_set_tuning("bz3", 3)
    for key, bad in (("zc3", 3), ("zc3", 1), ("conv3z", 6), ("conv3z", 128), ("ir_cpt", 0), ("ir_cpt", 3)):
        with pytest.raises(B.NeuphysError):
            B.np_set_tuning(key, bad)
    assert B.np_get_tuning("fused") == 0 and B.np_get_tuning("tail") == 1
    assert B.np_get_tuning("conv3z") == 1 and B.np_get_tuning("zc3") == 0


def test_resid_norm(B, orc):
    rng = np.random.default_rng(5)
    x, f = rng.standard_normal((64, 64, 64)), rng.standard_normal((64, 64, 64))
    got = B.np_op_resid_norm(dev(f), dev(x), 1 / 64, DIR)
    ref = np.linalg.norm(orc.residual(f, x, 1 / 64, DIR))
    assert abs(got - ref) / ref < 1e-13


# ----------------------------------------------------------------- full solves
def _parity_solve(B, orc, f, h, bc, tol=1e-10):
    ref = orc.mg_solve(f, h, bc, tol=tol)
    assert ref.status == 0
    xg = dev(np.zeros_like(f))
    st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, tol=tol, fixed_cycles=ref.cycles)
    assert stats["cycles"] == ref.cycles
    x = host(xg)
    assert rel(x, ref.x) < 1e-12, rel(x, ref.x)
    hist = np.array(stats["hist"])
    # residual norms agree to rounding of ||A x|| (absolute, in units of ||f||)
    assert np.max(np.abs(hist - ref.hist)) < 1e-13
    # tolerance-stopped run: the oracle judges the residual
    xg2 = dev(np.zeros_like(f))
    st, stats2 = B.mg_poisson_solve(dev(f), xg2, h, bc, tol=tol)
    assert abs(stats2["cycles"] - ref.cycles) <= 1
    assert orc.rel_res(f - (f.mean() if bc == PER else 0.0), host(xg2), h, bc) <= tol
    return x, stats


def test_solve_config_2d_128_dirichlet(B, orc):
    """128^2 unit square, zero Dirichlet, manufactured sin.sin + 8 modes source."""
    say("solve C1 128^2")
    g = inputs.manufactured_2d(128, seed=0)
    x, stats = _parity_solve(B, orc, g["f"], g["h"], DIR)
    assert stats["rel_res"] <= 1e-10


@pytest.mark.parametrize("d,n,bc", [(2, 4, DIR), (2, 8, PER), (2, 64, PER), (2, 512, DIR),
                                    (3, 4, DIR), (3, 8, DIR), (3, 16, PER), (3, 64, DIR)])
def test_solve_shapes(B, orc, d, n, bc):
    say("solve", d, n, bc)
    h = 1.0 / n if bc == DIR else 2 * np.pi / n
    f = inputs.sine_rhs(d, n, seed=n + d)["f"] if bc == DIR else \
        np.random.default_rng(n + d).standard_normal((n,) * d)
    _parity_solve(B, orc, f, h, bc)


def test_zero_rhs_and_warm_start(B, orc):
    import torch
    n = 32
    xg = dev(np.ones((n, n)))
    st, stats = B.mg_poisson_solve(dev(np.zeros((n, n))), xg, 1 / n, DIR, warm_start=2)
    assert stats["cycles"] == 0 and torch.all(xg == 0)
    g = inputs.manufactured_2d(n, seed=1)
    ref = orc.mg_solve(g["f"], g["h"], DIR)
    xg = dev(ref.x)
    st, stats = B.mg_poisson_solve(dev(g["f"]), xg, g["h"], DIR, warm_start=2)
    assert stats["cycles"] == 0  # a converged guess needs no cycle
    assert np.all(host(xg) == ref.x)


def test_error_paths(B):
    import torch
    x = torch.zeros((12, 12), dtype=torch.float64, device="cuda")
    x0 = x.clone()
    with pytest.raises(B.NeuphysError) as e:
        B.mg_poisson_solve(x.clone(), x, 1 / 12, DIR)
    assert e.value.status == B.NP_EINVAL and torch.equal(x, x0)
    f = torch.ones((16, 16), dtype=torch.float64, device="cuda")
    f[3, 4] = float("nan")
    xg = torch.zeros_like(f)
    with pytest.raises(B.NeuphysError) as e:
        B.mg_poisson_solve(f, xg, 1 / 16, DIR)
    assert e.value.status == B.NP_ENAN
    f = torch.ones((64, 64), dtype=torch.float64, device="cuda")
    st, stats = B.mg_poisson_solve(f, torch.zeros_like(f), 1 / 64, DIR, max_cycles=1, check=False)
    assert st == B.NP_ENOCONV and stats["cycles"] == 1
    with pytest.raises(B.NeuphysError):
        B.mg_poisson_solve(f, torch.zeros_like(f), -1.0, DIR)


# ----------------------------------------------------------- mixed precision
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d,n,bc", [(2, 128, DIR), (3, 64, DIR), (2, 256, PER), (3, 32, PER)])
def test_mixed_precision_reaches_tolerance(B, orc, prec, d, n, bc):
    say("mixed", prec, d, n, bc)
    h = 1.0 / n if bc == DIR else 2 * np.pi / n
    f = inputs.sine_rhs(d, n, seed=7)["f"] if bc == DIR else \
        np.random.default_rng(n).standard_normal((n,) * d)
    ref = orc.mg_solve(f, h, bc, tol=1e-12)
    xg = dev(np.zeros_like(f))
    p = B.FP32 if prec == "fp32" else B.BF16
    st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, tol=1e-10, smooth_prec=p)
    x = host(xg)
    fm = f - f.mean() if bc == PER else f
    rr = orc.rel_res(fm, x, h, bc)
    say("  outer", stats["outer_iters"], "cycles", stats["cycles"], "rel_res", rr,
        "err vs fp64 oracle", rel(x, ref.x))
    assert rr <= 1e-10
    assert abs(rr - stats["rel_res"]) <= 1e-3 * rr


# --------------------------------------------------------- full size, bench shape
@pytest.mark.slow
def test_full_size_3d_256(B, orc):
    """256^3 Dirichlet with the benchmark's source: one V-cycle from zero is compared
    element by element with the oracle; the converged FP64 and mixed solves are judged
    by the oracle's residual and by the closed-form discrete solution's error bound."""
    say("full size 256^3")
    n = 256
    g = inputs.sine_rhs(3, n, seed=0)
    f, h = g["f"], g["h"]
    xg = dev(np.zeros_like(f))
    fg = dev(f)
    B.np_op_vcycle(fg, xg, h, DIR)
    ref1 = orc.vcycle(f, np.zeros_like(f), h, DIR)
    assert rel(host(xg), ref1) < 1e-12
    lam_min = (12 / h ** 2) * np.sin(np.pi * h / 2) ** 2
    for p in (B.FP64, B.FP32):
        xg = dev(np.zeros_like(f))
        st, stats = B.mg_poisson_solve(fg, xg, h, DIR, tol=1e-10, smooth_prec=p)
        x = host(xg)
        rr = orc.rel_res(f, x, h, DIR)
        say("  prec", p, "cycles", stats["cycles"], "rel_res", rr)
        assert rr <= 1e-10
        x1 = np.sin(np.pi * (np.arange(n) + 0.5) * h)
        uh = np.zeros_like(f)
        for c, ks in g["modes"]:
            lam = (4 / h ** 2) * sum(np.sin(k * np.pi * h / 2) ** 2 for k in ks)
            term = np.array(c / lam)
            for a in reversed(range(3)):
                term = np.multiply.outer(term, np.sin(ks[a] * np.pi * (np.arange(n) + 0.5) * h))
            uh += term
        del x1
        assert np.linalg.norm(x - uh) <= rr * np.linalg.norm(f) / lam_min * (1 + 1e-6) + \
            1e-13 * np.linalg.norm(uh)


def test_full_size_fusion_bit_identical_256(B, orc):
    """The benchmark's 256^3 solve on the BF16-storage path (and plain FP64 for a fixed
    cycle count): the fused prolongation + sweep gives the two-kernel path's iterate bit
    for bit, and the BF16 result meets the tolerance by the oracle's residual."""
    n = 256
    g = inputs.sine_rhs(3, n, seed=0)
    f, h = g["f"], g["h"]
    fg = dev(f)
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("psweep", v)
            for p, kw in ((B.BF16, {}), (B.FP64, dict(fixed_cycles=2))):
                say("full size fusion", v, p)
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(fg, xg, h, DIR, tol=1e-10, smooth_prec=p, **kw)
                out[(v, p)] = (host(xg), stats["cycles"])
    finally:
        B.np_set_tuning("psweep", 1)
    for p in (B.BF16, B.FP64):
        assert out[(1, p)][1] == out[(0, p)][1]
        assert np.array_equal(out[(1, p)][0], out[(0, p)][0]), p
    assert orc.rel_res(f, out[(1, B.BF16)][0], h, DIR) <= 1e-10


# --------------------------------------------- the paper's sawtooth cycle (GPU)
@pytest.mark.parametrize("d,n", [(2, 4), (2, 64), (2, 256), (3, 16), (3, 64)])
@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("alpha,nu,copy", [(1.0, 1, True), (2.0 / 3.0, 2, False)])
def test_sawtooth_matches_oracle(B, orc, d, n, bc, alpha, nu, copy):
    """Fixed sawtooth cycles (the paper's settings, and damped Jacobi with linear
    prolongation) match the oracle's cycle for cycle, residual histories included."""
    say("sawtooth", d, n, bc, alpha, nu, copy)
    rng = np.random.default_rng(900 + n + d + bc)
    f = rng.standard_normal((n,) * d)
    h = 1.0 / n
    k = 5
    ref = orc.saw_solve(f, h, bc, fixed_cycles=k, alpha=alpha, nu=nu, prolong_const=copy)
    xg = dev(np.zeros_like(f))
    st, stats = B.mg_poisson_solve(dev(f), xg, h, bc, fixed_cycles=k, cycle=B.CYCLE_SAWTOOTH,
                                   prolong=B.PROLONG_COPY if copy else B.PROLONG_LINEAR, nu1=0, nu2=nu,
                                   omega=alpha)
    assert stats["cycles"] == k
    scale = max(np.max(np.abs(ref.x)), 1e-300)
    assert np.max(np.abs(host(xg) - ref.x)) / scale < 1e-11
    assert np.max(np.abs(np.array(stats["hist"][:k + 1]) - ref.hist)) < 1e-12 * max(1.0, np.max(ref.hist))


def test_sawtooth_convergence_measured(B, orc):
    """Measured behaviour on 2D Dirichlet 128^2: as printed (alpha = 1, one step,
    copying prolongation) the cycle does not converge and the solver says so; damped
    with linear prolongation it reaches 1e-10 (oracle residual), with a slower factor
    than V(2,2)."""
    g = inputs.manufactured_2d(128, seed=0)
    f, h = g["f"], g["h"]
    xg = dev(np.zeros_like(f))
    st, stats = B.mg_poisson_solve(dev(f), xg, h, DIR, check=False, cycle=B.CYCLE_SAWTOOTH,
                                   prolong=B.PROLONG_COPY, nu1=0, nu2=1, omega=1.0, max_cycles=60)
    assert st == B.NP_ENOCONV
    xg = dev(np.zeros_like(f))
    st, s2 = B.mg_poisson_solve(dev(f), xg, h, DIR, cycle=B.CYCLE_SAWTOOTH, nu1=0, nu2=2, omega=2.0 / 3.0)
    assert orc.rel_res(f, host(xg), h, DIR) <= 1e-10
    xg = dev(np.zeros_like(f))
    st, sv = B.mg_poisson_solve(dev(f), xg, h, DIR)
    rho_saw = s2["rho_est"]
    say("sawtooth damped: cycles %d rho %.3f; V(2,2): cycles %d rho %.3f" % (s2["cycles"], rho_saw, sv["cycles"],
                                                                             sv["rho_est"]))
    assert s2["cycles"] > sv["cycles"]


def test_sawtooth_option_checks(B):
    a = dev(np.zeros((16, 16)))
    for kw in (dict(cycle=B.CYCLE_SAWTOOTH), dict(cycle=B.CYCLE_SAWTOOTH, nu1=0, smooth_prec=B.FP32),
               dict(prolong=B.PROLONG_COPY), dict(cycle=2)):
        with pytest.raises(B.NeuphysError):
            B.mg_poisson_solve(a, a.clone(), 1 / 16, DIR, **kw)


@pytest.mark.parametrize("d,n", [(2, 8192), (3, 1024)])
def test_maximum_sizes(B, d, n):
    """The largest grids the solver accepts (8192^2, 1024^3), Dirichlet, one sine mode
    k = (1, 2[, 3]) as the right-hand side, whose discrete solution is f / lambda_k in
    closed form (A's eigenvector).  The residual cannot be resolved below about
    eps 4d / (h^2 lambda_k) relative (cancellation in A x at this size: 1e-9 at 8192^2),
    so the tolerance is 1e-10 or 50 times that floor.  FP64, the FP32-storage mixed path
    and (3D) the BF16-storage one reach it, and their error obeys ||x - x*|| <= ||r|| /
    lambda_min (on the device).  At 8192^2 BF16 storage of the correction is too coarse:
    its rounding, amplified by A (condition number ~1e7), keeps the residual above that
    floor, and the solver must say so (NP_ENOCONV) instead of returning a wrong answer."""
    import torch
    say("maximum size", d, n)
    h = 1.0 / n
    c = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) * h
    ks = (1, 2, 3)[:d]
    f = torch.sin(ks[0] * np.pi * c)
    for a in range(1, d):
        f = torch.sin(ks[a] * np.pi * c).reshape((n,) + (1,) * a) * f
    f = f.contiguous()
    lam = (4 / h ** 2) * sum(np.sin(k * np.pi * h / 2) ** 2 for k in ks)
    lam_min = (4 * d / h ** 2) * np.sin(np.pi * h / 2) ** 2
    tol = max(1e-10, 50 * np.finfo(np.float64).eps * 4 * d / (h ** 2 * lam))
    nf = float(torch.linalg.vector_norm(f))
    for p in (B.FP64, B.FP32, B.BF16):
        x = torch.zeros_like(f)
        st, stats = B.mg_poisson_solve(f, x, h, DIR, tol=tol, smooth_prec=p, check=False)
        if p == B.BF16 and d == 2:
            say("  prec", p, "status", st, "cycles", stats["cycles"], "rel_res", stats["rel_res"])
            assert st == 0 or (st == B.NP_ENOCONV and stats["rel_res"] > tol)
            if st != 0:
                continue
        assert st == 0 and stats["rel_res"] <= tol
        rr = B.np_op_resid_norm(f, x, h, DIR) / nf
        err = float(torch.linalg.vector_norm(x - f / lam))
        say("  prec", p, "tol", tol, "cycles", stats["cycles"], "rel_res", rr, "error", err / (nf / lam))
        assert rr <= tol * (1 + 1e-6)
        assert err <= rr * nf / lam_min * (1 + 1e-6) + 1e-13 * nf / lam
        del x


# ------------------------------------------ temporally blocked 3D level kernels
def level_arrays(prec, n, seed):
    """Seeded fine f, x and coarse c in the storage precision (BF16 as int16 bits)."""
    import torch
    rng = np.random.default_rng(seed)
    out = []
    for shape in ((n,) * 3, (n,) * 3, (n // 2,) * 3):
        a = torch.from_numpy(rng.standard_normal(shape)).cuda()
        if prec == B_FP32:
            a = a.float()
        elif prec == B_BF16:
            a = a.to(torch.bfloat16).view(torch.int16)
        out.append(a.contiguous())
    return out


B_FP64, B_FP32, B_BF16 = 0, 1, 2


def as64(t):
    import torch
    return (t.view(torch.bfloat16) if t.dtype == torch.int16 else t).double().cpu().numpy()


@pytest.mark.parametrize("prec", [B_FP64, B_FP32, B_BF16])
@pytest.mark.parametrize("n", [32, 64, 128])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_fused3_level_kernels_match_per_kernel_path(B, prec, n, bc):
    """The block kernels of the small levels -- k_down0_b (two sweeps from zero +
    residual + restriction in one pass) and k_up2_b (prolongation + correction + two
    sweeps in one pass) -- against the per-kernel path on the same buffers: bit for
    bit where that path restricts one coarse cell at a time (n < 128, children summed
    in (z, y, x) order), the iterates bit for bit and the restriction to rounding at
    n = 128 (z-marching restriction, another summation order)."""
    import torch
    say("fused3", prec, n, bc)
    h = 1.0 / n
    f, x, c = level_arrays(prec, n, 40 + n + bc + 10 * prec)
    xa, xb = torch.zeros_like(x), torch.zeros_like(x)
    ca, cb = torch.zeros_like(c), torch.zeros_like(c)
    B.np_op_level(B.LEVEL_ZERO2, f, xa, None, None, h, bc, prec)
    B.np_op_level(B.LEVEL_RESTRICT, f, xa, None, ca, h, bc, prec)
    ya, yo = x.clone(), torch.zeros_like(x)
    B.np_op_level(B.LEVEL_PSWEEP_SWEEP, f, ya, yo, c, h, bc, prec)
    knob = B.np_get_tuning("fbnt")
    try:
        for nt in (512, 1024):  # one thread per block cell, or twice as many
            B.np_set_tuning("fbnt", nt)
            xb, cb = torch.zeros_like(x), torch.zeros_like(c)
            B.np_op_level(B.LEVEL_DOWN0, f, xb, None, cb, h, bc, prec)
            say("  %d down x diff %.3e, c diff %.3e" % (nt, rel(as64(xb), as64(xa)), rel(as64(cb), as64(ca))))
            assert torch.equal(xa, xb)
            if n < 128:
                assert torch.equal(ca, cb)
            else:
                assert rel(as64(cb), as64(ca)) < {B_FP64: 1e-13, B_FP32: 1e-5, B_BF16: 1e-2}[prec]
            yb = torch.zeros_like(x)
            B.np_op_level(B.LEVEL_UP2, f, x, yb, c, h, bc, prec)
            say("  %d up diff %.3e" % (nt, rel(as64(yb), as64(ya))))
            assert torch.equal(ya, yb)
    finally:
        B.np_set_tuning("fbnt", knob)


@pytest.mark.parametrize("n", [32, 64, 128])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_fused3_level_kernels_match_oracle(B, orc, n, bc):
    """FP64: the fused down-leg and up-leg against the oracle's steps (Jacobi, residual,
    restriction, prolongation) within 1e-12."""
    say("fused3 oracle", n, bc)
    h = 1.0 / n
    f, x, c = level_arrays(B_FP64, n, 70 + n + bc)
    fh, xh, ch = host(f), host(x), host(c)
    xz, cz = torch_zeros_like(x), torch_zeros_like(c)
    B.np_op_level(B.LEVEL_DOWN0, f, xz, None, cz, h, bc, B_FP64)
    x1 = orc.jacobi(fh, np.zeros_like(fh), h, bc)
    x2 = orc.jacobi(fh, x1, h, bc)
    fc = orc.restrict(orc.residual(fh, x2, h, bc))
    assert rel(host(xz), x2) < 1e-12 and rel(host(cz), fc) < 1e-12
    y = torch_zeros_like(x)
    B.np_op_level(B.LEVEL_UP2, f, x, y, c, h, bc, B_FP64)
    yr = orc.prolong_add(ch, xh.copy(), bc)
    yr = orc.jacobi(fh, orc.jacobi(fh, yr, h, bc), h, bc)
    assert rel(host(y), yr) < 1e-12


@pytest.mark.parametrize("prec", [B_FP64, B_FP32, B_BF16])
@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_up2z_matches_per_kernel_path(B, prec, n, bc):
    """The one-pass z-marching up-leg of the large levels (k_sweep2z with correction:
    prolongation + correction and both post-sweeps, the first sweep formed one plane
    ahead on the tile and a one-cell ring) against prolongation-into-sweep then
    sweep: the same terms in the same order, bit for bit."""
    import torch
    say("up2z", prec, n, bc)
    h = 1.0 / n
    f, x, c = level_arrays(prec, n, 90 + n + bc + 10 * prec)
    ya, yo = x.clone(), torch.zeros_like(x)
    B.np_op_level(B.LEVEL_PSWEEP_SWEEP, f, ya, yo, c, h, bc, prec)
    yz = torch.zeros_like(x)
    B.np_op_level(B.LEVEL_UP2Z, f, x, yz, c, h, bc, prec)
    say("  up2z diff %.3e" % rel(as64(yz), as64(ya)))
    assert torch.equal(ya, yz)


@pytest.mark.parametrize("prec", [B_FP64, B_FP32, B_BF16])
@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_sweep2z_matches_two_sweeps(B, prec, n, bc):
    """Two Jacobi sweeps in one z-marching pass (k_sweep2z without correction, the
    down-leg of a nonzero iterate) against two launches of the single-sweep kernel:
    bit for bit."""
    import torch
    say("sweep2z", prec, n, bc)
    h = 1.0 / n
    f, x, _ = level_arrays(prec, n, 120 + n + bc + 10 * prec)
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    B.np_prof_level(B.PROF_LEVEL_SWEEP, f, x, y1, h, bc, prec, reps=1)
    B.np_prof_level(B.PROF_LEVEL_SWEEP, f, y1, y2, h, bc, prec, reps=1)
    yz = torch.zeros_like(x)
    B.np_op_level(B.LEVEL_SWEEP2Z, f, x, yz, None, h, bc, prec)
    say("  sweep2z diff %.3e" % rel(as64(yz), as64(y2)))
    assert torch.equal(y2, yz)


@pytest.mark.parametrize("bc", [DIR, PER])
def test_sweep2z_knob_same_solves(B, orc, bc):
    """Whole 128^3 solves with the one-pass two-sweep kernels on and off: FP64 fixed
    cycles bit for bit equal and within 1e-12 of the oracle's cycles; every path to
    the tolerance in the same cycle count with equal iterates, judged by the oracle's
    residual (the residual check sums its partials over other tiles, so the checked
    norms agree to rounding)."""
    n = 128
    g = inputs.sine_rhs(3, n, seed=4)
    f, h = g["f"], g["h"]
    if bc == PER:
        f = f - f.mean()
    fg = dev(f)
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("sweep2z", v)
            for p in (B.FP64, B.FP32, B.BF16):
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(fg, xg, h, bc, smooth_prec=p)
                out[(v, p)] = (host(xg), stats["cycles"], stats["rel_res"])
                assert orc.rel_res(f, out[(v, p)][0], h, bc) <= 1e-10
            xg = dev(np.zeros_like(f))
            B.mg_poisson_solve(fg, xg, h, bc, fixed_cycles=3)
            out[(v, "fixed")] = host(xg)
    finally:
        B.np_set_tuning("sweep2z", 1)
    say("sweep2z on/off cycles", [(k, v[1], v[2]) for k, v in out.items() if k[1] != "fixed"])
    assert np.array_equal(out[(1, "fixed")], out[(0, "fixed")])
    for p in (B.FP64, B.FP32, B.BF16):
        assert out[(1, p)][1] == out[(0, p)][1] and np.array_equal(out[(1, p)][0], out[(0, p)][0])
        assert abs(out[(1, p)][2] / out[(0, p)][2] - 1) < 1e-9
    ref = orc.mg_solve(f, h, bc, fixed_cycles=3)
    assert rel(out[(1, "fixed")], ref.x) < 1e-12


@pytest.mark.parametrize("prec", [B_FP64, B_FP32, B_BF16])
@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_down0z_matches_per_kernel_path(B, prec, n, bc):
    """The one-pass down-leg of the large levels from a zero iterate (k_down0z: both
    pre-sweeps, the residual and the restriction) against the two-sweeps-from-zero
    kernel then k_restrict3: iterate and coarse right-hand side bit for bit (the
    children are summed in k_restrict3's order)."""
    import torch
    say("down0z", prec, n, bc)
    h = 1.0 / n
    f, x, c = level_arrays(prec, n, 150 + n + bc + 10 * prec)
    xa, xb = torch.zeros_like(x), torch.zeros_like(x)
    ca, cb = torch.zeros_like(c), torch.zeros_like(c)
    B.np_op_level(B.LEVEL_ZERO2, f, xa, None, None, h, bc, prec)
    B.np_op_level(B.LEVEL_RESTRICT, f, xa, None, ca, h, bc, prec)
    B.np_op_level(B.LEVEL_DOWN0Z, f, xb, None, cb, h, bc, prec)
    say("  down0z x diff %.3e, c diff %.3e" % (rel(as64(xb), as64(xa)), rel(as64(cb), as64(ca))))
    assert torch.equal(xa, xb)
    assert torch.equal(ca, cb)


def test_down0z_matches_oracle(B, orc):
    """FP64 at 128^3 (Dirichlet) and periodic: the one-pass down-leg against the
    oracle's Jacobi, residual and restriction within 1e-12."""
    for bc in (DIR, PER):
        n = 128
        h = 1.0 / n
        f, x, c = level_arrays(B_FP64, n, 170 + bc)
        fh = host(f)
        xz, cz = torch_zeros_like(x), torch_zeros_like(c)
        B.np_op_level(B.LEVEL_DOWN0Z, f, xz, None, cz, h, bc, B_FP64)
        x1 = orc.jacobi(fh, np.zeros_like(fh), h, bc)
        x2 = orc.jacobi(fh, x1, h, bc)
        fc = orc.restrict(orc.residual(fh, x2, h, bc))
        assert rel(host(xz), x2) < 1e-12 and rel(host(cz), fc) < 1e-12


@pytest.mark.parametrize("prec", [B_FP64, B_FP32, B_BF16])
@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_down2z_matches_per_kernel_path(B, prec, n, bc):
    """The one-pass down-leg of a nonzero iterate (k_down2z: both pre-sweeps, the
    residual and the restriction, one cell per thread) against the two-sweep pass then
    k_restrict3: iterate and coarse right-hand side bit for bit (children summed in
    k_restrict3's order: two cells per thread, the x-pair first)."""
    import torch
    h = 1.0 / n
    f, x, c = level_arrays(prec, n, 190 + n + bc + 10 * prec)
    ya, ca = torch.zeros_like(x), torch.zeros_like(c)
    B.np_op_level(B.LEVEL_SWEEP2Z, f, x, ya, None, h, bc, prec)
    B.np_op_level(B.LEVEL_RESTRICT, f, ya, None, ca, h, bc, prec)
    prev = B.np_get_tuning("d2cpt")
    try:
        for cpt in (1, 2):  # k_down2z, and k_down2z2 on two cells per thread
            B.np_set_tuning("d2cpt", cpt)
            say("down2z", prec, n, bc, "cells per thread", cpt)
            yb, cb = torch.zeros_like(x), torch.zeros_like(c)
            B.np_op_level(B.LEVEL_DOWN2Z, f, x, yb, cb, h, bc, prec)
            say("  down2z x diff %.3e, c diff %.3e" % (rel(as64(yb), as64(ya)), rel(as64(cb), as64(ca))))
            assert torch.equal(ya, yb), cpt
            assert torch.equal(ca, cb), cpt
    finally:
        B.np_set_tuning("d2cpt", prev)


@pytest.mark.parametrize("bc", [DIR, PER])
def test_down2z_knob_same_solves(B, orc, bc):
    """Whole 256^3 solves with the one-pass nonzero down-leg on and off: FP64 fixed
    cycles bit for bit and within 1e-12 of the oracle's; FP64, FP32- and BF16-mixed
    solves to the tolerance in the same cycles with equal iterates, judged by the
    oracle."""
    n = 256
    g = inputs.sine_rhs(3, n, seed=6)
    f, h = g["f"], g["h"]
    if bc == PER:
        f = f - f.mean()
    fg = dev(f)
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("down2z", v)
            for p in (B.FP64, B.FP32, B.BF16):
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(fg, xg, h, bc, smooth_prec=p)
                out[(v, p)] = (host(xg), stats["cycles"], stats["rel_res"])
                assert orc.rel_res(f, out[(v, p)][0], h, bc) <= 1e-10
            xg = dev(np.zeros_like(f))
            B.mg_poisson_solve(fg, xg, h, bc, fixed_cycles=3)
            out[(v, "fixed")] = host(xg)
    finally:
        B.np_set_tuning("down2z", 1)
    say("down2z on/off cycles", [(k, v[1], v[2]) for k, v in out.items() if k[1] != "fixed"])
    assert np.array_equal(out[(1, "fixed")], out[(0, "fixed")])
    for p in (B.FP64, B.FP32, B.BF16):
        assert out[(1, p)][1] == out[(0, p)][1] and np.array_equal(out[(1, p)][0], out[(0, p)][0])
        assert abs(out[(1, p)][2] / out[(0, p)][2] - 1) < 1e-9
    ref = orc.mg_solve(f, h, bc, fixed_cycles=3)
    assert rel(out[(1, "fixed")], ref.x) < 1e-12


@pytest.mark.parametrize("prec", [B_FP64, B_BF16])
def test_onepass_kernels_512(B, prec):
    """The one-pass level kernels at 512^3 (Dirichlet), where a workgroup marches 64
    (BF16) or 128 (FP64) planes: each against its per-kernel pair, bit for bit."""
    import torch
    n, bc = 512, DIR
    say("one-pass 512", prec)
    h = 1.0 / n
    f, x, c = level_arrays(prec, n, 230 + prec)
    ya, yo, yz = x.clone(), torch.zeros_like(x), torch.zeros_like(x)
    B.np_op_level(B.LEVEL_PSWEEP_SWEEP, f, ya, yo, c, h, bc, prec)
    B.np_op_level(B.LEVEL_UP2Z, f, x, yz, c, h, bc, prec)
    assert torch.equal(ya, yz)
    del yo
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    B.np_prof_level(B.PROF_LEVEL_SWEEP, f, x, y1, h, bc, prec, reps=1)
    B.np_prof_level(B.PROF_LEVEL_SWEEP, f, y1, y2, h, bc, prec, reps=1)
    B.np_op_level(B.LEVEL_SWEEP2Z, f, x, yz, None, h, bc, prec)
    assert torch.equal(y2, yz)
    ca, cb = torch.zeros_like(c), torch.zeros_like(c)
    B.np_op_level(B.LEVEL_RESTRICT, f, y2, None, ca, h, bc, prec)
    B.np_op_level(B.LEVEL_DOWN2Z, f, x, yz, cb, h, bc, prec)
    assert torch.equal(y2, yz) and torch.equal(ca, cb)
    xa, xb = torch.zeros_like(x), torch.zeros_like(x)
    B.np_op_level(B.LEVEL_ZERO2, f, xa, None, None, h, bc, prec)
    B.np_op_level(B.LEVEL_RESTRICT, f, xa, None, ca, h, bc, prec)
    B.np_op_level(B.LEVEL_DOWN0Z, f, xb, None, cb, h, bc, prec)
    assert torch.equal(xa, xb) and torch.equal(ca, cb)


def test_up2z_needs_large_level(B):
    import torch
    f, x, c = level_arrays(B_FP64, 64, 1)
    for kind in (B.LEVEL_UP2Z, B.LEVEL_SWEEP2Z, B.LEVEL_DOWN0Z, B.LEVEL_DOWN2Z):
        with pytest.raises(B.NeuphysError):
            B.np_op_level(kind, f, x, torch.zeros_like(x), c, 1.0 / 64, DIR, B_FP64)


def torch_zeros_like(t):
    import torch
    return torch.zeros_like(t)


def test_fused3_knob_same_solves(B, orc):
    """Whole solves with the small levels' block kernels on and off: bit for bit equal
    (FP64 fixed cycles, and every path to the tolerance, judged by the oracle's
    residual), and FP64 equal to the oracle's cycles within 1e-12."""
    n = 128
    g = inputs.sine_rhs(3, n, seed=3)
    f, h = g["f"], g["h"]
    fg = dev(f)
    out = {}
    try:
        for v in (1, 0):
            B.np_set_tuning("fuseb", v)
            for p in (B.FP64, B.FP32, B.BF16):
                xg = dev(np.zeros_like(f))
                st, stats = B.mg_poisson_solve(fg, xg, h, DIR, smooth_prec=p)
                out[(v, p)] = (host(xg), stats["cycles"])
                assert orc.rel_res(f, out[(v, p)][0], h, DIR) <= 1e-10
            xg = dev(np.zeros_like(f))
            B.mg_poisson_solve(fg, xg, h, DIR, fixed_cycles=3)
            out[(v, "fixed")] = host(xg)
    finally:
        B.np_set_tuning("fuseb", 1)
    say("fuseb on/off cycles", [(k, v[1]) for k, v in out.items() if k[1] != "fixed"])
    assert np.array_equal(out[(1, "fixed")], out[(0, "fixed")])
    for p in (B.FP64, B.FP32, B.BF16):
        assert out[(1, p)][1] == out[(0, p)][1] and np.array_equal(out[(1, p)][0], out[(0, p)][0])
    ref = orc.mg_solve(f, h, DIR, fixed_cycles=3)
    assert rel(out[(1, "fixed")], ref.x) < 1e-12
