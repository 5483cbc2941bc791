"""GPU parity of the implicit advection-diffusion multigrid (np_ad_implicit_solve)
against the FP64 oracle.

Bar: FP64 throughout; the operator alone to 1e-13 relative, fixed cycle counts to
1e-11 relative (x) and 1e-12 (residual histories); tolerance-stopped solves judged
by the oracle's own residual of the GPU result.
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


def ops(B, orc, d, bc, dt, nu, a, scheme):
    return B.ad_op(dt, nu, a[:d], scheme), orc.ad_op(d, bc, dt, nu, a[:d], scheme)


VEL = [1.0, -0.6, 0.35]
PAPER = dict(dt=50.0, nu=2.0, a=[1.0, 1.0, 1.0])  # Section 3.2: C = 50, dx = 1


def oracle_rel_res(orc, op_o, f, x, h):
    r = f - orc.ad_apply(op_o, x, h)
    return np.linalg.norm(r) / np.linalg.norm(f)


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("d,n", [(2, 4), (2, 8), (2, 64), (2, 256), (3, 4), (3, 8), (3, 32)])
@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("scheme", [0, 1])
def test_ad_apply(B, orc, d, n, bc, scheme):
    say("ad apply", d, n, bc, scheme)
    rng = np.random.default_rng(10 + n + d + bc + 7 * scheme)
    x = rng.standard_normal((n,) * d)
    h = 0.5
    op_g, op_o = ops(B, orc, d, bc, 3.0, 0.7, VEL, scheme)
    y = dev(np.zeros_like(x))
    B.np_ad_apply(dev(x), y, h, bc, op_g)
    assert rel(host(y), orc.ad_apply(op_o, x, h)) < 1e-13


# ------------------------------------------------------------- fixed cycles
@pytest.mark.parametrize("d,n", [(2, 4), (2, 16), (2, 128), (2, 512), (2, 1024), (3, 8), (3, 32), (3, 64), (3, 128)])
@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("scheme", [0, 1])
def test_ad_vcycles_match_oracle(B, orc, d, n, bc, scheme):
    """k V(2,2) cycles from zero match the oracle's k cycles, residual histories included."""
    say("ad vcycle", d, n, bc, scheme)
    f = np.random.default_rng(200 + n + d + bc).standard_normal((n,) * d)
    h, k = 1.0, 4
    op_g, op_o = ops(B, orc, d, bc, 8.0, 1.5, VEL, scheme)
    ref = orc.ad_solve(op_o, f, h, fixed_cycles=k)
    xg = dev(np.zeros_like(f))
    st, stats = B.np_ad_implicit_solve(dev(f), xg, h, bc, op_g, fixed_cycles=k)
    assert stats["cycles"] == k
    assert rel(host(xg), ref.x) < 1e-11
    assert np.max(np.abs(np.array(stats["hist"][:k + 1]) - ref.hist)) < 1e-12


@pytest.mark.parametrize("d,n", [(2, 8), (2, 128), (3, 16), (3, 64)])
@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("alpha,nu,copy", [(1.0, 1, True), (1.0, 1, False), (2.0 / 3.0, 2, False)])
def test_ad_sawtooth_matches_oracle(B, orc, d, n, bc, alpha, nu, copy):
    say("ad sawtooth", d, n, bc, alpha, nu, copy)
    f = np.random.default_rng(300 + n + d + bc).standard_normal((n,) * d)
    h, k = 1.0, 5
    op_g, op_o = ops(B, orc, d, bc, PAPER["dt"], PAPER["nu"], PAPER["a"], 0)
    ref = orc.ad_solve(op_o, f, h, cycle=1, nu1=0, nu2=nu, omega=alpha, prolong_const=copy, fixed_cycles=k)
    xg = dev(np.zeros_like(f))
    st, stats = B.np_ad_implicit_solve(dev(f), xg, h, bc, op_g, fixed_cycles=k, cycle=B.CYCLE_SAWTOOTH,
                                       prolong=B.PROLONG_COPY if copy else B.PROLONG_LINEAR, nu1=0, nu2=nu,
                                       omega=alpha)
    assert stats["cycles"] == k
    assert rel(host(xg), ref.x) < 1e-11
    assert np.max(np.abs(np.array(stats["hist"][:k + 1]) - ref.hist)) < 1e-12 * max(1.0, np.max(ref.hist))


# ------------------------------------------------- the paper's experiment
def test_ad_paper_experiment_l1_gauge(B, orc):
    """Section 3.2 (128^2, Dirichlet, u = v = 1, nu = 2, dt = 50, Gaussian gamma = 10,
    upwind, zero first estimate): the per-cycle L1 change matches the oracle's for the
    sawtooth with linear prolongation (over three orders of reduction in 50 cycles) and
    for V(2,2)."""
    n = 128
    T0 = inputs.gaussian_2d(n, gamma=10.0)
    op_g, op_o = ops(B, orc, 2, DIR, PAPER["dt"], PAPER["nu"], PAPER["a"], 0)
    ref = orc.ad_solve(op_o, T0, 1.0, cycle=1, nu1=0, nu2=1, omega=1.0, prolong_const=False, fixed_cycles=50)
    xg = dev(np.zeros_like(T0))
    st, s = B.np_ad_implicit_solve(dev(T0), xg, 1.0, DIR, op_g, l1=True, fixed_cycles=50, cycle=B.CYCLE_SAWTOOTH,
                                   nu1=0, nu2=1, omega=1.0)
    l1 = np.array(s["l1_change"])
    assert len(l1) == 50
    assert rel(l1, ref.l1diff) < 1e-9
    assert l1[-1] < 1e-3 * l1[0]
    say("sawtooth (linear) L1 change: first %.3g, 50th %.3g" % (l1[0], l1[-1]))
    refv = orc.ad_solve(op_o, T0, 1.0, fixed_cycles=10)
    xg = dev(np.zeros_like(T0))
    st, s = B.np_ad_implicit_solve(dev(T0), xg, 1.0, DIR, op_g, l1=True, fixed_cycles=10)
    assert rel(np.array(s["l1_change"]), refv.l1diff) < 1e-9


def test_ad_paper_experiment_converges(B, orc):
    """Tolerance-stopped V(2,2) on the paper's case: the oracle's residual of the GPU
    result meets the tolerance, in the oracle's number of cycles."""
    n = 128
    T0 = inputs.gaussian_2d(n, gamma=10.0)
    op_g, op_o = ops(B, orc, 2, DIR, PAPER["dt"], PAPER["nu"], PAPER["a"], 0)
    ref = orc.ad_solve(op_o, T0, 1.0, tol=1e-10)
    xg = dev(np.zeros_like(T0))
    st, s = B.np_ad_implicit_solve(dev(T0), xg, 1.0, DIR, op_g, tol=1e-10)
    assert st == 0 and s["cycles"] == ref.cycles
    assert oracle_rel_res(orc, op_o, T0, host(xg), 1.0) <= 1e-10 * (1 + 1e-6)


# ------------------------------------------------------------ full sizes
@pytest.mark.parametrize("d,n,gamma", [(2, 4096, 320.0), (3, 256, 20.0)])
@pytest.mark.parametrize("bc", [DIR, PER])
def test_ad_full_size(B, orc, d, n, gamma, bc):
    """Benchmark sizes (the paper's per-cell coefficients C = 50, nu dt / dx^2 = 100):
    the oracle's residual of the GPU solution meets the tolerance; periodic runs
    conserve the total (column sums of A are 1)."""
    say("ad full size", d, n, bc)
    T0 = inputs.gaussian_2d(n, gamma=gamma) if d == 2 else inputs.gaussian_3d(n, gamma=gamma)
    op_g, op_o = ops(B, orc, d, bc, PAPER["dt"], PAPER["nu"], PAPER["a"], 0)
    xg = dev(np.zeros_like(T0))
    st, s = B.np_ad_implicit_solve(dev(T0), xg, 1.0, bc, op_g, tol=1e-10)
    x = host(xg)
    assert st == 0
    assert oracle_rel_res(orc, op_o, T0, x, 1.0) <= 1e-10 * (1 + 1e-6)
    if bc == PER:
        assert abs(x.sum() - T0.sum()) <= 1e-9 * T0.sum()
    say("  cycles", s["cycles"], "rho", s["rho_est"])


# --------------------------------------------------------------- edge cases
def test_ad_coarsest_only_grid_is_exact(B, orc):
    """n = 4: one cycle is the exact (pivoted) solve."""
    f = np.random.default_rng(4).standard_normal((4, 4))
    op_g, op_o = ops(B, orc, 2, DIR, PAPER["dt"], PAPER["nu"], PAPER["a"], 0)
    xg = dev(np.zeros_like(f))
    B.np_ad_implicit_solve(dev(f), xg, 1.0, DIR, op_g, fixed_cycles=1)
    ref = orc.ad_vcycle(op_o, f, np.zeros_like(f), 1.0)
    assert rel(host(xg), ref) < 1e-13


def test_ad_zero_rhs_and_warm_start(B, orc):
    n = 64
    op_g, op_o = ops(B, orc, 2, PER, 4.0, 1.0, VEL, 1)
    xg = dev(np.ones((n, n)))
    st, s = B.np_ad_implicit_solve(dev(np.zeros((n, n))), xg, 1.0, PER, op_g)
    assert st == 0 and s["cycles"] == 0 and np.all(host(xg) == 0.0)
    f = np.random.default_rng(5).standard_normal((n, n))
    xg = dev(np.zeros_like(f))
    B.np_ad_implicit_solve(dev(f), xg, 1.0, PER, op_g, tol=1e-11)
    st, s = B.np_ad_implicit_solve(dev(f), xg, 1.0, PER, op_g, tol=1e-10, warm_start=2)
    assert st == 0 and s["cycles"] == 0


def test_ad_operator_changes_between_solves(B, orc):
    """Replayed cycles are keyed by the operator: alternating two operators on one
    grid gives each its own oracle result, bit-identical on repetition."""
    n = 64
    f = np.random.default_rng(6).standard_normal((n, n))
    outs = []
    for dt in (50.0, 5.0, 50.0):
        op_g, op_o = ops(B, orc, 2, DIR, dt, 2.0, PAPER["a"], 0)
        ref = orc.ad_solve(op_o, f, 1.0, fixed_cycles=3)
        xg = dev(np.zeros_like(f))
        B.np_ad_implicit_solve(dev(f), xg, 1.0, DIR, op_g, fixed_cycles=3)
        assert rel(host(xg), ref.x) < 1e-11
        outs.append(host(xg))
    assert np.array_equal(outs[0], outs[2])


def test_ad_argument_checks(B):
    n = 16
    a = dev(np.zeros((n, n)))
    f = dev(np.ones((n, n)))
    good = B.ad_op(1.0, 1.0, [1.0, 1.0])
    for op, kw in ((B.ad_op(0.0, 1.0, [1.0, 1.0]), {}), (B.ad_op(1.0, -1.0, [1.0, 1.0]), {}),
                   (B.ad_op(1.0, 1.0, [1.0, float("nan")]), {}), (B.ad_op(1.0, 1.0, [1.0, 1.0], 2), {}),
                   (good, dict(smooth_prec=B.FP32)), (good, dict(warm_start=1)),
                   (good, dict(cycle=B.CYCLE_SAWTOOTH)), (good, dict(prolong=B.PROLONG_COPY))):
        with pytest.raises(B.NeuphysError):
            B.np_ad_implicit_solve(f, a, 1.0, DIR, op, **kw)


def test_ad_solver_reports_divergence(B):
    """The sawtooth as printed diverges on the paper's case: the solver stops with
    NP_ENOCONV (three successive residual increases) instead of running on."""
    n = 128
    T0 = inputs.gaussian_2d(n, gamma=10.0)
    xg = dev(np.zeros_like(T0))
    st, s = B.np_ad_implicit_solve(dev(T0), xg, 1.0, DIR, B.ad_op(50.0, 2.0, [1.0, 1.0]), check=False,
                                   cycle=B.CYCLE_SAWTOOTH, prolong=B.PROLONG_COPY, nu1=0, nu2=1, omega=1.0)
    assert st == B.NP_ENOCONV


def test_ad_level_timing_entry(B, orc):
    """np_ad_prof_level runs the solver's finest-level kernels (2D row-marching and 3D
    z-marching shapes included) and reports a positive duration; the timed sweep and
    restriction leave the oracle's values in y."""
    for d, n in ((2, 1024), (3, 128), (2, 64)):
        fh = np.random.default_rng(7).standard_normal((n,) * d)
        xh = np.random.default_rng(8).standard_normal((n,) * d)
        f, x = dev(fh), dev(xh)
        y = dev(np.zeros((n,) * d))
        yc = dev(np.zeros((n // 2,) * d))
        op_g, op_o = ops(B, orc, d, DIR, 50.0, 2.0, [1.0, 1.0, 1.0], 0)
        assert B.np_ad_prof_level(B.PROF_LEVEL_SWEEP, f, x, y, 1.0, DIR, op_g, reps=3) > 0.0
        assert rel(host(y), orc.ad_jacobi(op_o, fh, xh, 1.0, omega=2.0 / 3.0)) < 1e-13
        assert B.np_ad_prof_level(B.PROF_LEVEL_RESTRICT, f, x, yc, 1.0, DIR, op_g, reps=3) > 0.0
        r = fh - orc.ad_apply(op_o, xh, 1.0)
        rc = r.reshape(tuple(v for k in range(d) for v in (n // 2, 2))).mean(axis=tuple(range(1, 2 * d, 2)))
        assert rel(host(yc), rc) < 1e-12
        assert B.np_ad_prof_level(B.PROF_LEVEL_PROLONG, None, x.clone(), yc, 1.0, DIR, op_g, reps=3) > 0.0
