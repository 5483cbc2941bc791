"""GPU parity of the collocated projection step (ns_collocated_step: the paper's
collocated nodes with the central, upwind and finite-element filter families) against
the FP64 oracle.

Bar: FP64 with the oracle's pressure-solve cycle count: velocity and pressure <= 1e-11
relative; the approximate projection's divergence factor checked as a property at the
benchmark sizes.
"""
import numpy as np
import pytest

from paper_2402_17913_amd import inputs

pytestmark = pytest.mark.gpu


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


def case(d, n, seed):
    g = inputs.divfree_velocity(d, n, seed=seed)
    p = 0.1 * np.random.default_rng(seed).standard_normal((n,) * d)
    return g["q"], p - p.mean(), g["h"], g["dt"]


@pytest.mark.parametrize("d,n,seed", [(2, 16, 0), (2, 64, 1), (2, 256, 2), (3, 8, 3), (3, 16, 4), (3, 32, 5)])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_collocated_step_parity(B, orc, d, n, seed, scheme):
    print("collocated", d, n, scheme, flush=True)
    q0, p0, h, dt = case(d, n, seed)
    nu = 1e-2
    q_ref, p_ref, cyc = orc.nsc_step(q0, p0, h, dt, nu, scheme=scheme, tol=1e-10)
    q = [dev(c) for c in q0]
    pg = dev(p0)
    st, stats = B.ns_collocated_step(q[0], q[1], q[2] if d == 3 else None, pg, h, dt, nu, scheme=scheme,
                                     fixed_cycles=cyc)
    assert stats["cycles"] == cyc
    for c in range(d):
        assert rel(host(q[c]), q_ref[c]) < 1e-11
    assert rel(host(pg), p_ref) < 1e-11


@pytest.mark.parametrize("scheme", [0, 2])
def test_collocated_ten_steps(B, orc, scheme):
    q0, p0, h, dt = case(2, 64, 7)
    q_or, p_or = [c.copy() for c in q0], p0.copy()
    q, pg = [dev(c) for c in q0], dev(p0)
    for _ in range(10):
        q_or, p_or, cyc = orc.nsc_step(q_or, p_or, h, dt, 1e-2, scheme=scheme, tol=1e-10)
        B.ns_collocated_step(q[0], q[1], None, pg, h, dt, 1e-2, scheme=scheme, fixed_cycles=cyc)
    assert max(rel(host(q[c]), q_or[c]) for c in range(2)) < 1e-10


@pytest.mark.parametrize("d,n", [(2, 1024), (3, 128)])
def test_collocated_divergence_property_full_size(B, orc, d, n):
    """At the benchmark's sizes: the oracle's divergence of the GPU result is no larger
    than that of the momentum update it projected (the factor 1 - |s|^2/lambda_A lies in
    [0, 1] per mode), and the pressure solve converged."""
    print("collocated full size", d, n, flush=True)
    q0, p0, h, dt = case(d, n, 0)
    q, pg = [dev(c) for c in q0], dev(p0)
    st, stats = B.ns_collocated_step(q[0], q[1], q[2] if d == 3 else None, pg, h, dt, 1e-3, scheme=2)
    assert st == 0 and stats["rel_res"] <= 1e-10
    qs = orc.nsc_momentum(q0, p0, h, dt, 1e-3, scheme=2)
    div = lambda v: sum(orc.nsc_derivative(v[e], h, e, scheme=2) for e in range(d))
    before, after = np.linalg.norm(div(qs)), np.linalg.norm(div([host(c) for c in q]))
    print("  divergence %.3e -> %.3e" % (before, after), flush=True)
    assert after <= before * (1 + 1e-9)


def test_collocated_argument_checks(B):
    a = dev(np.zeros((16, 16)))
    for kw in (dict(scheme=3), dict(warm_start=2), dict(dt=0.0)):
        args = dict(dt=0.1, scheme=2)
        args.update(kw)
        ws = args.pop("warm_start", 0)
        with pytest.raises(B.NeuphysError):
            B.ns_collocated_step(a, a.clone(), None, a.clone(), 1.0, args["dt"], 0.1, scheme=args["scheme"],
                                 warm_start=ws)


@pytest.mark.parametrize("d,n", [(2, 64), (3, 16)])
@pytest.mark.parametrize("scheme", [0, 2])
def test_collocated_divergence_entry(B, orc, d, n, scheme):
    q0, _, h, _ = case(d, n, 9)
    q = [dev(c) for c in q0]
    div = dev(np.zeros((n,) * d))
    B.np_nsc_divergence(q[0], q[1], q[2] if d == 3 else None, div, h, scheme=scheme)
    ref = sum(orc.nsc_derivative(q0[e], h, e, scheme=scheme) for e in range(d))
    assert rel(host(div), ref) < 1e-12


@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_collocated_zmarch_matches_per_cell_kernels(B, n, scheme):
    """The 3D z-marching momentum, divergence and correction kernels give the per-cell
    kernels' step bit for bit (same neighbourhoods, same arithmetic)."""
    q0, p0, h, dt = case(3, n, 11)
    outs = []
    for zm in (1, 0):
        B.np_set_tuning("zmarch_explicit", zm)
        try:
            q, pg = [dev(c) for c in q0], dev(p0)
            B.ns_collocated_step(q[0], q[1], q[2], pg, h, dt, 1e-2, scheme=scheme, fixed_cycles=6)
            outs.append([host(c) for c in q] + [host(pg)])
        finally:
            B.np_set_tuning("zmarch_explicit", 1)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
