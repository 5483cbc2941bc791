"""GPU parity of the projection step and the scalar advection-diffusion step."""
import json
import os

import numpy as np
import pytest

from paper_2402_17913_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


@pytest.mark.parametrize("d,n,seed", [(2, 64, 0), (2, 256, 3), (3, 16, 1), (3, 32, 2)])
def test_projection_step_parity(B, orc, d, n, seed):
    print("ns step", d, n, flush=True)
    g = inputs.divfree_velocity(d, n, seed=seed)
    h, dt, nu = g["h"], g["dt"], 1e-3
    rng = np.random.default_rng(seed)
    p = 0.1 * rng.standard_normal((n,) * d)
    p -= p.mean()
    q_ref, p_ref, cyc, rr, st = orc.ns_step(g["q"], p, h, dt, nu)
    assert st == 0
    q = [dev(c) for c in g["q"]]
    pg = dev(p)
    w = q[2] if d == 3 else None
    st, stats = B.ns_projection_step(q[0], q[1], w, pg, h, dt, nu, fixed_cycles=cyc)
    assert stats["cycles"] == cyc
    for c in range(d):
        assert rel(host(q[c]), q_ref[c]) < 1e-12
    assert rel(host(pg), p_ref) < 1e-12
    div = orc.divergence([host(c) for c in q], h)
    qs = orc.ns_momentum(g["q"], p, h, dt, nu)
    assert np.linalg.norm(div) / np.linalg.norm(orc.divergence(qs, h)) <= 1.5e-10


def test_projection_step_parity_2d_1024(B, orc):
    """One step of the 2D periodic workload at its own size (1024^2, seed 0, nu 1e-3,
    dt = CFL 0.5) from a shared state with a seeded mean-free pressure, against the
    oracle's step (Section 2.4, the projection algorithm) at the oracle's cycle count."""
    n, d = 1024, 2
    print("ns step 2d 1024", flush=True)
    g = inputs.divfree_velocity(d, n, seed=0)
    h, dt, nu = g["h"], g["dt"], 1e-3
    rng = np.random.default_rng(11)
    p = 0.1 * rng.standard_normal((n, n))
    p -= p.mean()
    q_ref, p_ref, cyc, rr, st = orc.ns_step(g["q"], p, h, dt, nu)
    assert st == 0 and rr <= 1e-10
    q = [dev(c) for c in g["q"]]
    pg = dev(p)
    st, stats = B.ns_projection_step(q[0], q[1], None, pg, h, dt, nu, fixed_cycles=cyc)
    assert stats["cycles"] == cyc
    errs = [rel(host(q[c]), q_ref[c]) for c in range(d)] + [rel(host(pg), p_ref)]
    print("2d 1024: %d cycles, rel diffs %s" % (cyc, ["%.2e" % e for e in errs]), flush=True)
    assert max(errs) < 1e-12


def test_projection_step_parity_3d_256(B, orc):
    """One step of the 3D periodic workload at its own size (256^3, seed 0) with two
    pressure cycles (bounding the oracle's time): momentum stages, divergence, the
    periodic 256^3 multigrid solve and the correction against the oracle's step."""
    n, d = 256, 3
    print("ns step 3d 256", flush=True)
    g = inputs.divfree_velocity(d, n, seed=0)
    h, dt, nu = g["h"], g["dt"], 1e-3
    rng = np.random.default_rng(12)
    p = 0.1 * rng.standard_normal((n,) * 3)
    p -= p.mean()
    q_ref, p_ref, cyc, rr, st = orc.ns_step(g["q"], p, h, dt, nu, fixed_cycles=2)
    assert st == 0 and cyc == 2
    q = [dev(c) for c in g["q"]]
    pg = dev(p)
    st, stats = B.ns_projection_step(q[0], q[1], q[2], pg, h, dt, nu, fixed_cycles=2)
    assert stats["cycles"] == 2
    errs = [rel(host(q[c]), q_ref[c]) for c in range(d)] + [rel(host(pg), p_ref)]
    print("3d 256: rel diffs %s" % ["%.2e" % e for e in errs], flush=True)
    assert max(errs) < 1e-12


@pytest.mark.parametrize("n", [32, 64, 128])
def test_projection_step_zmarch_matches_per_cell(B, n):
    """The staggered momentum stages on z-marching tiles (LDS rings of the advecting
    velocity, the advanced field and p; three planes per field, or two with the
    out-of-ring z-neighbours of the own column in registers; 4 or 8 corrector tile
    rows) against the one-cell-per-thread kernels: the same terms in the same order,
    so the whole step agrees bit for bit."""
    import torch
    g = inputs.divfree_velocity(3, n, seed=7)
    rng = np.random.default_rng(8)
    p0 = 0.1 * rng.standard_normal((n,) * 3)
    configs = [(0, 2, 4), (1, 2, 4), (1, 2, 8), (1, 3, 4), (1, 3, 8)]  # zmarch, ring planes, corrector rows
    out = {}
    try:
        for cfg in configs:
            for key, v in zip(("zmarch_explicit", "mom_ring", "mom_rows"), cfg):
                B.np_set_tuning(key, v)
            q = [dev(c) for c in g["q"]]
            pg = dev(p0)
            B.ns_projection_step(q[0], q[1], q[2], pg, g["h"], g["dt"], 1e-3, fixed_cycles=3)
            out[cfg] = [host(t) for t in q] + [host(pg)]
    finally:
        for key, v in (("zmarch_explicit", 1), ("mom_ring", 2), ("mom_rows", 4)):
            B.np_set_tuning(key, v)
    for cfg in configs[1:]:
        for a, b in zip(out[cfg], out[configs[0]]):
            assert np.array_equal(a, b), (cfg, rel(a, b))


def test_projection_step_many_steps_drift(B, orc):
    """Ten steps from a shared start stay within 1e-11 of the oracle (reported drift)."""
    n, d = 64, 2
    g = inputs.divfree_velocity(d, n, seed=5)
    h, dt, nu = g["h"], g["dt"], 1e-3
    q_or, p_or = [c.copy() for c in g["q"]], np.zeros((n, n))
    q = [dev(c) for c in g["q"]]
    pg = dev(np.zeros((n, n)))
    for s in range(10):
        q_or, p_or, cyc, rr, st = orc.ns_step(q_or, p_or, h, dt, nu)
        B.ns_projection_step(q[0], q[1], None, pg, h, dt, nu, fixed_cycles=cyc)
    drift = max(rel(host(q[c]), q_or[c]) for c in range(d))
    print("10-step drift", drift, flush=True)
    assert drift < 1e-11


@pytest.mark.parametrize("d,n,bc", [(2, 33, 0), (2, 64, 1), (3, 17, 0), (3, 16, 1)])
def test_ad_scalar_step_parity(B, orc, d, n, bc):
    rng = np.random.default_rng(n)
    T = rng.standard_normal((n,) * d)
    a = [rng.standard_normal((n,) * d) for _ in range(d)]
    h, dt, nu = 0.5, 0.01, 0.3
    Tg = dev(T)
    B.np_ad_scalar_step(Tg, h, dt, nu, bc, a=[dev(c) for c in a])
    assert rel(host(Tg), orc.ad_scalar_step(T, h, bc, dt, nu, a=a)) < 1e-13
    Tg = dev(T)
    B.np_ad_scalar_step(Tg, h, dt, nu, bc)
    assert rel(host(Tg), orc.ad_scalar_step(T, h, bc, dt, nu)) < 1e-13


def test_diffusion_peaks_on_gpu(B):
    gold = json.load(open(os.path.join(GOLDEN, "diffusion_peaks.json")))
    Tg = dev(inputs.gaussian_2d(301, 40.0))
    dt, nu = 0.1, 2.0
    targets = {int(round(t / dt)): p for t, p in zip(gold["t"], gold["peak"])}
    for s in range(1, max(targets) + 1):
        B.np_ad_scalar_step(Tg, 1.0, dt, nu, 0)
        if s in targets:
            assert abs(float(Tg.max()) - targets[s]) < 5e-4
