"""The static-workspace solve (mg_poisson_solve_noalloc) through the C ABI: the
same results as mg_poisson_solve, call after call, with nothing allocated."""
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


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def case(d, n, bc, seed):
    if bc == DIR:
        g = inputs.sine_rhs(d, n, seed=seed)
        return g["f"], g["h"]
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n,) * d), 1.0 / n


def test_noalloc_matches_solve_on_consecutive_calls(B, orc):
    """Largest 3D grid the workspace holds, then smaller grids of the other kinds:
    each result equals the cached-workspace solve (same cycles) and meets the
    tolerance as judged by the oracle."""
    import torch
    for d, n, bc, seed in ((3, 128, DIR, 0), (2, 64, PER, 1), (2, 1024, DIR, 2), (3, 16, PER, 3)):
        print("noalloc", d, n, bc, flush=True)
        f, h = case(d, n, bc, seed)
        fd = dev(f)
        xr = torch.zeros_like(fd)
        _, sr = B.mg_poisson_solve(fd, xr, h, bc)
        x = torch.full_like(fd, 3.0)  # stale contents: the solve starts from zero
        _, sn = B.mg_poisson_solve_noalloc(fd, x, h, bc)
        assert sn["cycles"] == sr["cycles"] and sn["rel_res"] == pytest.approx(sr["rel_res"], rel=1e-9)
        assert rel(x.cpu().numpy(), xr.cpu().numpy()) < 1e-12
        fm = f - f.mean() if bc == PER else f
        assert orc.rel_res(fm, x.cpu().numpy(), h, bc) <= 1e-10


def test_noalloc_matches_oracle_cycle_for_cycle(B, orc):
    import torch
    for d, n, bc in ((3, 64, PER), (2, 32, DIR)):
        f, h = case(d, n, bc, 7)
        ref = orc.mg_solve(f, h, bc, fixed_cycles=3)
        x = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
        _, st = B.mg_poisson_solve_noalloc(dev(f), x, h, bc, fixed_cycles=3)
        assert st["cycles"] == 3
        assert rel(x.cpu().numpy(), ref.x) < 1e-12
        assert np.max(np.abs(np.array(st["hist"][:4]) - ref.hist)) < 1e-12


def test_noalloc_warm_start_and_zero_rhs(B, orc):
    import torch
    f, h = case(2, 128, DIR, 4)
    fd = dev(f)
    x = torch.zeros_like(fd)
    B.mg_poisson_solve_noalloc(fd, x, h, DIR, tol=1e-6)
    _, st = B.mg_poisson_solve_noalloc(fd, x, h, DIR, warm_start=2)
    assert 0 < st["cycles"] < 15 and orc.rel_res(f, x.cpu().numpy(), h, DIR) <= 1e-10
    z = torch.zeros_like(fd)
    x.fill_(5.0)
    _, st = B.mg_poisson_solve_noalloc(z, x, h, DIR)
    assert st["cycles"] == 0 and bool(torch.all(x == 0))


def test_noalloc_rejects_what_it_cannot_hold(B):
    import torch
    for shape in ((2048, 2048), (256, 256, 256)):
        a = torch.zeros(shape, dtype=torch.float64, device="cuda")
        with pytest.raises(B.NeuphysError) as e:
            B.mg_poisson_solve_noalloc(a, a.clone(), 1.0 / shape[0], DIR)
        assert e.value.status == B.NP_EINVAL and "workspace" in str(e.value)
    a = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    for kw in (dict(smooth_prec=B.FP32), dict(warm_start=1), dict(cycle=B.CYCLE_SAWTOOTH, nu1=0)):
        with pytest.raises(B.NeuphysError):
            B.mg_poisson_solve_noalloc(a, a.clone(), 1.0 / 64, DIR, **kw)
