"""GPU parity of the learned warm-start network (forward, gradients, training) and
of the solver's use of it.  The FP64 reference runs on BF16-rounded weights and
inputs; the GPU also rounds every activation to BF16, so agreement is judged by
relative L2 error (<= 2e-2) and cosine similarity (>= 0.999)."""
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


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def cosine(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


def params_for(levels, seed):
    from oracle import cnn
    ps = cnn.init_params(levels, seed=seed)
    rng = np.random.default_rng(seed + 100)
    out = []
    for k, (W, b) in enumerate(ps):
        b = rng.standard_normal(16) * 0.05
        if k == len(ps) - 1:
            b[1:] = 0.0
        out.append((cnn.bf16_round(W), cnn.bf16_round(b).astype(np.float64)))
    return out


@pytest.mark.parametrize("n,levels", [(32, 2), (64, 3)])
def test_cnn_forward_matches_oracle(B, n, levels):
    import torch
    from oracle import cnn
    print("cnn forward", n, levels, flush=True)
    ps = params_for(levels, seed=n)
    rng = np.random.default_rng(7)
    f = cnn.bf16_round(rng.standard_normal((n, n, n)))
    ref = cnn.forward(ps, f, levels)
    net = B.Cnn(n, levels)
    net.set_params(cnn.flatten(ps).astype(np.float32))
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    y = torch.empty_like(x)
    net.forward(x, y)
    got = y.cpu().numpy().astype(np.float64)
    net.close()
    print("  rel L2", rel_l2(got, ref), "cos", cosine(got, ref), flush=True)
    assert rel_l2(got, ref) <= 2e-2 and cosine(got, ref) >= 0.999


def test_cnn_gradients_match_oracle(B):
    import torch
    from oracle import cnn
    n, levels = 32, 2
    ps = params_for(levels, seed=3)
    rng = np.random.default_rng(8)
    f = cnn.bf16_round(rng.standard_normal((n, n, n)))
    t = rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    loss_ref, grads = cnn.loss_and_grads(ps, f, t, levels)
    net = B.Cnn(n, levels)
    net.set_params(cnn.flatten(ps).astype(np.float32))
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    tt = torch.from_numpy(t.astype(np.float32)).cuda()
    loss = net.gradients([x], [tt])
    g = net.get_grads().astype(np.float64)
    net.close()
    gref = cnn.flatten(grads)
    assert abs(loss - loss_ref) / loss_ref <= 2e-2
    print("all grads: rel L2 %.3e cos %.6f" % (rel_l2(g, gref), cosine(g, gref)), flush=True)
    per = 27 * 16 * 16 + 16
    for k in range(cnn.n_convs(levels)):
        a, b = g[k * per:(k + 1) * per], gref[k * per:(k + 1) * per]
        print("  conv %d: rel L2 %.3e cos %.6f" % (k, rel_l2(a, b), cosine(a, b)), flush=True)
        assert cosine(a, b) >= 0.999 and rel_l2(a, b) <= 5e-2
    assert cosine(g, gref) >= 0.999 and rel_l2(g, gref) <= 2e-2


@pytest.mark.parametrize("n,levels", [(16, 1), (32, 2), (64, 3)])
def test_cnn_zmarch_tiles_bit_identical(B, n, levels):
    """The z-marching convolution runs the same MFMA sequence per output as the
    one-plane form, so forward outputs and gradients agree bit for bit, for the
    automatic and for fixed plane counts (including one plane count above n)."""
    import torch
    from oracle import cnn
    print("cnn zmarch", n, levels, flush=True)
    ps = params_for(levels, seed=n + 1)
    rng = np.random.default_rng(9)
    f = cnn.bf16_round(rng.standard_normal((n, n, n)))
    t = rng.standard_normal((n, n, n)).astype(np.float32)
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    tt = torch.from_numpy(t).cuda()
    net = B.Cnn(n, levels)
    net.set_params(cnn.flatten(ps).astype(np.float32))
    res = {}
    try:
        for v in (0, 1, 2, 8, 64):
            B.np_set_tuning("conv3z", v)
            y = torch.empty_like(x)
            net.forward(x, y)
            loss = net.gradients([x], [tt])
            res[v] = (y.cpu().numpy(), loss, net.get_grads())
    finally:
        B.np_set_tuning("conv3z", 1)
        net.close()
    y0, l0, g0 = res[0]
    assert np.isfinite(y0).all() and np.abs(y0).max() > 0
    for v in (1, 2, 8, 64):
        y, l, g = res[v]
        assert np.array_equal(y, y0), v
        assert l == l0, v
        assert np.array_equal(g, g0), v


@pytest.mark.parametrize("n,levels", [(16, 1), (32, 2), (64, 3)])
def test_cnn_wgrad_matrix_cores_match_vector_path(B, n, levels):
    """The weight gradients on the matrix cores (voxels as the contraction, FP32
    accumulation in another order) agree with the FP32 vector-unit reduction to FP32
    rounding, layer by layer, and so does the loss."""
    import torch
    from oracle import cnn
    print("cnn wgrad", n, levels, flush=True)
    ps = params_for(levels, seed=n + 5)
    rng = np.random.default_rng(11)
    f = cnn.bf16_round(rng.standard_normal((n, n, n)))
    t = rng.standard_normal((n, n, n)).astype(np.float32)
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    tt = torch.from_numpy(t).cuda()
    net = B.Cnn(n, levels)
    net.set_params(cnn.flatten(ps).astype(np.float32))
    res = {}
    try:
        for v in (0, 1):
            B.np_set_tuning("wgrad_mfma", v)
            loss = net.gradients([x, x], [tt, tt])
            res[v] = (loss, net.get_grads().astype(np.float64))
    finally:
        B.np_set_tuning("wgrad_mfma", 1)
        net.close()
    (l0, g0), (l1, g1) = res[0], res[1]
    assert l0 == l1  # the forward pass and the loss do not depend on the gradient kernel
    per = 27 * 16 * 16 + 16
    for k in range(cnn.n_convs(levels)):
        a, b = g1[k * per:(k + 1) * per], g0[k * per:(k + 1) * per]
        print("  conv %d: rel L2 %.3e" % (k, rel_l2(a, b)), flush=True)
        assert np.abs(b).max() > 0 and rel_l2(a, b) <= 1e-5


@pytest.fixture(scope="module")
def trained(B, tmp_path_factory):
    """A 2-level net on the 32^3 restriction of 64^3 projection steps, trained by
    np_cnn_train on 48 pairs from seeds 11..18 (held-out evaluation seed 0)."""
    from paper_2402_17913_amd import learned
    path = str(tmp_path_factory.mktemp("cnn") / "net.npcnn")
    rs, ps, tgen = learned.make_pairs(64, seeds=list(range(11, 19)), steps=6, n_keep=32)
    hist, ttrain = learned.train(rs, ps, path, n_in=32, levels=2, epochs=30, batch=4, lr=5e-4, seed=1)
    print("pairs %d gen %.1fs train %.1fs loss %.3e -> %.3e" % (len(rs), tgen, ttrain, hist[0], hist[-1]),
          flush=True)
    net = B.Cnn(path=path)
    yield net, hist, path
    B.Cnn.detach()
    net.close()


def test_cnn_training_reduces_loss(B, trained):
    """Training lowers the loss well below the targets' variance (a network that
    collapsed to a constant output would stop at the variance) and the held-out
    prediction correlates with the held-out target."""
    import torch
    net, hist, _ = trained
    assert net.n_in == 32 and net.levels == 2
    assert hist[-1] < 0.25 * hist[0]
    n = 64
    g = inputs.divfree_velocity(3, n, seed=0)
    q = [torch.from_numpy(c).cuda() for c in g["q"]]
    p = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    rhs, dp = torch.empty_like(p), torch.empty_like(p)
    B.ns_projection_step_io(q[0], q[1], q[2], p, g["h"], g["dt"], 1e-3, rhs_out=rhs, dp_out=dp)
    xin = torch.empty((32,) * 3, dtype=torch.float32, device="cuda")
    t, y = torch.empty_like(xin), torch.empty_like(xin)
    net.prepare(rhs, dp, xin, t)
    net.forward(xin, y)
    tt = t.cpu().numpy().astype(np.float64)
    yy = y.cpu().numpy().astype(np.float64)
    yy -= yy.mean()
    var = float(np.mean(tt ** 2))
    print("held-out: target var %.3e, err %.3e, corr %.4f" % (var, np.mean((yy - tt) ** 2), cosine(yy, tt)),
          flush=True)
    assert hist[-1] < 0.2 * var and cosine(yy, tt) >= 0.9


def held_out_rhs(B):
    """The pressure right-hand side of the first 64^3 projection step of held-out seed 0."""
    import torch
    n = 64
    g = inputs.divfree_velocity(3, n, seed=0)
    q = [torch.from_numpy(c).cuda() for c in g["q"]]
    p = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    rhs = torch.empty_like(p)
    dp = torch.empty_like(p)
    B.ns_projection_step_io(q[0], q[1], q[2], p, g["h"], g["dt"], 1e-3, rhs_out=rhs, dp_out=dp)
    return rhs, g["h"]


def test_learned_warm_start_reaches_tolerance_and_gains(B, orc, trained):
    """The network loaded by np_cnn_load(path) warm-starts the pressure solve: the
    guess is accepted and the solve still meets the tolerance (judged by the
    oracle's residual).  Gain, stated as a margin: the guess's energy-norm error
    ||x0 - x*||_A (x* the oracle's solution) is below 0.9 of the zero guess's
    ||x*||_A.  The cycle counts with and without the guess are logged, not gated."""
    import torch
    _, _, path = trained
    rhs, h = held_out_rhs(B)
    f = rhs.cpu().numpy()
    fm = f - f.mean()
    ref = orc.mg_solve(fm, h, 1, tol=1e-13)
    xs = ref.x
    res = {}
    for ws in (0, 1):
        B.np_cnn_load(path if ws == 1 else None)
        for prec in (B.FP64, B.FP32):
            x = torch.zeros_like(rhs)
            st, stats = B.mg_poisson_solve(rhs, x, h, B.BC_PERIODIC, warm_start=ws, smooth_prec=prec)
            rr = orc.rel_res(fm, x.cpu().numpy(), h, 1)
            assert rr <= 1e-10
            res[(ws, prec)] = stats
            print("warm_start=%d prec=%d cycles=%d outer=%d fallback=%d first rel_res=%.3e" % (
                ws, prec, stats["cycles"], stats["outer_iters"], stats["used_fallback"], stats["hist"][0]),
                flush=True)
    B.np_cnn_load(path)
    x0 = torch.zeros_like(rhs)
    st, stats = B.mg_poisson_solve(rhs, x0, h, B.BC_PERIODIC, warm_start=1, max_cycles=0, check=False)
    assert stats["used_fallback"] == 0 and stats["cycles"] == 0
    e = x0.cpu().numpy() - xs
    ratio = np.sqrt(np.vdot(e, orc.apply_A(e, h, 1)) / np.vdot(xs, orc.apply_A(xs, h, 1)))
    print("learned guess: energy-norm error %.3f of the zero guess's; cycles FP64 %d vs %d from zero, "
          "FP32 %d vs %d" % (ratio, res[(1, B.FP64)]["cycles"], res[(0, B.FP64)]["cycles"],
                             res[(1, B.FP32)]["cycles"], res[(0, B.FP32)]["cycles"]), flush=True)
    for prec in (B.FP64, B.FP32):
        assert res[(1, prec)]["used_fallback"] == 0
    assert ratio < 0.9
    B.np_cnn_load(None)


def test_learned_coarse_grid_correction(B, orc, trained):
    """The network as the coarse-grid correction (cnn_cgc): in the first cycles the
    32^3 level of the 64^3 solve starts from the network's prediction for its
    restricted residual.  The solve meets the tolerance (oracle judge), the first
    cycle's prediction is kept (it lowers that level's energy-norm error), and the
    cycle counts are logged against the plain solve."""
    import torch
    _, _, path = trained
    rhs, h = held_out_rhs(B)
    fm = rhs.cpu().numpy() - float(rhs.mean())
    B.np_cnn_load(path)
    try:
        out = {}
        for cgc in (0, 1, 3, 256):
            x = torch.zeros_like(rhs)
            st, stats = B.mg_poisson_solve(rhs, x, h, B.BC_PERIODIC, cnn_cgc=cgc)
            assert orc.rel_res(fm, x.cpu().numpy(), h, 1) <= 1e-10
            out[cgc] = stats
            print("cnn_cgc=%d: %d cycles, %d corrections kept" % (cgc, stats["cycles"], stats["cgc_accepted"]),
                  flush=True)
        assert out[0]["cgc_accepted"] == 0
        assert out[1]["cgc_accepted"] == 1
        assert 1 <= out[3]["cgc_accepted"] <= 3
        with pytest.raises(B.NeuphysError):
            B.mg_poisson_solve(rhs, torch.zeros_like(rhs), h, B.BC_PERIODIC, cnn_cgc=1, smooth_prec=B.FP32)
    finally:
        B.np_cnn_load(None)


def test_learned_coarse_grid_correction_rejected_is_the_plain_cycle(B, orc):
    """A network with zero weights predicts zero, which does not lower the coarse
    level's energy: the correction is rejected and the solve equals the plain one
    cycle for cycle, bit for bit (the hooked cycles run the same kernels)."""
    import torch
    net = B.Cnn(32, 2)
    net.set_params(np.zeros(net.n, dtype=np.float32))
    net.attach()
    try:
        n = 64
        rng = np.random.default_rng(3)
        f = torch.from_numpy(rng.standard_normal((n, n, n))).cuda()
        xa, xb = torch.zeros_like(f), torch.zeros_like(f)
        _, sa = B.mg_poisson_solve(f, xa, 1.0 / n, B.BC_PERIODIC)
        _, sb = B.mg_poisson_solve(f, xb, 1.0 / n, B.BC_PERIODIC, cnn_cgc=4)
        assert sb["cgc_accepted"] == 0 and sa["cycles"] == sb["cycles"]
        assert torch.equal(xa, xb)
        ref = orc.mg_solve(f.cpu().numpy(), 1.0 / n, 1, fixed_cycles=3)
        xc = torch.zeros_like(f)
        B.mg_poisson_solve(f, xc, 1.0 / n, B.BC_PERIODIC, cnn_cgc=3, fixed_cycles=3)
        assert np.max(np.abs(xc.cpu().numpy() - ref.x)) / np.max(np.abs(ref.x)) < 1e-12
    finally:
        B.Cnn.detach()
        net.close()


def test_learned_warm_start_falls_back(B, orc):
    """A network with zero weights predicts zero: its energy-norm error equals that
    of the zero iterate, so the solver falls back and still converges."""
    import torch
    net = B.Cnn(16, 1)
    net.set_params(np.zeros(net.n, dtype=np.float32))
    net.attach()
    n = 32
    g = inputs.divfree_velocity(3, n, seed=2)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, n, n))
    fm = f - f.mean()
    x = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    st, stats = B.mg_poisson_solve(torch.from_numpy(f).cuda(), x, g["h"], B.BC_PERIODIC, warm_start=1)
    assert stats["used_fallback"] == 1
    assert orc.rel_res(fm, x.cpu().numpy(), g["h"], 1) <= 1e-10
    B.Cnn.detach()
    net.close()


def test_cnn_train_is_deterministic(B, tmp_path):
    """Same pairs and seed: byte-identical weight files (fixed-order reductions,
    seeded initialisation and shuffle); another seed gives other weights."""
    import torch
    rng = np.random.default_rng(5)
    rs = [torch.from_numpy(rng.standard_normal((32, 32, 32))).cuda() for _ in range(5)]
    ps = [torch.from_numpy(rng.standard_normal((32, 32, 32))).cuda() for _ in range(5)]
    files = []
    for k, seed in enumerate((3, 3, 4)):
        path = str(tmp_path / ("w%d.npcnn" % k))
        B.np_cnn_train(rs, ps, path, dict(n_in=16, levels=1, epochs=2, batch=2, seed=seed))
        files.append(open(path, "rb").read())
    assert files[0] == files[1]
    assert files[0] != files[2]
