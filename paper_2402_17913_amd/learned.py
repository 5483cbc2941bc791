"""Learned warm start: parameter initialisation, solver-generated training pairs
and the training loop (orchestration only; every operation runs in the HIP
library through `binding`).

Pairs come from the projection step itself: for a seeded divergence-free
velocity on the periodic [0, 2pi)^3 grid, each step's pressure-correction
right-hand side -(1/dt) D q* and the increment dp the multigrid solved for
form one (input, target) pair, restricted to the network's grid and scaled by
the rms of the restricted right-hand side (the map rhs -> dp is linear).
"""
import time

import numpy as np
import torch

from . import binding as B
from . import inputs

C = 16


def n_convs(levels):
    return 4 * levels - 1


def init_params(levels, seed=0, out_scale=0.1):
    """He-normal weights (first convolution reads channel 0, the output
    convolution writes channel 0), zero biases; layout of np_cnn_set_params.
    The output convolution starts `out_scale` times smaller: the targets
    (pressure increments over the rms of the right-hand side) have a variance
    near 1e-2, and a full-scale initial output makes the first Adam steps
    shrink every layer until the ReLUs die and the network predicts a constant."""
    rng = np.random.default_rng(seed)
    nc = n_convs(levels)
    out = []
    for k in range(nc):
        W = np.zeros((27, C, C), dtype=np.float64)
        if k == 0:
            W[:, :, 0] = rng.standard_normal((27, C)) * np.sqrt(2.0 / 27)
        elif k == nc - 1:
            W[:, 0, :] = rng.standard_normal((27, C)) * np.sqrt(1.0 / (27 * C)) * out_scale
        else:
            W[:] = rng.standard_normal((27, C, C)) * np.sqrt(2.0 / (27 * C))
        out.append(W.reshape(-1))
        out.append(np.zeros(C))
    return np.concatenate(out).astype(np.float32)


def make_pairs(net, n, seeds, steps, nu=1e-3, tol=1e-10, log=None):
    """Runs `steps` projection steps for each seed on the n^3 periodic grid and
    returns the prepared (input, target) FP32 tensors at the network's size,
    plus the wall time spent."""
    t0 = time.perf_counter()
    xs, ts = [], []
    for seed in seeds:
        g = inputs.divfree_velocity(3, n, seed=seed)
        q = [torch.from_numpy(c).cuda() for c in g["q"]]
        p = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        rhs = torch.empty_like(p)
        dp = torch.empty_like(p)
        for s in range(steps):
            B.ns_projection_step_io(q[0], q[1], q[2], p, g["h"], g["dt"], nu, rhs_out=rhs, dp_out=dp, tol=tol)
            x = torch.empty(_net_grid(net), dtype=torch.float32, device="cuda")
            t = torch.empty_like(x)
            net.prepare(rhs, dp, x, t)
            xs.append(x)
            ts.append(t)
        if log:
            log("  pairs from seed %d: %d" % (seed, len(xs)))
    return xs, ts, time.perf_counter() - t0


def _net_grid(net):
    return (net.n_in,) * 3


def train(net, xs, ts, epochs=10, batch=4, lr=5e-4, seed=0, log=None):
    """Adam on minibatches of the pairs, reshuffled (seeded) every epoch;
    returns the per-epoch mean loss and the wall time."""
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(xs))
        tot, cnt = 0.0, 0
        for i in range(0, len(order), batch):
            idx = order[i:i + batch]
            tot += net.train_step([xs[j] for j in idx], [ts[j] for j in idx], lr)
            cnt += len(idx)
        hist.append(tot / cnt)
        if log:
            log("  epoch %d  mse %.4e" % (ep, hist[-1]))
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def new_net(n_in, levels, seed=0):
    net = B.Cnn(n_in, levels)
    net.set_params(init_params(levels, seed))
    return net
