"""Learned warm start: solver-generated training pairs and training through the
library (orchestration only; every operation runs in the HIP library through
`binding`).

Pairs come from the projection step itself: for a seeded divergence-free
velocity on the periodic [0, 2pi)^3 grid, each step's pressure-correction
right-hand side -(1/dt) D q* and the increment dp the multigrid solved for
form one (rhs, dp) pair.  Both are restricted on the device, by 2^3 averaging,
to the size the network reads, so that thousands of pairs stay resident in
FP64; np_cnn_train then scales each pair by the rms of its right-hand side
(the map rhs -> dp is linear) and trains with Adam.
"""
import time

import torch

from . import binding as B
from . import inputs


def restrict(t, n_out):
    """2^3-average a device FP64 cube down to n_out^3 (the multigrid
    restriction of the residual of the zero iterate is the average of the
    field itself)."""
    cur = t
    while cur.shape[0] > n_out:
        n = cur.shape[0] // 2
        nxt = torch.empty((n, n, n), dtype=torch.float64, device=cur.device)
        B.np_op_resid_restrict(cur, torch.zeros_like(cur), nxt, 1.0, B.BC_PERIODIC)
        cur = nxt
    return cur.clone() if cur is t else cur


def make_pairs(n, seeds, steps, n_keep, nu=1e-3, tol=1e-10, log=None):
    """Runs `steps` projection steps from each seed's velocity on the n^3
    periodic grid; returns the (rhs, dp) pairs restricted to n_keep^3 (device
    FP64 lists) and the wall time spent."""
    t0 = time.perf_counter()
    rs, ps = [], []
    for seed in seeds:
        g = inputs.divfree_velocity(3, n, seed=seed)
        q = [torch.from_numpy(c).cuda() for c in g["q"]]
        p = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        rhs = torch.empty_like(p)
        dp = torch.empty_like(p)
        for _ in range(steps):
            B.ns_projection_step_io(q[0], q[1], q[2], p, g["h"], g["dt"], nu, rhs_out=rhs, dp_out=dp, tol=tol)
            rs.append(restrict(rhs, n_keep))
            ps.append(restrict(dp, n_keep))
        if log:
            log("  pairs from seed %d: %d" % (seed, len(rs)))
    torch.cuda.synchronize()
    return rs, ps, time.perf_counter() - t0


def train(rhs, dp, weights_out, n_in, levels, epochs=10, batch=4, lr=5e-4, seed=0, verbose=False):
    """np_cnn_train on the pairs; returns the per-epoch mean loss and the wall
    time."""
    t0 = time.perf_counter()
    hist = B.np_cnn_train(rhs, dp, weights_out, dict(n_in=n_in, levels=levels, epochs=epochs, batch=batch,
                                                      lr=lr, seed=seed, verbose=int(verbose)))
    return hist, time.perf_counter() - t0


def new_net(n_in, levels, seed=0):
    """A caller-owned network with seeded He-normal weights (np_cnn_init)."""
    net = B.Cnn(n_in, levels)
    net.init(seed)
    return net
