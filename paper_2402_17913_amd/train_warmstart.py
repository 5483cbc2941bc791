"""Trains the learned warm start for 3D periodic projection steps and writes
the weight file the solver loads with np_cnn_load.

Default recipe: 256^3 periodic grid on [0, 2pi)^3, nu = 1e-3, seeds 1..20
(seed 0 is held out for evaluation), 100 projection steps per seed -> 2000
(rhs, dp) pairs, restricted on the device to the 128^3 network input; a
4-level, 16-channel network trained for 8 epochs (Adam, lr 5e-4, batch 4).

    python -m paper_2402_17913_amd.train_warmstart [--out PATH] [--seeds 1-20] ...
"""
import argparse
import json
import os
import sys
import time

import torch

from . import binding as B
from . import learned

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "ns3d_periodic_256_in128_L4.npcnn")


def seed_range(s):
    a, _, b = s.partition("-")
    return list(range(int(a), int(b or a) + 1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seeds", type=seed_range, default=seed_range("1-20"))
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--n-in", type=int, default=128)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("training needs a GPU")

    def log(msg):
        print(msg, flush=True)

    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    log("generating %d x %d pairs on %d^3 (kept at %d^3)" % (len(a.seeds), a.steps, a.n, a.n_in))
    rs, ps, tgen = learned.make_pairs(a.n, a.seeds, a.steps, a.n_in, log=log)
    log("generated %d pairs in %.1f s; training %d epochs" % (len(rs), tgen, a.epochs))
    hist, ttrain = learned.train(rs, ps, a.out, a.n_in, a.levels, epochs=a.epochs, batch=a.batch, lr=a.lr,
                                 seed=a.seed, verbose=True)
    for ep, l in enumerate(hist):
        log("  epoch %d  mean mse %.4e" % (ep, l))
    report = dict(grid=a.n, seeds=[a.seeds[0], a.seeds[-1]], steps_per_seed=a.steps, pairs=len(rs), n_in=a.n_in,
                  levels=a.levels, epochs=a.epochs, batch=a.batch, lr=a.lr, init_seed=a.seed, epoch_loss=hist,
                  pair_generation_s=round(tgen, 2), training_s=round(ttrain, 2),
                  device=torch.cuda.get_device_name(0))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fp:
        json.dump(report, fp, indent=1)
    log("wrote %s (%.1f s training)" % (a.out, ttrain))
    del rs, ps
    B.np_release_all()


if __name__ == "__main__":
    main()
