"""Train the format-selector network on the GPU from intermediates the engine produces.

    python -m paper_2004_09350_amd.train_selector --plans 13334 --out selector_weights.npy

Runs `--plans` star-query plans (fact rows log-uniform in [1e5, 1e7], filter
selectivities uniform in [1 %, 20 %], seeds from 10000 on, disjoint from the
evaluation seeds), records the 32 statistics and the exact six-format footprints of
every intermediate, trains the 32-64-64-6 network with the library's kernels and
writes its parameters (float32[6662], numpy .npy without pickling).  Prints the
training-set regret against exhaustive selection.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--plans", type=int, default=13_334)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed0", type=int, default=10_000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--data-out", default=None, help="also save the training set (.npz)")
    a = ap.parse_args(argv)
    from . import morphgpu as M
    from . import selector as S
    M.init()
    log = lambda *x: print(*x, flush=True)
    t0 = time.time()
    X, F, N, names = S.collect(a.plans, seed0=a.seed0, log=log)
    log(f"collected {len(X)} intermediates from {a.plans} plans in {time.time() - t0:.1f}s")
    if a.data_out:
        np.savez(a.data_out, X=X, F=F, N=N)
    T = S.targets(F, N)
    t1 = time.time()
    p = S.train(X, T, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    M.sync()
    log(f"trained {a.epochs} epochs in {time.time() - t1:.1f}s")
    picks = S.pick(p, X)
    log(f"training-set regret {S.regret(F, picks):.5f}; exact picks {np.mean(picks == F.argmin(axis=1)):.4f}")
    S.save(p, a.out)
    log(f"wrote {a.out}")


if __name__ == "__main__":
    sys.exit(main())
