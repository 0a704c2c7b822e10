"""Train the format selector's two networks on the GPU from intermediates the engine produces.

    python -m paper_2004_09350_amd.train_selector --plans 13334 --cost-plans 3000 --out selector.msw

Runs `--plans` star-query plans (fact rows log-uniform in [1e5, 1e7], filter
selectivities uniform in [1 %, 20 %], seeds from 10000 on, disjoint from the evaluation
seeds) and records the 32 statistics and the exact six-format footprints of every
intermediate; for the intermediates of the first `--cost-plans` plans it also measures the
decode time of each format.  The library computes the targets and trains the size network
on all intermediates and the decode-cost network on the timed ones, then the selector is
written in the library's file format.  Prints the training-set regrets against the
exhaustive choice (footprint) and against the fastest measured format (decode time).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--plans", type=int, default=13_334)
    ap.add_argument("--cost-plans", type=int, default=3_000)
    ap.add_argument("--cost-reps", type=int, default=5, help="timed decodes per format and intermediate")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed0", type=int, default=10_000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--data-out", default=None, help="also save the training set (.npz)")
    a = ap.parse_args(argv)
    import torch

    from . import morphgpu as M
    from . import selector as S
    M.init()
    log = lambda *x: print(*x, flush=True)
    t0 = time.time()
    nc = min(a.cost_plans, a.plans)
    Xc, Fc, Nc, C, _ = S.collect(nc, seed0=a.seed0, cost_labels=True, cost_reps=a.cost_reps, log=log)
    log(f"collected {len(Xc)} timed intermediates from {nc} plans in {time.time() - t0:.1f}s")
    if a.plans > nc:
        Xr, Fr, Nr, _, _ = S.collect(a.plans - nc, seed0=a.seed0 + 1_000_000, log=log)
        X, F, N = np.concatenate([Xc, Xr]), np.concatenate([Fc, Fr]), np.concatenate([Nc, Nr])
    else:
        X, F, N = Xc, Fc, Nc
    log(f"collected {len(X)} intermediates from {a.plans} plans in {time.time() - t0:.1f}s")
    if a.data_out:
        np.savez(a.data_out, X=X, F=F, N=N, Xc=Xc, Nc=Nc, C=C)
    t1 = time.time()
    sel = S.new_selector()
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    loss = sel.train(M.NET_SIZE, x, M.size_targets(F, N), epochs=a.epochs, batch=a.batch, lr=a.lr, seed=S.INIT_SEED)
    log(f"size network: last-pass loss {loss:.3e}")
    xc = torch.from_numpy(np.ascontiguousarray(Xc, np.float32)).cuda()
    loss = sel.train(M.NET_COST, xc, M.cost_targets(C, Nc), epochs=a.epochs, batch=a.batch, lr=a.lr,
                     seed=S.INIT_SEED + 1)
    log(f"decode-cost network: last-pass loss {loss:.3e}")
    M.sync()
    log(f"trained {a.epochs} epochs in {time.time() - t1:.1f}s")
    picks = S.pick(sel, X)
    log(f"training-set footprint regret {S.regret(F, picks):.5f}; "
        f"exact picks {np.mean(picks == S.exhaustive(F)):.4f}")
    dp = S.pick(sel, Xc, M.OBJ_DECODE)
    dec = C[np.arange(len(C)), dp].sum() / C.min(axis=1).sum() - 1
    log(f"training-set decode-time regret {dec:.5f}; "
        f"fastest picks {np.mean(C[np.arange(len(C)), dp] == C.min(axis=1)):.4f}")
    sel.save(a.out)
    log(f"wrote {a.out}")


if __name__ == "__main__":
    sys.exit(main())
