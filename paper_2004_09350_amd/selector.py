"""Learned format selection (section 5.2: formats chosen per intermediate by a cost model
over data characteristics that estimates both the compression rate and the decompression
performance; exhaustive selection, whose per-column optimum is the plan optimum because
footprints add up, is the reference its regret is measured against).

The engine produces its own training data: it runs star-query plans (the shape of the
evaluation workload, with other seeds, sizes and selectivities), and for every
intermediate records the 32 statistics (``ms_stats``), the exact footprint in each
format (``ms_footprints``) and, on request, the measured decode time of each format
(``ms_decode_cost``).  The library turns those labels into targets, trains its two
32-64-64-6 networks (size, decode cost) with its own gradient and Adam kernels and picks
formats (``ms_selector_*``); this module only drives the plans and moves arrays.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import torch

from . import datagen
from . import gen_gpu as gen
from . import morphgpu as M
from .queries import Q3, Q3_INPUTS

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "selector.msw")
INIT_SEED = 77


def new_selector(seed: int = INIT_SEED) -> M.Selector:
    """Both networks at their seeded He-uniform initialisation (size: seed, cost: seed + 100)."""
    return M.Selector.create(datagen.mlp_init(seed), datagen.mlp_init(seed + 100))


def star_inputs(seed: int, n_fact: int, fact_fmt=None, dims=None):
    """Base columns of one star instance on the GPU, encoded (static BP by default).
    `dims` reuses already encoded dimension columns."""
    fact_fmt = fact_fmt if fact_fmt is not None else M.fmt(M.STATIC_BP)
    s = datagen.star_seeds(seed)
    D = datagen.STAR_DIM_SIZES
    cols = {}
    for d in range(4):
        cols[f"fk{d}"] = M.encode(gen.uniform_range(s["fk"][d], n_fact, 0, D[d]), fact_fmt)
    cols["m1"] = M.encode(gen.uniform_range(s["m1"], n_fact, *datagen.STAR_M1), fact_fmt)
    cols["m2"] = M.encode(gen.uniform_range(s["m2"], n_fact, *datagen.STAR_M2), fact_fmt)
    if dims is None:
        dims = {}
        for d in range(4):
            dims[f"dimattr{d}"] = M.encode(gen.uniform_range(s["dimattr"][d], D[d], 0, 100), M.fmt(M.STATIC_BP))
        g = (torch.arange(D[3], dtype=torch.int32, device="cuda") // 10).to(torch.int32)
        dims["dimgroup3"] = M.encode(g, M.fmt(M.STATIC_BP))
    cols.update(dims)
    return cols, dims


def collect(n_plans: int, seed0: int = 10_000, n_lo: float = 1e5, n_hi: float = 1e7, s_lo: float = 0.01,
            s_hi: float = 0.20, plans_per_seed: int = 8, cost_labels: bool = False, cost_reps: int = 3, log=None):
    """Statistics, footprints and sizes (and decode times when cost_labels) of every
    intermediate of `n_plans` star plans.  Plan j uses seed seed0 + j // plans_per_seed for
    its dimensions (shared by a group of plans) and its own fact seed, size (log-uniform)
    and selectivities (uniform).  Returns X (k x 32 float32), F (k x 6 uint64 bytes),
    N (k uint64), C (k x 6 float32 ns per decode, or None) and the intermediates' names."""
    X, F, N, C, names = [], [], [], [], []
    dims, dims_seed = None, None
    t0 = time.time()
    for j in range(n_plans):
        dseed = seed0 + j // plans_per_seed
        u = datagen.stream(seed0 * 7919 + j, 0, 5).astype(np.float64) / 2.0 ** 64
        n_fact = int(math.exp(math.log(n_lo) + u[0] * (math.log(n_hi) - math.log(n_lo))))
        sel = [s_lo + (s_hi - s_lo) * x for x in u[1:5]]
        if dseed != dims_seed:
            dims, dims_seed = None, dseed
        cols, dims = star_inputs(dseed * 100 + (j % plans_per_seed) + 1, n_fact, dims=dims)
        q = Q3(cols, datagen.star_thresholds(sel), datagen.STAR_DIM_SIZES, n_fact, extra=("stats", "footprints"))
        q.plan.run()
        for name in q.names:
            X.append(q.plan.read(q.stats_step[name]))
            F.append(q.plan.read(q.fp_step[name]))
            col = q.plan.column(q.names[name])
            N.append(col.info()["n"])
            if cost_labels:
                C.append(M.decode_cost(col, cost_reps))
            names.append(name)
        q.plan.close()
        del cols, q
        if log and (j + 1) % 100 == 0:
            log(f"collected {j + 1}/{n_plans} plans, {len(X)} intermediates, {time.time() - t0:.1f}s")
    return (np.stack(X), np.stack(F).astype(np.uint64), np.asarray(N, np.uint64),
            np.stack(C).astype(np.float32) if cost_labels else None, names)


def train(X: np.ndarray, F: np.ndarray, N: np.ndarray, C: np.ndarray | None = None, epochs: int = 60,
          batch: int = 512, lr: float = 2e-3, seed: int = INIT_SEED, log=None) -> M.Selector:
    """A selector trained on the GPU by the library: the size network on the footprints'
    targets, and the decode-cost network on the decode times' targets when C is given."""
    sel = new_selector(seed)
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    loss = sel.train(M.NET_SIZE, x, M.size_targets(F, N), epochs=epochs, batch=batch, lr=lr, seed=seed)
    if log:
        log(f"size network: last-pass loss {loss:.3e}")
    if C is not None:
        loss = sel.train(M.NET_COST, x, M.cost_targets(C, N), epochs=epochs, batch=batch, lr=lr, seed=seed + 1)
        if log:
            log(f"decode-cost network: last-pass loss {loss:.3e}")
    return sel


def load(path: str = WEIGHTS) -> M.Selector:
    return M.Selector.load(path)


def pick(sel: M.Selector, X: np.ndarray, objective: int = M.OBJ_FOOTPRINT) -> np.ndarray:
    return sel.pick(np.ascontiguousarray(X, np.float32), objective).cpu().numpy()


def exhaustive(F: np.ndarray) -> np.ndarray:
    """The library's exhaustive choice for rows of footprints (ties to the lower kind)."""
    return M.select_argmin(np.asarray(F, np.uint64)).cpu().numpy()


def regret(F: np.ndarray, picks: np.ndarray) -> float:
    """Sum of the picked costs over the sum of the exhaustive choice's, minus one."""
    F = np.asarray(F, np.float64)
    rows = np.arange(F.shape[0])
    best = F[rows, exhaustive(F.astype(np.uint64))].sum()
    got = F[rows, np.asarray(picks)].sum()
    return float(got / best - 1.0) if best > 0 else 0.0
