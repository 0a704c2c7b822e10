"""Learned format selection (section 5.2: formats chosen per intermediate by a cost model
over data characteristics; exhaustive selection, whose per-column optimum is the plan
optimum because footprints add up, is the reference its regret is measured against).

The engine produces its own training data: it runs star-query plans (the shape of the
evaluation workload, with other seeds, sizes and selectivities), and for every
intermediate records the 32 statistics (``ms_stats``) and the exact footprint in each
format (``ms_footprints``).  The network (32-64-64-6, ReLU) learns
t_f = log2(1 + 8 * footprint_f / n) / 6, the log-scaled bits per value of format f,
with the library's own gradient and Adam kernels; the pick is the smallest output.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import datagen
from . import gen_gpu as gen
from . import morphgpu as M
from .queries import Q3, Q3_INPUTS

TARGET_SCALE = 6.0


def targets(fp6: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Training targets from exact footprints (bytes) and element counts."""
    n = np.maximum(np.asarray(n, np.float64), 1.0)[:, None]
    return (np.log2(1.0 + 8.0 * np.asarray(fp6, np.float64) / n) / TARGET_SCALE).astype(np.float32)


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
            s_hi: float = 0.20, plans_per_seed: int = 8, log=None):
    """Statistics, footprints and sizes of every intermediate of `n_plans` star plans.
    Plan j uses seed seed0 + j // plans_per_seed for its dimensions (shared by a group of
    plans) and its own fact seed, size (log-uniform) and selectivities (uniform)."""
    X, F, N, names = [], [], [], []
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
            N.append(q.plan.column(q.names[name]).info()["n"])
            names.append(name)
        q.plan.close()
        del cols, q
        if log and (j + 1) % 100 == 0:
            log(f"collected {j + 1}/{n_plans} plans, {len(X)} intermediates, {time.time() - t0:.1f}s")
    return np.stack(X), np.stack(F).astype(np.uint64), np.asarray(N, np.uint64), names


def train(X: np.ndarray, T: np.ndarray, epochs: int = 60, batch: int = 512, lr: float = 2e-3, seed: int = 77,
          log=None) -> torch.Tensor:
    """Mini-batch Adam on the GPU with the library's gradient and update kernels."""
    p = torch.from_numpy(datagen.mlp_init(seed)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T, np.float32)).cuda()
    n = Xd.shape[0]
    order_seed = seed
    step = 0
    g = torch.empty_like(p)
    for ep in range(epochs):
        perm = torch.from_numpy(np.argsort(datagen.stream(order_seed + ep, 0, n))).cuda()
        losses = []
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            xb, tb = Xd[idx].contiguous(), Td[idx].contiguous()
            _, loss = M.mlp_grad(p, xb, tb, grad=g)
            step += 1
            M.adam_step(p, g, m, v, step, lr=lr)
            losses.append(loss)
        if log and (ep + 1) % 10 == 0:
            log(f"epoch {ep + 1}: mean batch loss {float(torch.stack(losses).mean()):.3e}")
    return p


def save(params: torch.Tensor, path: str):
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load(path: str) -> torch.Tensor:
    p = np.load(path, allow_pickle=False)
    if p.shape != (M.MLP_NPARAM,) or p.dtype != np.float32:
        raise ValueError(f"{path}: expected float32[{M.MLP_NPARAM}]")
    return torch.from_numpy(p).cuda()


def pick(params: torch.Tensor, X: np.ndarray) -> np.ndarray:
    _, k = M.mlp_forward(params, torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda(), want_y=False)
    return k.cpu().numpy()


def regret(F: np.ndarray, picks: np.ndarray) -> float:
    """Sum of picked footprints over the sum of the least footprints, minus one."""
    F = np.asarray(F, np.float64)
    best = F.min(axis=1).sum()
    got = F[np.arange(F.shape[0]), picks].sum()
    return float(got / best - 1.0) if best > 0 else 0.0
