"""Seeded synthetic column generators shared by the oracle tests and the GPU path.

This module holds no compression or operator arithmetic: it only turns a seed
and a row index into a uint32 value.  Every generator is counter based, so the
value of row i depends only on (seed, i) and the GPU generator library
(``csrc/datagen.hip``) reproduces the same numbers bit for bit.

Base stream: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  The stream keyed by
``seed`` is x_i = mix64(mix64(seed) + (i + 1) * GAMMA) with the published
constants, i.e. the i-th output of a SplitMix64 generator whose state starts at
mix64(seed).

Distributions (all uint32):
  * uniform_bits(b):        x_i >> (64 - b), uniform in [0, 2^b)
  * uniform_range(lo, span): lo + (((x_i >> 32) * span) >> 32), uniform-ish in [lo, lo + span)
  * sorted_gaps:            v_0 = start, v_i = v_{i-1} + (x_i >> 61) (gaps uniform in [0, 8)),
                            start = x'_0 >> 44 (uniform in [0, 2^20)) from the stream of seed + 1
  * runs:                   row i > 0 starts a new run when (x_i >> 58) == 0 (probability 1/64,
                            so run lengths are geometric with mean 64); run r holds
                            2 * (x'_r >> 49) + (r & 1), x' the stream of seed + 1, so values are
                            in [0, 2^16) and adjacent runs always differ (alternating parity).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * M1
        z = (z ^ (z >> _S27)) * M2
    return z ^ (z >> _S31)


def stream(seed: int, start: int, count: int) -> np.ndarray:
    """x_i for i in [start, start + count) of the counter-based stream keyed by seed."""
    key = mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + idx * GAMMA)


def stream_at(seed: int, idx) -> np.ndarray:
    """x_i of the same stream at arbitrary indices i (for sampled checks of huge columns)."""
    key = mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + (i + np.uint64(1)) * GAMMA)


def uniform_range_at(seed: int, idx, lo: int, span: int) -> np.ndarray:
    """Element idx of uniform_range(seed, n, lo, span), for any n > idx."""
    x = stream_at(seed, idx) >> np.uint64(32)
    with np.errstate(over="ignore"):
        v = (x * np.uint64(span)) >> np.uint64(32)
    return (v + np.uint64(lo)).astype(np.uint32)


def uniform_bits(seed: int, n: int, b: int, start: int = 0) -> np.ndarray:
    if not 0 <= b <= 32:
        raise ValueError("bit width must be in [0, 32]")
    if b == 0:
        return np.zeros(n, dtype=np.uint32)
    return (stream(seed, start, n) >> np.uint64(64 - b)).astype(np.uint32)


def uniform_range(seed: int, n: int, lo: int, span: int, start: int = 0) -> np.ndarray:
    if not (0 < span <= (1 << 32)) or lo < 0 or lo + span > (1 << 32):
        raise ValueError("range must lie inside uint32")
    x = stream(seed, start, n) >> np.uint64(32)
    with np.errstate(over="ignore"):
        v = (x * np.uint64(span)) >> np.uint64(32)
    return (v + np.uint64(lo)).astype(np.uint32)


def sorted_gaps(seed: int, n: int) -> np.ndarray:
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    start = int(stream(seed + 1, 0, 1)[0] >> np.uint64(44))
    g = (stream(seed, 0, n) >> np.uint64(61)).astype(np.uint64)
    g[0] = start
    v = np.cumsum(g, dtype=np.uint64)
    if n and int(v[-1]) >= (1 << 32):
        raise ValueError("sorted column overflows uint32; use fewer rows")
    return v.astype(np.uint32)


def runs(seed: int, n: int) -> np.ndarray:
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    f = ((stream(seed, 0, n) >> np.uint64(58)) == 0).astype(np.uint64)
    f[0] = 0
    r = np.cumsum(f, dtype=np.uint64)
    nr = int(r[-1]) + 1
    u = stream(seed + 1, 0, nr) >> np.uint64(49)
    vals = (np.uint64(2) * u + (np.arange(nr, dtype=np.uint64) & np.uint64(1))).astype(np.uint32)
    return vals[r.astype(np.int64)]


# Named distributions of the operator/format sweep (1e8-row columns in the full workload).
SWEEP_DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")


def sweep_column(dist: str, seed: int, n: int) -> np.ndarray:
    if dist.startswith("U"):
        return uniform_bits(seed, n, int(dist[1:]))
    if dist == "SORTED":
        return sorted_gaps(seed, n)
    if dist == "RUNS":
        return runs(seed, n)
    raise ValueError(f"unknown distribution {dist}")


def he_uniform(seed: int, fan_in: int, count: int) -> np.ndarray:
    """Seeded He-uniform initial weights, float32, in [-sqrt(6/fan_in), sqrt(6/fan_in)).

    u = (x >> 40) / 2^24 is a float in [0, 1) with 24 exact bits; w = (2u - 1) * limit.
    """
    u = (stream(seed, 0, count) >> np.uint64(40)).astype(np.float64) / float(1 << 24)
    limit = np.sqrt(6.0 / fan_in)
    return ((2.0 * u - 1.0) * limit).astype(np.float32)



def mlp_init(seed: int) -> np.ndarray:
    """Initial parameters of the 32-64-64-6 selector network, float32[6662]:
    He-uniform weights (seeds seed, seed+1, seed+2 for the three layers), zero biases,
    in the order W1[64][32], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]."""
    return np.concatenate([he_uniform(seed, 32, 64 * 32), np.zeros(64, np.float32),
                           he_uniform(seed + 1, 64, 64 * 64), np.zeros(64, np.float32),
                           he_uniform(seed + 2, 64, 6 * 64), np.zeros(6, np.float32)])

# Star-style query workload: fact table with four foreign keys and two measures,
# four dimensions with a filter attribute each; dimension 3 also carries a
# 250-valued group attribute (floor(k / 10) over 2,500 rows).
STAR_DIM_SIZES = (200_000, 3_000_000, 2_000_000, 2_500)
STAR_M1 = (1, 100_000 - 1)      # m1 uniform in [1, 1e5)
STAR_M2 = (0, 11)               # m2 uniform in [0, 10]
STAR_GROUPS = 250
STAR_WIDE = (0.20, 0.20, 0.20, 0.20)
STAR_NARROW = (0.01, 0.05, 0.10, 0.20)


def star_seeds(seed: int) -> dict:
    """Per-column seeds of one star workload instance."""
    b = 1000 * seed
    return dict(fk=[b + d for d in range(4)], m1=b + 10, m2=b + 11, dimattr=[b + 20 + d for d in range(4)])


def star_columns(seed: int, n_fact: int, dim_sizes=STAR_DIM_SIZES) -> dict:
    s = star_seeds(seed)
    cols = {f"fk{d}": uniform_range(s["fk"][d], n_fact, 0, dim_sizes[d]) for d in range(4)}
    cols["m1"] = uniform_range(s["m1"], n_fact, STAR_M1[0], STAR_M1[1])
    cols["m2"] = uniform_range(s["m2"], n_fact, STAR_M2[0], STAR_M2[1])
    for d in range(4):
        cols[f"dimattr{d}"] = uniform_range(s["dimattr"][d], dim_sizes[d], 0, 100)
    cols["dimgroup3"] = (np.arange(dim_sizes[3], dtype=np.uint32) // 10).astype(np.uint32)
    return cols


def star_thresholds(sel) -> list:
    """Filter constants: dimension rows with attribute < floor(100 * s_d) qualify."""
    return [int(np.floor(100 * s + 1e-9)) for s in sel]
