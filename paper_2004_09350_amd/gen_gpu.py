"""GPU twin of datagen.py: the same seeded columns, generated directly in HBM.

libmsgen.so evaluates the counter-based SplitMix64 stream per row; the two
distributions that need a running sum (sorted gaps, run ids) use torch.cumsum on
int64.  Tests check these columns against datagen.py bit for bit.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import datagen

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmsgen.so")
if not os.path.exists(_LIB):
    raise ImportError(f"{_LIB} is not built; run __graft_entry__.build()")
_g = ctypes.CDLL(_LIB)
_V, _U64 = ctypes.c_void_p, ctypes.c_uint64
_g.msgen_uniform_bits.argtypes = [_U64, _U64, _U64, ctypes.c_uint, _V, _V]
_g.msgen_uniform_range.argtypes = [_U64, _U64, _U64, _U64, _U64, _V, _V]
_g.msgen_gaps.argtypes = [_U64, _U64, _V, _V]
_g.msgen_run_flags.argtypes = [_U64, _U64, _V, _V]
_g.msgen_run_values.argtypes = [_U64, _V, _U64, _V, _V]


def _s():
    return torch.cuda.current_stream().cuda_stream


def _ok(rc):
    if rc != 0:
        raise RuntimeError(f"libmsgen error {rc}")


def _empty(n):
    return torch.empty(max(n, 4), dtype=torch.int32, device="cuda")


def uniform_bits(seed: int, n: int, b: int) -> torch.Tensor:
    t = _empty(n)
    _ok(_g.msgen_uniform_bits(seed & (2**64 - 1), 0, n, b, t.data_ptr(), _s()))
    return t[:n]


def uniform_range(seed: int, n: int, lo: int, span: int) -> torch.Tensor:
    t = _empty(n)
    _ok(_g.msgen_uniform_range(seed & (2**64 - 1), 0, n, lo, span, t.data_ptr(), _s()))
    return t[:n]


def sorted_gaps(seed: int, n: int) -> torch.Tensor:
    if n == 0:
        return _empty(0)[:0]
    g = torch.empty(n, dtype=torch.int64, device="cuda")
    _ok(_g.msgen_gaps(seed & (2**64 - 1), n, g.data_ptr(), _s()))
    v = torch.cumsum(g, 0)
    del g
    return v.to(torch.int32) if int(v[-1]) < 2**31 else (v - (v >= 2**31).to(torch.int64) * 2**32).to(torch.int32)


def runs(seed: int, n: int) -> torch.Tensor:
    if n == 0:
        return _empty(0)[:0]
    f = torch.empty(n, dtype=torch.int64, device="cuda")
    _ok(_g.msgen_run_flags(seed & (2**64 - 1), n, f.data_ptr(), _s()))
    r = torch.cumsum(f, 0)
    del f
    t = _empty(n)
    _ok(_g.msgen_run_values(seed & (2**64 - 1), r.data_ptr(), n, t.data_ptr(), _s()))
    return t[:n]


def sweep_column(dist: str, seed: int, n: int) -> torch.Tensor:
    if dist.startswith("U"):
        return uniform_bits(seed, n, int(dist[1:]))
    if dist == "SORTED":
        return sorted_gaps(seed, n)
    if dist == "RUNS":
        return runs(seed, n)
    raise ValueError(dist)


def star_columns(seed: int, n_fact: int, dim_sizes=datagen.STAR_DIM_SIZES) -> dict:
    s = datagen.star_seeds(seed)
    cols = {f"fk{d}": uniform_range(s["fk"][d], n_fact, 0, dim_sizes[d]) for d in range(4)}
    cols["m1"] = uniform_range(s["m1"], n_fact, *datagen.STAR_M1)
    cols["m2"] = uniform_range(s["m2"], n_fact, *datagen.STAR_M2)
    for d in range(4):
        cols[f"dimattr{d}"] = uniform_range(s["dimattr"][d], dim_sizes[d], 0, 100)
    cols["dimgroup3"] = (torch.arange(dim_sizes[3], dtype=torch.int32, device="cuda") // 10).to(torch.int32)
    return cols
