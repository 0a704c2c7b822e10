"""The oracle's star query evaluated over fact-row chunks (test infrastructure).

The star plan is row-local up to its additive group-sums: on a horizontal slice of the
fact table, selects, semi-joins, intersects and projections give exactly that slice's
part of every intermediate (positions shifted by the slice's first row), and the
group-sums of the slices add up to the whole table's.  So a fact table too large for
one oracle pass is evaluated slice by slice, in parallel threads (numpy's generators and
the C oracle release the interpreter lock), and the parts are concatenated or added.
Inputs come from the numpy generators only.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle.queries as OQ
from paper_2004_09350_amd import datagen

WORKERS = max(1, min(16, os.cpu_count() or 1))


def oracle_star_chunk(seed, r0, r1, thr):
    """The oracle's star query over fact rows [r0, r1): (P + r0, out1, out2)."""
    s = datagen.star_seeds(seed)
    D = datagen.STAR_DIM_SIZES
    n = r1 - r0
    cols = {f"fk{d}": datagen.uniform_range(s["fk"][d], n, 0, D[d], start=r0) for d in range(4)}
    cols["m1"] = datagen.uniform_range(s["m1"], n, *datagen.STAR_M1, start=r0)
    cols["m2"] = datagen.uniform_range(s["m2"], n, *datagen.STAR_M2, start=r0)
    for d in range(4):
        cols[f"dimattr{d}"] = datagen.uniform_range(s["dimattr"][d], D[d], 0, 100)
    cols["dimgroup3"] = (np.arange(D[3], dtype=np.uint32) // 10).astype(np.uint32)
    r = OQ.q3(cols, thr, D)
    P = (r["intermediates"]["P"].astype(np.uint64) + np.uint64(r0)).astype(np.uint32)
    return P, r["out1"], r["out2"]


def oracle_star(seed, n, thr, chunk=25_000_000):
    """(P, out1, out2) of the star query over n fact rows, evaluated chunk by chunk."""
    bounds = [(r0, min(n, r0 + chunk)) for r0 in range(0, n, chunk)]
    with ThreadPoolExecutor(WORKERS) as ex:
        parts = list(ex.map(lambda b: oracle_star_chunk(seed, b[0], b[1], thr), bounds))
    P = np.concatenate([p for p, _, _ in parts]) if parts else np.zeros(0, np.uint32)
    with np.errstate(over="ignore"):
        out1 = np.sum(np.stack([o for _, o, _ in parts]), axis=0, dtype=np.uint64)
        out2 = np.sum(np.stack([o for _, _, o in parts]), axis=0, dtype=np.uint64)
    return P, out1, out2
