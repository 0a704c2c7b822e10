"""Element-by-element parity on the paths where every wave walks many chunks.

The persistent grid gives a workgroup min(ceil(C/4), CUs x wg_per_cu) segments' worth of
chunks; at the default shape a 1e6-row column leaves each wave one or two chunks.  Here
every operator runs as a step of a plan launched with one branch and one workgroup per
CU (set_tune(1, 1)) over columns of about 1e7 rows with ragged tails, so a wave walks
~19 chunks: the steady-state window look-ahead and directory prefetch, the per-wave RLE
quarter walk with its run ring, the emit phase's eight-chunk units, blocks shared by
neighbouring waves (the fix-up kernel) and the narrowing pass of automatic-width static
BP outputs.  Every output is compared with the oracle's encoding of the expected values
block by block (widths, bases, payload words, remainder, runs, footprint).
"""
import numpy as np
import pytest

import oracle as O
from paper_2004_09350_amd import datagen
from tests._parity import assert_column

pytestmark = pytest.mark.gpu

N = 10_000_037          # 19 531 full 512-blocks + 165 rows (and 5 past a multiple of 32)
DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")
TUNE = (1, 1)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu
    morphgpu.init()
    return morphgpu


def run_plan(M, steps, inputs):
    plan = M.Plan(steps, inputs)
    plan.set_tune(*TUNE)
    plan.run()
    M.sync()
    return plan


def quantile_threshold(v, s):
    return int(np.sort(v)[min(v.size - 1, int(s * v.size))])


def thresholds(dist, v):
    if dist.startswith("U"):
        b = int(dist[1:])
        return [max(1, round(s * (1 << b))) if b < 32 else int(s * (1 << 32)) for s in (0.1, 0.5)]
    if dist == "RUNS":
        return [int(s * (1 << 16)) for s in (0.1, 0.5)]
    return [quantile_threshold(v, s) for s in (0.1, 0.5)]


@pytest.mark.parametrize("dist", DISTS)
def test_select_project_morph_multichunk(M, dist):
    """select (10 % and 50 %) and project from every input format into every output
    format, and morph between every ordered pair, each as a plan step."""
    v = datagen.sweep_column(dist, 8000 + DISTS.index(dist), N)
    cols = [M.encode(v, M.fmt(k)) for k in O.KINDS]
    enc_src = datagen.uniform_bits(8100, N, 12)
    pos = O.select(enc_src, O.LT, 410)
    P = M.encode(pos, M.fmt(M.DELTA_DYN_BP))
    steps, expect = [], []
    for kin in O.KINDS:
        for c in thresholds(dist, v):
            for kout in O.KINDS:
                steps.append(M.step(M.OP_SELECT, a=M.inp(kin), cmp=M.LT, c0=c, out=M.fmt(kout)))
                expect.append(("sel", c, kout, f"select {dist} {kin}->{kout} v<{c}"))
        for kout in O.KINDS:
            steps.append(M.step(M.OP_PROJECT, a=M.inp(kin), b=M.inp(6), out=M.fmt(kout)))
            expect.append(("prj", None, kout, f"project {dist} {kin}->{kout}"))
        for kout in O.KINDS:
            if kout != kin:
                steps.append(M.step(M.OP_MORPH, a=M.inp(kin), out=M.fmt(kout)))
                expect.append(("mor", None, kout, f"morph {dist} {kin}->{kout}"))
    plan = run_plan(M, steps, cols + [P])
    sel_cache = {}
    proj = O.project(v, pos)
    for i, (what, c, kout, label) in enumerate(expect):
        if what == "sel":
            if c not in sel_cache:
                sel_cache[c] = O.select(v, O.LT, c)
            want = sel_cache[c]
        elif what == "prj":
            want = proj
        else:
            want = v
        try:
            assert_column(plan.column(i), want, kout)
        except AssertionError as e:
            raise AssertionError(f"{label}: {e}") from None
    plan.close()
    M.sync()


def test_select_emit_step_forms_multichunk(M):
    """The emit phase's forms of a 4096-row step, each reached in one column: the per-lane
    loop over a whole step of 512..1536 outputs (uniform 25 % and 35 %), the two halves or
    chunk by chunk (uniform 40 %), row planes and halves of different density (a column
    whose density alternates between 70 % and 15 % every 4096 rows, so that steps straddle
    the change at every offset), into every output format."""
    u = datagen.uniform_bits(8500, N, 12)
    i = np.arange(N, dtype=np.int64)
    alt = np.where((i // 4096) % 2 == 0, u % 1429, u + 400).astype(np.uint32)  # v < 1000: 70 % / 15 %
    cols = [M.encode(u, M.fmt(M.STATIC_BP)), M.encode(alt, M.fmt(M.STATIC_BP))]
    cases = [(0, 1024), (0, 1434), (0, 1638), (1, 1000)]
    steps, expect = [], []
    for j, c in cases:
        for kout in O.KINDS:
            steps.append(M.step(M.OP_SELECT, a=M.inp(j), cmp=M.LT, c0=c, out=M.fmt(kout)))
            expect.append((j, c, kout))
    plan = run_plan(M, steps, cols)
    vals = (u, alt)
    want = {(j, c): O.select(vals[j], O.LT, c) for j, c in cases}
    for k, (j, c, kout) in enumerate(expect):
        try:
            assert_column(plan.column(k), want[(j, c)], kout)
        except AssertionError as e:
            raise AssertionError(f"select column {j} v<{c} -> {kout}: {e}") from None
    plan.close()
    M.sync()


@pytest.mark.parametrize("D", [200_000, 3_000_000])
def test_semijoin_multichunk(M, D):
    """dimension select -> bitmap -> semi-join of keys stored in every format, into
    every output format (D = 2e5: bitmap in LDS; 3e6: the first 2^18 bits in LDS, the
    rest probed through the caches)."""
    keys = datagen.uniform_range(8200 + D % 7, N, 0, D + D // 50)   # 2 % of keys fall outside the domain
    attr = datagen.uniform_range(8300, D, 0, 100)
    S = O.select(attr, O.LT, 20)
    want = O.semijoin(keys, O.bitmap_from_positions(S, D), D)
    cols = [M.encode(keys, M.fmt(k)) for k in O.KINDS] + [M.encode(attr, M.fmt(M.STATIC_BP))]
    steps = [M.step(M.OP_SELECT, a=M.inp(6), cmp=M.LT, c0=20, out=M.fmt(M.DELTA_DYN_BP)),
             M.step(M.OP_BITMAP, a=0, param=D)]
    idx = []
    for kin in O.KINDS:
        for kout in O.KINDS:
            steps.append(M.step(M.OP_SEMIJOIN, a=M.inp(kin), b=1, param=D, out=M.fmt(kout)))
            idx.append((len(steps) - 1, kin, kout))
    plan = run_plan(M, steps, cols)
    np.testing.assert_array_equal(plan.read(1), O.bitmap_from_positions(S, D))
    for i, kin, kout in idx:
        try:
            assert_column(plan.column(i), want, kout)
        except AssertionError as e:
            raise AssertionError(f"semijoin D={D} {kin}->{kout}: {e}") from None
    plan.close()
    M.sync()


def test_intersect_multichunk(M):
    """P_a (10 %) in every format against P_b (50 %), in both operand orders, into every
    output format."""
    a = datagen.uniform_bits(8400, N, 12)
    b = datagen.uniform_bits(8401, N, 12)
    pa, pb = O.select(a, O.LT, 410), O.select(b, O.LT, 2048)
    want = O.intersect(pa, pb)
    inputs = [M.encode(pa, M.fmt(k)) for k in O.KINDS] + [M.encode(pb, M.fmt(M.DELTA_DYN_BP))]
    steps, idx = [], []
    for kin in O.KINDS:
        for kout in O.KINDS:
            steps.append(M.step(M.OP_INTERSECT, a=M.inp(kin), b=M.inp(6), param=N, out=M.fmt(kout)))
            idx.append((len(steps) - 1, kin, kout, "a&b"))
        steps.append(M.step(M.OP_INTERSECT, a=M.inp(6), b=M.inp(kin), param=N, out=M.fmt(M.DELTA_DYN_BP)))
        idx.append((len(steps) - 1, kin, M.DELTA_DYN_BP, "b&a"))
    plan = run_plan(M, steps, inputs)
    for i, kin, kout, order in idx:
        try:
            assert_column(plan.column(i), want, kout)
        except AssertionError as e:
            raise AssertionError(f"intersect {order} {kin}->{kout}: {e}") from None
    plan.close()
    M.sync()


@pytest.mark.parametrize("G", [250, 10_000])
def test_sum_and_group_sum_multichunk(M, G):
    """sum of every format and group-sum (LDS histograms for 250 groups, global atomics
    for 10 000) with many chunks per wave."""
    g = datagen.uniform_range(8500 + G, N, 0, G)
    v = datagen.uniform_bits(8501, N, 20)
    runs = datagen.runs(8502, N)
    inputs = [M.encode(v, M.fmt(k)) for k in O.KINDS] + [M.encode(runs, M.fmt(k)) for k in O.KINDS]
    inputs += [M.encode(g, M.fmt(k)) for k in (M.STATIC_BP, M.RLE)]
    steps = [M.step(M.OP_SUM, a=M.inp(j)) for j in range(12)]
    steps += [M.step(M.OP_GROUP_SUM, a=M.inp(12), b=M.inp(k), param=G) for k in O.KINDS]
    steps.append(M.step(M.OP_GROUP_SUM, a=M.inp(13), b=M.inp(3), param=G))
    plan = run_plan(M, steps, inputs)
    for j in range(12):
        want = O.sum_(v if j < 6 else runs)
        assert int(plan.read(j)[0]) == want, f"sum input {j}"
    want = O.group_sum(g, v, G)
    for k in range(12, len(steps)):
        np.testing.assert_array_equal(plan.read(k), want, err_msg=f"group-sum step {k}")
    plan.close()
    M.sync()
