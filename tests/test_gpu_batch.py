"""A mixed batch in one plan against the oracle: 64 independent tasks of every operator
(select, semi-join, project, intersect, sum, group-sum, morph), every input and output
format, every value distribution and sizes log-uniform over three decades, run eagerly,
as a captured graph with the autotuned launch shape (replayed several times with other
work in between), with one launch sequence per task on eight branches, and with batched
persistent launches (one launch per kernel and phase for each of the plan's levels, eager
and as a replayed graph).  Every column
result is compared block by block with the oracle's encoding of the expected values."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2004_09350_amd import datagen
from tests._parity import assert_column

pytestmark = pytest.mark.gpu

T = 64
DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")
OPS = ("select", "semijoin", "project", "intersect", "sum", "group_sum", "morph")


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu
    morphgpu.init()
    return morphgpu


def build(M):
    """Steps, inputs and the oracle's expected result of every task."""
    u = (datagen.stream(7777, 0, 8 * T).astype(np.float64) / 2.0 ** 64).reshape(T, 8)
    steps, inputs, expect = [], [], []

    def add_input(values, kind):
        inputs.append(M.encode(values, M.fmt(kind)))
        return M.inp(len(inputs) - 1)

    for t in range(T):
        n = int(math.exp(math.log(2e3) + u[t, 0] * (math.log(2e6) - math.log(2e3))))
        op = OPS[t % len(OPS)]  # every operator about equally often, in a mixed order
        dist = DISTS[int(u[t, 2] * 6)]
        kin, kout = int(u[t, 3] * 6), int(u[t, 4] * 6)
        v = datagen.sweep_column(dist, 90_000 + t, n)
        if op == "select":
            c = int(np.sort(v)[min(n - 1, int(u[t, 5] * n))])
            steps.append(M.step(M.OP_SELECT, a=add_input(v, kin), cmp=M.LT, c0=c, out=M.fmt(kout)))
            expect.append(("col", O.select(v, O.LT, c), kout))
        elif op == "semijoin":
            D = 1 + int(u[t, 5] * 300_000)
            keys = datagen.uniform_range(91_000 + t, n, 0, D + D // 8)  # some keys out of the domain
            dim = datagen.uniform_range(92_000 + t, D, 0, 100)
            s = O.select(dim, O.LT, 30)
            a = add_input(keys, kin)
            steps.append(M.step(M.OP_SELECT, a=add_input(dim, M.STATIC_BP), cmp=M.LT, c0=30, out=M.fmt(M.DELTA_DYN_BP)))
            expect.append(("col", s, M.DELTA_DYN_BP))
            steps.append(M.step(M.OP_BITMAP, a=len(steps) - 1, param=D))
            expect.append(("bitmap", O.bitmap_from_positions(s, D), None))
            steps.append(M.step(M.OP_SEMIJOIN, a=a, b=len(steps) - 1, param=D, out=M.fmt(kout)))
            expect.append(("col", O.semijoin(keys, O.bitmap_from_positions(s, D), D), kout))
        elif op == "project":
            pos = datagen.uniform_range(93_000 + t, max(1, n // 7), 0, n)  # unsorted, with repeats
            steps.append(M.step(M.OP_PROJECT, a=add_input(v, kin), b=add_input(pos, M.DELTA_DYN_BP if kin % 2 else
                                                                                 M.STATIC_BP), out=M.fmt(kout)))
            expect.append(("col", O.project(v, pos), kout))
        elif op == "intersect":
            pa = O.select(datagen.uniform_bits(94_000 + t, n, 12), O.LT, 410)
            pb = O.select(datagen.uniform_bits(95_000 + t, n, 12), O.LT, 2048)
            ka = kin if kin != M.RLE else M.DYN_BP
            steps.append(M.step(M.OP_INTERSECT, a=add_input(pa, ka), b=add_input(pb, M.DELTA_DYN_BP), param=n,
                                out=M.fmt(kout)))
            expect.append(("col", O.intersect(pa, pb), kout))
        elif op == "sum":
            steps.append(M.step(M.OP_SUM, a=add_input(v, kin)))
            expect.append(("u64", np.array([O.sum_(v)], np.uint64), None))
        elif op == "group_sum":
            G = 1 + int(u[t, 5] * 3000)
            g = datagen.uniform_range(96_000 + t, n, 0, G)
            steps.append(M.step(M.OP_GROUP_SUM, a=add_input(g, kin), b=add_input(v, kout), param=G))
            expect.append(("u64", O.group_sum(g, v, G), None))
        else:
            steps.append(M.step(M.OP_MORPH, a=add_input(v, kin), out=M.fmt(kout)))
            expect.append(("col", v, kout))
    return steps, inputs, expect


def check(M, plan, expect):
    for i, (what, want, kind) in enumerate(expect):
        if what == "col":
            assert_column(plan.column(i), want, kind)
        elif what == "u64":
            np.testing.assert_array_equal(plan.read(i).astype(np.uint64), want, err_msg=f"step {i}")
        else:
            np.testing.assert_array_equal(plan.read(i)[: want.size].astype(np.uint32), want, err_msg=f"step {i}")


def test_mixed_batch_eager_graph_and_branches(M, tmp_path):
    steps, inputs, expect = build(M)
    plan = M.Plan(steps, inputs)
    plan.run()
    M.sync()
    check(M, plan, expect)
    best, _ = plan.autotune(reps=1, cache=str(tmp_path / "tune.txt"))
    other = M.encode(datagen.uniform_bits(3, 100_001, 9), M.fmt(M.FOR_DYN_BP))
    for rep in range(3):  # replays with unrelated eager work in between
        plan.launch()
        M.sync()
        check(M, plan, expect)
        M.morph(other, M.fmt(M.RLE))
        M.sync()
    plan.set_tune(8, 0)
    plan.run()
    M.sync()
    check(M, plan, expect)
    # batched persistent launches: the plan's three levels, one launch per kernel and phase
    for tune in ((1, 0, 0, 1), (4, 2, 8, 1)):
        plan.set_tune(*tune)
        plan.run()
        M.sync()
        check(M, plan, expect)
        for rep in range(3):
            plan.launch()
            M.sync()
            check(M, plan, expect)
            M.morph(other, M.fmt(M.DYN_BP))
            M.sync()
    plan.close()
