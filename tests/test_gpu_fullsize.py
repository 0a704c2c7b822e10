"""Parity at the benchmark's full sizes, in the launch shapes the benchmark times:
1e8-row sweep columns and the 6e8-row star query.

Every output element is compared with the oracle.  The oracle's inputs are the numpy
generators' columns (never the GPU generator's); its expected outputs (position lists,
projected values, the star query's intermediate P and both 250-group answers) are
uploaded and compared with the decoded GPU outputs by exact equality on the device.  The
star query is row-local up to its additive group-sums (section 3.3's operators on a
horizontal slice of the fact table give that slice's positions, and group-sums add), so
the oracle evaluates it over fact-row chunks in parallel and concatenates / adds the
chunk results."""
import numpy as np
import pytest

import oracle as O
from paper_2004_09350_amd import datagen
from tests._oracle_star import oracle_star

pytestmark = pytest.mark.gpu

N = 100_000_000
DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu
    morphgpu.init()
    return morphgpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def assert_equal_dev(M, col, want_dev, label):
    """Decoded GPU column == expected values (a device tensor), element by element."""
    import torch
    n = int(col.info()["n"])
    assert n == want_dev.numel(), f"{label}: {n} elements, want {want_dev.numel()}"
    got = col.decode(n)
    if not torch.equal(got, want_dev):
        bad = torch.nonzero(got != want_dev)[:5, 0].cpu().numpy()
        raise AssertionError(f"{label}: {int((got != want_dev).sum())} elements differ, first at {bad}")
    del got


def threshold_10(dist, v):
    if dist.startswith("U"):
        b = int(dist[1:])
        return max(1, round(0.1 * (1 << b))) if b < 32 else int(0.1 * (1 << 32))
    if dist == "RUNS":
        return int(0.1 * (1 << 16))
    return int(v[int(0.1 * v.size)])   # sorted: the value at the 10 % quantile


@pytest.mark.parametrize("dist", DISTS)
def test_sweep_column_fullsize(M, dist):
    """1e8 rows, every input format: decode, sum, select (10 %) into every format,
    project at a 10 % position list into every format, morph into every other format."""
    import torch
    seed = 7000 + DISTS.index(dist)
    v = datagen.sweep_column(dist, seed, N)
    vd = dev(v)
    c = threshold_10(dist, v)
    want_sel = dev(O.select(v, O.LT, c))
    want_sum = O.sum_(v)
    pos = O.select(datagen.uniform_bits(7100, N, 12), O.LT, 410)
    P = M.encode(pos, M.fmt(M.DELTA_DYN_BP))
    want_prj = dev(O.project(v, pos))
    del pos
    for kin in M.KINDS:
        col = M.encode(vd, M.fmt(kin))
        assert int(M.sum_(col).cpu()) & 0xFFFFFFFFFFFFFFFF == want_sum, (dist, kin)
        assert_equal_dev(M, col, vd, f"decode {dist} {kin}")
        for kout in M.KINDS:
            assert_equal_dev(M, M.select(col, M.LT, c, 0, M.fmt(kout)), want_sel, f"select {dist} {kin}->{kout}")
            assert_equal_dev(M, M.project(col, P, M.fmt(kout)), want_prj, f"project {dist} {kin}->{kout}")
            if kout != kin:
                assert_equal_dev(M, M.morph(col, M.fmt(kout)), vd, f"morph {dist} {kin}->{kout}")
        del col
        torch.cuda.empty_cache()
    M.sync()


def test_intersect_fullsize(M):
    a = datagen.uniform_bits(7100, N, 12)
    b = datagen.uniform_bits(7101, N, 12)
    pa, pb = O.select(a, O.LT, 410), O.select(b, O.LT, 2048)
    want = dev(O.intersect(pa, pb))
    Pa = M.encode(pa, M.fmt(M.DELTA_DYN_BP))
    Pb = M.encode(pb, M.fmt(M.DELTA_DYN_BP))
    for kout in M.KINDS:
        assert_equal_dev(M, M.intersect(Pa, Pb, N, M.fmt(kout)), want, f"intersect -> {kout}")
        assert_equal_dev(M, M.intersect(Pb, Pa, N, M.fmt(kout)), want, f"intersect (swapped) -> {kout}")
    M.sync()


# ----------------------------------------------------------------------------- star query
STAR_N = 600_000_000


def test_star_query_fullsize(M):
    """6e8 fact rows, wide and narrow filters, the captured graph the benchmark replays:
    the intersected position list P and both group-sum answers equal the oracle's."""
    from paper_2004_09350_amd import queries, selector
    D = datagen.STAR_DIM_SIZES
    cols, _ = selector.star_inputs(1, STAR_N)
    for sel in (datagen.STAR_WIDE, datagen.STAR_NARROW):
        thr = datagen.star_thresholds(sel)
        P, out1, out2 = oracle_star(1, STAR_N, thr)
        q = queries.Q3(cols, thr, D, STAR_N)
        q.plan.set_tune(2, 0)
        q.plan.launch()
        M.sync()
        assert_equal_dev(M, q.plan.column(q.names["P"]), dev(P), f"star P {sel}")
        g1, g2 = q.results()
        np.testing.assert_array_equal(g1, out1, err_msg=f"star out1 {sel}")
        np.testing.assert_array_equal(g2, out2, err_msg=f"star out2 {sel}")
        q.plan.close()
    M.sync()
