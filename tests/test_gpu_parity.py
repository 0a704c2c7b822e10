"""GPU parity: the HIP library against the CPU oracle, element by element.

Sizes span several 512-value chunks, several workgroup segments and ragged tails;
every compressed output is decoded by the oracle's decoder and its per-block
sections are compared with the oracle's own encoding of the expected values.
"""
import numpy as np
import pytest

import oracle as O
from paper_2004_09350_amd import datagen
from tests._parity import assert_column

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu
    morphgpu.init()
    return morphgpu


SIZES = [0, 1, 31, 32, 33, 511, 512, 513, 1025, 100_003, 1_000_123]


def dists(n):
    return {
        "U7": datagen.uniform_bits(11, n, 7),
        "U32": datagen.uniform_bits(12, n, 32),
        "SORTED": datagen.sorted_gaps(13, n),
        "RUNS": datagen.runs(14, n),
    }


def fmt_of(M, kind, bw=O.BW_AUTO):
    return M.fmt(kind, bw)


@pytest.mark.parametrize("n", SIZES)
def test_encode_canonical_and_decode(M, n):
    for name, v in dists(n).items():
        for kind in O.KINDS:
            col = M.encode(v, fmt_of(M, kind))
            assert_column(col, v, kind, canonical=True)
            np.testing.assert_array_equal(M.u32(col.decode()), v, err_msg=f"{name} kind {kind}")
            M.sync()


@pytest.mark.parametrize("b", [0, 1, 3, 4, 5, 8, 12, 13, 16, 20, 24, 27, 31, 32])
def test_static_bp_every_width(M, b):
    v = datagen.uniform_bits(100 + b, 70_001, b)
    col = M.encode(v, fmt_of(M, O.STATIC_BP, b))
    assert_column(col, v, O.STATIC_BP, b, canonical=True)
    M.sync()


def test_dynbp_mixed_block_widths(M):
    rng = np.random.default_rng(3)
    blocks = [rng.integers(0, 1 << w, 512, dtype=np.uint64) if w else np.zeros(512, np.uint64)
              for w in list(range(33)) * 3]
    v = np.concatenate(blocks + [rng.integers(0, 1 << 32, 77, dtype=np.uint64)]).astype(np.uint32)
    for kind in (O.DYN_BP, O.DELTA_DYN_BP, O.FOR_DYN_BP):
        col = M.encode(v, fmt_of(M, kind))
        assert_column(col, v, kind, canonical=True)
    M.sync()


@pytest.mark.parametrize("n", [513, 100_003])
def test_morph_all_pairs(M, n):
    for name, v in dists(n).items():
        for kin in O.KINDS:
            src = M.encode(v, fmt_of(M, kin))
            for kout in O.KINDS:
                out = M.morph(src, fmt_of(M, kout))
                assert_column(out, v, kout)
                back = M.morph(out, fmt_of(M, kin)).shrink()
                assert_column(back, v, kin, canonical=True)  # f -> g -> f is the canonical f
    M.sync()


PREDS = [(O.LT, 103, 0), (O.EQ, 5, 0), (O.NE, 5, 0), (O.GE, 0, 0), (O.LT, 0, 0), (O.BETWEEN, 100, 900),
         (O.GT, 0xFFFFFFFF, 0), (O.LE, 1 << 31, 0)]


@pytest.mark.parametrize("n", [1, 600, 100_003, 1_000_000])
def test_select_all_formats(M, n):
    v = datagen.uniform_bits(21, n, 10)
    for kin in O.KINDS:
        col = M.encode(v, fmt_of(M, kin))
        for cmp, c0, c1 in PREDS:
            want = O.select(v, cmp, c0, c1)
            for kout in O.KINDS:
                p = M.select(col, cmp, c0, c1, fmt_of(M, kout))
                assert_column(p, want, kout)
    M.sync()


def narrow_preds(W):
    """Every comparison with constants inside, at the edges of and beyond [0, 2^W)."""
    top = (1 << W) - 1
    cs = sorted({0, 1, top // 3, top // 2, top - 1, top, top + 1, 1 << 31, 0xFFFFFFFF})
    out = []
    for c in cs:
        for cmp in (O.EQ, O.NE, O.LT, O.LE, O.GT, O.GE):
            out.append((cmp, c, 0))
    out += [(O.BETWEEN, 1, top - 1), (O.BETWEEN, top // 2, top + 5), (O.BETWEEN, top + 1, 1 << 20),
            (O.BETWEEN, 3, 2)]
    return out


@pytest.mark.parametrize("W", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("n", [1, 33, 2047, 2049, 100_003, 1_000_123, 3_000_017])
def test_select_narrow_static_bp(M, W, n):
    """Static BP at widths 1..8: the predicate on packed words (four chunks per wave step,
    SWAR for widths 1, 2, 4, 8), every comparison, ragged tails and remainders."""
    v = datagen.uniform_bits(500 + W, n, W)
    for bw in (W, O.BW_AUTO):
        col = M.encode(v, fmt_of(M, O.STATIC_BP, bw))
        for cmp, c0, c1 in narrow_preds(W):
            want = O.select(v, cmp, c0, c1)
            p = M.select(col, cmp, c0, c1, fmt_of(M, O.DELTA_DYN_BP))
            np.testing.assert_array_equal(M.u32(p.decode()), want, err_msg=f"W={W} n={n} bw={bw} {cmp} {c0} {c1}")
    if n == 100_003:
        for kout in O.KINDS:
            want = O.select(v, O.LT, (1 << W) // 3)
            assert_column(M.select(col, O.LT, (1 << W) // 3, 0, fmt_of(M, kout)), want, kout)
    M.sync()


@pytest.mark.parametrize("sel", [0.0005, 0.01, 0.5, 0.999])
def test_select_selectivity_sweep(M, sel):
    """Low selectivity makes output blocks span many segments (global staging)."""
    n = 3_000_017
    v = datagen.uniform_bits(22, n, 16)
    c = int(sel * 65536)
    want = O.select(v, O.LT, c)
    col = M.encode(v, fmt_of(M, O.STATIC_BP, 16))
    for kout in O.KINDS:
        assert_column(M.select(col, O.LT, c, 0, fmt_of(M, kout)), want, kout)
    M.sync()


def test_select_sorted_and_runs_inputs(M):
    n = 400_001
    for v in (datagen.sorted_gaps(31, n), datagen.runs(32, n)):
        thr = int(np.quantile(v, 0.3))
        want = O.select(v, O.LT, thr)
        for kin in (O.DELTA_DYN_BP, O.RLE, O.FOR_DYN_BP):
            col = M.encode(v, fmt_of(M, kin))
            for kout in (O.DELTA_DYN_BP, O.STATIC_BP, O.RLE):
                assert_column(M.select(col, O.LT, thr, 0, fmt_of(M, kout)), want, kout)
    M.sync()


@pytest.mark.parametrize("n", [1000, 250_007])
def test_project_all_formats(M, n):
    data = {"U20": datagen.uniform_bits(41, n, 20), "SORTED": datagen.sorted_gaps(42, n),
            "RUNS": datagen.runs(43, n)}
    rng = np.random.default_rng(4)
    pos_sorted = np.sort(rng.choice(n, n // 7, replace=False)).astype(np.uint32)
    pos_any = rng.integers(0, n, n // 5).astype(np.uint32)  # any order, duplicates
    for dname, d in data.items():
        for kd in O.KINDS:
            dc = M.encode(d, fmt_of(M, kd))
            for pos, kp in ((pos_sorted, O.DELTA_DYN_BP), (pos_any, O.UNCOMPR), (pos_any, O.STATIC_BP)):
                pc = M.encode(pos, fmt_of(M, kp))
                want = O.project(d, pos)
                for kout in O.KINDS:
                    assert_column(M.project(dc, pc, fmt_of(M, kout)), want, kout)
    M.sync()


def test_project_static_bp_auto_narrowing(M):
    """Auto width is the width of the projected main part, narrower than the data's."""
    n = 70_000
    d = datagen.uniform_bits(44, n, 12)
    d[5] = 0xFFFFF  # the one 20-bit value, never projected
    pos = np.arange(6, n, 3, dtype=np.uint32)
    dc = M.encode(d, fmt_of(M, O.DYN_BP))
    pc = M.encode(pos, fmt_of(M, O.DELTA_DYN_BP))
    got = assert_column(M.project(dc, pc, fmt_of(M, O.STATIC_BP)), O.project(d, pos), O.STATIC_BP)
    assert got["bit_width"] == 12
    M.sync()


def test_semijoin_and_bitmap(M):
    rng = np.random.default_rng(5)
    D = 300_000
    dim = datagen.uniform_range(51, D, 0, 100)
    s = O.select(dim, O.LT, 20)
    keys = datagen.uniform_range(52, 1_500_001, 0, D)
    bm_want = O.bitmap_from_positions(s, D)
    want = O.semijoin(keys, bm_want, D)
    sc = M.encode(s, fmt_of(M, O.DELTA_DYN_BP))
    bm = M.bitmap_from_positions(sc, D)
    np.testing.assert_array_equal(M.u32(bm)[: bm_want.size], bm_want)
    for kk in (O.STATIC_BP, O.UNCOMPR, O.DYN_BP):
        kc = M.encode(keys, fmt_of(M, kk))
        for kout in O.KINDS:
            assert_column(M.semijoin(kc, bm, D, fmt_of(M, kout)), want, kout)
    # keys outside the domain never match
    keys2 = keys.copy()
    keys2[::7] = D + 5
    kc = M.encode(keys2, fmt_of(M, O.UNCOMPR))
    assert_column(M.semijoin(kc, bm, D, fmt_of(M, O.DELTA_DYN_BP)), O.semijoin(keys2, bm_want, D), O.DELTA_DYN_BP)
    M.sync()
    del rng


@pytest.mark.parametrize("D", [2_500, 262_144, 262_145, 1_308_672, 1_308_673, 2_000_000, 2_617_344, 3_000_000,
                               3_926_016, 3_926_017])
def test_semijoin_small_domains(M, D):
    """Bitmaps built from select outputs (recorded as increasing), domains that fit the
    probe's LDS or exceed it (probed partly in LDS, the wide kernel's 1 308 672 bits and
    above), and keys in and out of the domain."""
    dim = datagen.uniform_range(61, D, 0, 100)
    s = O.select(dim, O.LT, 13)
    keys = datagen.uniform_range(62, 2_000_003, 0, D + D // 50)
    bm_want = O.bitmap_from_positions(s, D)
    want = O.semijoin(keys, bm_want, D)
    sc = M.select(M.encode(dim, fmt_of(M, O.STATIC_BP)), M.LT, 13, 0, fmt_of(M, O.DELTA_DYN_BP))
    bm = M.bitmap_from_positions(sc, D)
    np.testing.assert_array_equal(M.u32(bm)[: bm_want.size], bm_want)
    for kk in (O.STATIC_BP, O.UNCOMPR, O.DYN_BP, O.RLE):
        kc = M.encode(keys, fmt_of(M, kk))
        for kout in (O.UNCOMPR, O.DELTA_DYN_BP, O.RLE):
            assert_column(M.semijoin(kc, bm, D, fmt_of(M, kout)), want, kout)
    M.sync()


def test_intersect(M):
    rng = np.random.default_rng(6)
    N = 2_000_000
    a = np.sort(rng.choice(N, 200_000, replace=False)).astype(np.uint32)
    b = np.sort(rng.choice(N, 1_000_000, replace=False)).astype(np.uint32)
    want = O.intersect(a, b)
    for ka in (O.DELTA_DYN_BP, O.UNCOMPR, O.RLE):
        for kb in (O.DELTA_DYN_BP, O.STATIC_BP):
            ac = M.encode(a, fmt_of(M, ka))
            bc = M.encode(b, fmt_of(M, kb))
            for kout in O.KINDS:
                assert_column(M.intersect(ac, bc, N, fmt_of(M, kout)), want, kout)
                assert_column(M.intersect(bc, ac, N, fmt_of(M, kout)), want, kout)
    M.sync()


@pytest.mark.parametrize("n", [0, 1, 777, 1_000_003])
def test_sum(M, n):
    for name, v in dists(n).items():
        for kind in O.KINDS:
            col = M.encode(v, fmt_of(M, kind))
            assert int(M.u64(M.sum_(col))[0]) == O.sum_(v), (name, kind)
    M.sync()


def test_group_sum(M):
    n = 500_001
    g = datagen.uniform_range(61, n, 0, 250)
    v = datagen.uniform_bits(62, n, 17)
    want = O.group_sum(g, v, 250)
    for kg in (O.STATIC_BP, O.DELTA_DYN_BP, O.UNCOMPR):
        for kv in (O.STATIC_BP, O.FOR_DYN_BP, O.RLE):
            out = M.group_sum(M.encode(g, fmt_of(M, kg)), M.encode(v, fmt_of(M, kv)), 250)
            np.testing.assert_array_equal(M.u64(out), want)
    # more groups than the LDS histogram holds
    g2 = datagen.uniform_range(63, n, 0, 10_000)
    out = M.group_sum(M.encode(g2, fmt_of(M, O.STATIC_BP)), M.encode(v, fmt_of(M, O.STATIC_BP)), 10_000)
    np.testing.assert_array_equal(M.u64(out), O.group_sum(g2, v, 10_000))
    M.sync()


def test_q1_end_to_end(M):
    """select(A < 103) as delta+DynBP -> project(B) as static BP(auto) -> sum, 1M rows."""
    import oracle.queries as Q
    n = 1_000_000
    a = datagen.uniform_bits(1, n, 10)
    b = datagen.uniform_bits(2, n, 20)
    want = Q.q1(a, b)
    ca = M.encode(a, fmt_of(M, O.STATIC_BP, 10))
    cb = M.encode(b, fmt_of(M, O.STATIC_BP, 20))
    p = M.select(ca, O.LT, 103, 0, fmt_of(M, O.DELTA_DYN_BP))
    bp = M.project(cb, p, fmt_of(M, O.STATIC_BP))
    s = M.sum_(bp)
    assert int(M.u64(s)[0]) == want["sum"]
    assert_column(p, want["P"], O.DELTA_DYN_BP)
    assert_column(bp, want["Bp"], O.STATIC_BP)
    M.sync()


# ---------------------------------------------------------------------------------------- errors
def _expect(M, code):
    with pytest.raises(M.MorphError) as ei:
        M.sync()
    assert ei.value.status == code


def test_error_paths(M):
    d = M.encode(np.arange(100, dtype=np.uint32), fmt_of(M, O.STATIC_BP))
    p = M.encode(np.array([1, 5, 100], np.uint32), fmt_of(M, O.UNCOMPR))
    M.project(d, p, fmt_of(M, O.UNCOMPR))
    _expect(M, "OUT_OF_RANGE")
    M.sync()  # the flag was cleared
    a = M.encode(np.array([1, 3, 3, 7], np.uint32), fmt_of(M, O.UNCOMPR))
    b = M.encode(np.arange(10, dtype=np.uint32), fmt_of(M, O.UNCOMPR))
    M.intersect(a, b, 16)
    _expect(M, "NOT_SORTED")
    g = M.encode(np.array([0, 1, 2, 9], np.uint32), fmt_of(M, O.UNCOMPR))
    v = M.encode(np.array([1, 1, 1, 1], np.uint32), fmt_of(M, O.UNCOMPR))
    M.group_sum(g, v, 5)
    _expect(M, "OUT_OF_RANGE")
    with pytest.raises(M.MorphError) as ei:
        M.group_sum(g, M.encode(np.ones(3, np.uint32), fmt_of(M, O.UNCOMPR)), 5)
    assert ei.value.status == "LENGTH_MISMATCH"
    M.encode(np.arange(64, dtype=np.uint32), fmt_of(M, O.STATIC_BP, 5))
    _expect(M, "VALUE_TOO_WIDE")
    pos = M.encode(np.array([3, 70], np.uint32), fmt_of(M, O.UNCOMPR))
    M.bitmap_from_positions(pos, 64)
    _expect(M, "OUT_OF_RANGE")
    with pytest.raises(M.MorphError) as ei:
        M.select(d, 99, 0, 0, fmt_of(M, O.UNCOMPR))
    assert ei.value.status == "INVALID_ARG"
    with pytest.raises(M.MorphError) as ei:
        M.morph(d, M.Format(7, 0))
    assert ei.value.status == "INVALID_ARG"
    M.sync()
