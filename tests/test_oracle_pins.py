"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each pin uses an independent route: Python big-integer bit streams for packing,
numpy library routines for the operators, closed forms for footprints, brute
force on tiny inputs, the paper's qualitative format claims, finite differences
for the network's gradient and the closed form of Adam's first step.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2004_09350_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_packing.json")


def bigint_pack(vals, b):
    """Independent packing: the stream as one Python integer, split into 32-bit words."""
    s = 0
    for j, v in enumerate(vals):
        assert 0 <= v < (1 << b) or b == 0 and v == 0
        s |= int(v) << (j * b)
    nwords = (len(vals) * b + 31) // 32
    return [(s >> (32 * q)) & 0xFFFFFFFF for q in range(nwords)]


def np_bw(a):
    a = np.asarray(a, np.uint64)
    out = np.zeros(a.shape, np.int64)
    x = a.copy()
    while np.any(x):
        nz = x != 0
        out[nz] += 1
        x >>= np.uint64(1)
    return out


def block_or(a, bs):
    return np.bitwise_or.reduce(a.reshape(-1, bs), axis=1) if a.size else np.zeros(0, a.dtype)


# ----------------------------------------------------------------------------- hand-worked encodings
def test_handworked_fixtures():
    g = json.load(open(GOLD))
    cases = {c["name"]: c for c in g["cases"]}

    c = cases["static_bp_b10"]
    v = c["values_head"] + [0] * (c["pad_to"] - 4)
    e = O.encode(v, O.STATIC_BP, 10)
    assert e["payload_words"] == c["payload_words"]
    assert [int(x) for x in e["payload"][:2]] == [int(h, 16) for h in c["payload_head"]]
    assert list(e["payload"]) == bigint_pack(v, 10)

    c = cases["static_bp_b2"]
    v = c["values_head"] + [0] * 29
    e = O.encode(v, O.STATIC_BP, 2)
    assert [int(e["payload"][0])] == [int(c["payload_head"][0], 16)]
    assert e["payload_words"] == 2

    c = cases["dynbp_zeros_then_5"]
    v = [0] * 511 + [5]
    e = O.encode(v, O.DYN_BP)
    assert int(e["widths"][0]) == 3 and e["payload_words"] == 48
    assert int(e["payload"][47]) == 0xA0000000 and not np.any(e["payload"][:47])

    c = cases["delta_half_steps"]
    v = [100 + j // 2 for j in range(512)]
    e = O.encode(v, O.DELTA_DYN_BP)
    assert int(e["bases"][0]) == 100 and int(e["widths"][0]) == 1 and e["payload_words"] == 16
    assert int(e["payload"][0]) == 0x55555554 and all(int(x) == 0x55555555 for x in e["payload"][1:16])

    c = cases["for_mod8"]
    v = [1000 + (j % 8) for j in range(512)]
    e = O.encode(v, O.FOR_DYN_BP)
    assert int(e["bases"][0]) == 1000 and int(e["widths"][0]) == 3
    assert [int(x) for x in e["payload"][:3]] == [0x88FAC688, 0xC688FAC6, 0xFAC688FA]
    assert list(e["payload"]) == bigint_pack([j % 8 for j in range(512)], 3)

    v = [5] + [3] * 511
    e = O.encode(v, O.DELTA_DYN_BP)
    assert int(e["widths"][0]) == 32 and int(e["payload"][1]) == 0xFFFFFFFE and int(e["bases"][0]) == 5

    c = cases["rle_small"]
    e = O.encode(c["values"], O.RLE)
    assert list(e["rvalues"]) == c["rvalues"] and list(e["rstarts"]) == c["rstarts"]
    assert O.sum_(c["values"]) == c["sum"]
    lengths = np.diff(np.append(e["rstarts"], len(c["values"])))
    assert int(np.sum(e["rvalues"].astype(np.uint64) * lengths.astype(np.uint64))) == c["sum"]


@pytest.mark.parametrize("b", list(range(0, 33)))
def test_static_bp_matches_bigint_stream(b):
    n = 96 + 7
    v = datagen.uniform_bits(1000 + b, n, b)
    e = O.encode(v, O.STATIC_BP, b)
    assert e["bit_width"] == b and e["n_main"] == 96 and e["n_rem"] == 7
    assert list(e["payload"]) == bigint_pack(list(v[:96]), b)
    assert list(e["rem"]) == list(v[96:])


@pytest.mark.parametrize("kind", [O.DYN_BP, O.DELTA_DYN_BP, O.FOR_DYN_BP])
def test_dynbp_family_blocks_match_bigint_stream(kind):
    rng = np.random.default_rng(7)
    n = 512 * 5 + 100
    widths = [0, 1, 13, 31, 32]
    v = np.concatenate([rng.integers(0, 1 << w, 512, dtype=np.uint64) if w else np.zeros(512, np.uint64)
                        for w in widths] + [rng.integers(0, 1 << 32, 100, dtype=np.uint64)]).astype(np.uint32)
    if kind == O.DELTA_DYN_BP:
        v = np.cumsum(v.astype(np.uint64)).astype(np.uint32)  # wrapping prefix sums, residuals are the draws
    e = O.encode(v, kind)
    assert e["nb"] == 5 and e["n_rem"] == 100
    off = 0
    for k in range(5):
        blk = v[512 * k: 512 * (k + 1)].astype(np.int64)
        if kind == O.DYN_BP:
            r, base = blk, None
        elif kind == O.FOR_DYN_BP:
            base = int(blk.min())
            r = blk - base
        else:
            base = int(blk[0])
            r = np.concatenate([[0], np.diff(blk) % (1 << 32)])
        w = int(np_bw([np.bitwise_or.reduce(r.astype(np.uint64))])[0])
        assert int(e["widths"][k]) == w
        assert int(e["offsets"][k]) == off
        if base is not None:
            assert int(e["bases"][k]) == base
        assert list(e["payload"][off: off + 16 * w]) == bigint_pack([int(x) for x in r], w)
        off += 16 * w
    assert e["payload_words"] == off
    assert list(e["rem"]) == list(v[2560:])


# ----------------------------------------------------------------------------- round trips and footprints
SIZES = [0, 1, 31, 32, 33, 511, 512, 513, 1023, 1024, 1025, 100_003]


def _cols(n):
    yield datagen.uniform_bits(11, n, 7)
    yield datagen.uniform_bits(12, n, 32)
    yield np.full(n, 0xFFFFFFFF, np.uint32)
    yield np.zeros(n, np.uint32)
    yield datagen.sorted_gaps(13, n)
    yield datagen.runs(14, n)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", O.KINDS)
def test_round_trip(kind, n):
    for v in _cols(n):
        e = O.encode(v, kind)
        np.testing.assert_array_equal(O.decode(e), v)


def closed_form_footprints(v):
    v = np.asarray(v, np.uint32)
    n = v.size
    out = [4 * n]
    nm = n // 32 * 32
    b = int(np_bw([np.bitwise_or.reduce(v[:nm].astype(np.uint64))])[0]) if nm else 0
    out.append(nm * b // 8 + 4 * (n - nm))
    nm = n // 512 * 512
    blocks = v[:nm].reshape(-1, 512).astype(np.int64)
    rem = 4 * (n - nm)
    w_dyn = np_bw(block_or(v[:nm].astype(np.uint64), 512)) if nm else np.zeros(0, np.int64)
    out.append(int(np.sum(5 + 64 * w_dyn)) + rem)
    if nm:
        d = np.concatenate([np.zeros((blocks.shape[0], 1), np.int64), np.diff(blocks, axis=1) % (1 << 32)], axis=1)
        w_d = np_bw(np.bitwise_or.reduce(d.astype(np.uint64), axis=1))
        f = blocks - blocks.min(axis=1, keepdims=True)
        w_f = np_bw(np.bitwise_or.reduce(f.astype(np.uint64), axis=1))
    else:
        w_d = w_f = np.zeros(0, np.int64)
    out.append(int(np.sum(9 + 64 * w_d)) + rem)
    out.append(int(np.sum(9 + 64 * w_f)) + rem)
    runs = 0 if n == 0 else 1 + int(np.count_nonzero(v[1:] != v[:-1]))
    out.append(8 * runs)
    return out


@pytest.mark.parametrize("n", [0, 33, 511, 513, 5000, 100_003])
def test_footprint_closed_forms(n):
    for v in _cols(n):
        cf = closed_form_footprints(v)
        assert [int(x) for x in O.footprints(v)] == cf
        for kind in O.KINDS:
            assert O.encode(v, kind)["footprint"] == cf[kind]


def test_static_bp_width_errors_and_auto():
    v = np.arange(64, dtype=np.uint32)
    assert O.encode(v, O.STATIC_BP)["bit_width"] == 6
    with pytest.raises(O.OracleError) as ei:
        O.encode(v, O.STATIC_BP, 5)
    assert ei.value.code == O.ERR_VALUE_TOO_WIDE
    # the remainder is not constrained by the width
    v = np.concatenate([np.zeros(32, np.uint32), np.array([0xFFFFFFFF], np.uint32)])
    e = O.encode(v, O.STATIC_BP, 0)
    assert e["bit_width"] == 0 and e["payload_words"] == 0 and list(e["rem"]) == [0xFFFFFFFF]


def test_brute_force_tiny_round_trip():
    alphabet = [0, 1, 2, 0xFFFFFFFF]
    for n in range(0, 5):
        for t in itertools.product(alphabet, repeat=n):
            v = np.array(t, np.uint32)
            for kind in O.KINDS:
                np.testing.assert_array_equal(O.decode(O.encode(v, kind)), v)


# ----------------------------------------------------------------------------- operators
def py_pred(v, cmp, c0, c1):
    return [v == c0, v != c0, v < c0, v <= c0, v > c0, v >= c0, c0 <= v <= c1][cmp]


def test_brute_force_tiny_select():
    alphabet = [0, 1, 5, 0xFFFFFFFF]
    consts = [(0, 0), (1, 5), (5, 1), (0xFFFFFFFF, 0xFFFFFFFF), (2, 0xFFFFFFFF)]
    for n in range(0, 5):
        for t in itertools.product(alphabet, repeat=n):
            for cmp in range(7):
                for c0, c1 in consts:
                    want = [i for i, x in enumerate(t) if py_pred(x, cmp, c0, c1)]
                    assert list(O.select(t, cmp, c0, c1)) == want


def test_select_matches_numpy():
    v = datagen.uniform_bits(3, 200_000, 12)
    for cmp, f in [(O.EQ, lambda x: x == 100), (O.NE, lambda x: x != 100), (O.LT, lambda x: x < 410),
                   (O.LE, lambda x: x <= 410), (O.GT, lambda x: x > 3000), (O.GE, lambda x: x >= 3000)]:
        np.testing.assert_array_equal(O.select(v, cmp, {O.EQ: 100, O.NE: 100, O.LT: 410, O.LE: 410,
                                                        O.GT: 3000, O.GE: 3000}[cmp]), np.nonzero(f(v))[0])
    np.testing.assert_array_equal(O.select(v, O.BETWEEN, 7, 900), np.nonzero((v >= 7) & (v <= 900))[0])
    np.testing.assert_array_equal(O.select(v, O.GE, 0), np.arange(v.size))  # always true = iota
    assert O.select(v, O.LT, 0).size == 0  # always false
    assert O.select(v, O.BETWEEN, 9, 8).size == 0


def test_semijoin_bitmap_project_intersect_sum_groupsum_vs_numpy():
    rng = np.random.default_rng(5)
    D = 10_000
    dim_pos = np.sort(rng.choice(D, 1234, replace=False)).astype(np.uint32)
    bm = O.bitmap_from_positions(dim_pos, D)
    dense = np.zeros(D, bool)
    dense[dim_pos] = True
    np.testing.assert_array_equal(np.unpackbits(bm.view(np.uint8), bitorder="little")[:D].astype(bool), dense)
    keys = rng.integers(0, D + 50, 100_000).astype(np.uint32)  # some keys outside the domain
    inside = keys < D
    want = np.nonzero(inside & dense[np.minimum(keys, D - 1)])[0]
    np.testing.assert_array_equal(O.semijoin(keys, bm, D), want)

    data = datagen.uniform_bits(9, 50_000, 20)
    pos = rng.integers(0, data.size, 30_000).astype(np.uint32)  # any order, duplicates allowed
    np.testing.assert_array_equal(O.project(data, pos), data[pos])

    a = np.sort(rng.choice(1_000_000, 100_000, replace=False)).astype(np.uint32)
    b = np.sort(rng.choice(1_000_000, 500_000, replace=False)).astype(np.uint32)
    np.testing.assert_array_equal(O.intersect(a, b), np.intersect1d(a, b, assume_unique=True))
    np.testing.assert_array_equal(O.intersect(a, b), O.intersect(b, a))

    v = datagen.uniform_bits(10, 300_000, 32)
    assert O.sum_(v) == int(np.sum(v, dtype=np.uint64))
    g = rng.integers(0, 250, v.size).astype(np.uint32)
    want = np.zeros(250, np.uint64)
    np.add.at(want, g, v.astype(np.uint64))
    got = O.group_sum(g, v, 250)
    np.testing.assert_array_equal(got, want)
    assert int(np.sum(got, dtype=np.uint64)) == O.sum_(v)  # sum over groups = total sum


def test_sum_exact_in_64_bits():
    """Sums are exact uint64 arithmetic: beyond 32 bits and beyond the 53 bits a double
    holds exactly (a wrap past 2^64 needs more than 2^32 values, more than a column holds)."""
    n = 1 << 22
    v = np.full(n, 0xFFFFFFFF, np.uint32)
    want = n * 0xFFFFFFFF                      # 18 014 398 505 287 680 > 2^53
    assert want > 1 << 53
    assert O.sum_(v) == want
    v[-1] = 0xFFFFFFFE                         # off by one in the last bit: still exact
    assert O.sum_(v) == want - 1
    assert O.group_sum([0, 0], [0xFFFFFFFF, 1], 1)[0] == 0x100000000
    g = np.arange(n, dtype=np.uint32) & 1
    got = O.group_sum(g, v, 2)
    assert int(got[0]) == (n // 2) * 0xFFFFFFFF and int(got[1]) == (n // 2) * 0xFFFFFFFF - 1


def test_error_paths():
    with pytest.raises(O.OracleError) as ei:
        O.project([1, 2, 3], [0, 3])
    assert ei.value.code == O.ERR_OUT_OF_RANGE
    with pytest.raises(O.OracleError) as ei:
        O.bitmap_from_positions([1, 64], 64)
    assert ei.value.code == O.ERR_OUT_OF_RANGE
    with pytest.raises(O.OracleError) as ei:
        O.intersect([1, 1, 2], [1])
    assert ei.value.code == O.ERR_NOT_SORTED
    with pytest.raises(O.OracleError) as ei:
        O.intersect([1, 2], [3, 2])
    assert ei.value.code == O.ERR_NOT_SORTED
    with pytest.raises(O.OracleError) as ei:
        O.group_sum([0, 1], [1], 2)
    assert ei.value.code == O.ERR_LENGTH_MISMATCH
    with pytest.raises(O.OracleError) as ei:
        O.group_sum([0, 2], [1, 1], 2)
    assert ei.value.code == O.ERR_OUT_OF_RANGE
    assert O.project([], []).size == 0
    assert O.select([], O.LT, 5).size == 0


def test_format_invariance_of_query_answers():
    """Compression is lossless: a query gives the same answer under every format assignment."""
    x = datagen.uniform_bits(21, 20_000, 10)
    y = datagen.uniform_bits(22, 20_000, 20)
    want = O.sum_(y[x < 103])
    for kx in O.KINDS:
        xp = O.decode(O.encode(x, kx))
        p = O.select(xp, O.LT, 103)
        for kp in O.KINDS:
            pp = O.decode(O.encode(p, kp))
            for ky in (O.STATIC_BP, O.RLE, O.DELTA_DYN_BP):
                yp = O.project(O.decode(O.encode(y, ky)), pp)
                assert O.sum_(O.decode(O.encode(yp, O.FOR_DYN_BP))) == want


# ----------------------------------------------------------------------------- the paper's format claims
def test_best_format_claims_on_32bit_analogs():
    """Section 5.1: small uniform values favour static BP, rare huge outliers favour per-block
    BP, a narrow range of huge values favours FOR + BP, sorted data favours DELTA + BP, and
    sorted position lists favour DELTA."""
    n = 1 << 20
    c1 = datagen.uniform_range(31, n, 0, 64)
    c2 = c1.copy()
    out_idx = np.nonzero(datagen.uniform_range(32, n, 0, 10_000) == 0)[0]  # about 0.01 %
    c2[out_idx] = 0xFFFFFFFF
    c3 = datagen.uniform_range(33, n, 1 << 31, 64)
    c4 = np.sort(datagen.uniform_range(34, n, 1 << 31, 100_001))
    assert int(np.argmin(O.footprints(c1))) == O.STATIC_BP
    assert int(np.argmin(O.footprints(c2))) == O.DYN_BP
    assert int(np.argmin(O.footprints(c3))) == O.FOR_DYN_BP
    assert int(np.argmin(O.footprints(c4))) == O.DELTA_DYN_BP
    pos = O.select(c1, O.LT, 30)
    assert int(np.argmin(O.footprints(pos))) == O.DELTA_DYN_BP


# ----------------------------------------------------------------------------- statistics
def test_stats_closed_forms():
    f = O.stats(np.full(1024, 7, np.uint32))
    assert f[1] == 1.0 and f[0] == 0.0  # bw(7) = 3 -> bin {1-3}
    assert f[12] == 1.0  # every difference is 0
    assert f[20] == 1.0
    assert f[21] == pytest.approx(9 / 32)  # two chunks of one run of 512 each
    assert f[23] == 0.0 and f[25] == pytest.approx(3 / 32) and f[26] == 0.0 and f[27] == 0.0
    assert f[31] == 1.0 and f[28] == f[29] == f[30] == pytest.approx(3 / 32)
    assert f[22] == pytest.approx(np.log2(1 + 256 * np.log(256 / 255)) / 32)  # one distinct value
    assert f[24] == pytest.approx(np.log2(1025) / 32)

    n = 65536
    f = O.stats(np.arange(n, dtype=np.uint32))
    assert f[20] == 1.0 and f[21] == 0.0 and f[13] == 1.0  # difference 1 -> bw 1 -> bin {1-5}
    assert f[22] == pytest.approx(np.log2(n) / 32, abs=np.log2(1.25) / 32)  # HLL: 6.5 % standard error
    assert f[23] == pytest.approx(np.log2(n) / 32)
    assert sum(f[0:12]) == pytest.approx(1.0) and sum(f[12:20]) == pytest.approx(1.0)
    hist = np.bincount([0 if b == 0 else 1 + (b - 1) // 3 for b in np_bw(np.arange(n))], minlength=12) / n
    np.testing.assert_allclose(f[0:12], hist)

    f = O.stats(datagen.uniform_bits(5, 10 * n, 16))  # sampled path: 128 chunks
    assert f[24] == pytest.approx(np.log2(10 * n + 1) / 32)
    # 65536 sampled values drawn from 2^16 keys hold 2^16 (1 - 1/e) distinct values on average
    assert f[22] == pytest.approx(np.log2(65536 * (1 - np.exp(-1))) / 32, abs=np.log2(1.25) / 32)
    assert 0.45 < f[20] < 0.55


@pytest.mark.parametrize("k", range(2, 8))
def test_stats_delta_width_classes(k):
    """Constant-stride ramps: every neighbouring difference (mod 2^32) equals the stride,
    whose bit width 5(k-1)+1 falls in delta class k; feature 27 is that width / 32."""
    t = 5 * (k - 1)
    stride = 1 << t
    n = 4096
    v = (np.arange(n, dtype=np.uint64) * stride % (1 << 32)).astype(np.uint32)
    f = O.stats(v)
    want = np.zeros(8)
    want[k] = 1.0
    np.testing.assert_array_equal(f[12:20], want)
    assert f[27] == pytest.approx((t + 1) / 32)


@pytest.mark.parametrize("t", [0, 3, 11, 20])
def test_stats_for_residual_width(t):
    """Ascending ramps v = j * 2^t inside 512-value chunks (no wrap): the chunk minimum is
    the first value, the residuals are j' * 2^t for j' < 512, whose OR is 511 * 2^t, so
    feature 26 is (9 + t) / 32; feature 25 (OR of the values) is bw of the last chunk's
    OR averaged over chunks."""
    n = 512 * 8
    v = (np.arange(n, dtype=np.uint64) << np.uint64(t)).astype(np.uint32)
    f = O.stats(v)
    assert f[26] == pytest.approx((9 + t) / 32)
    or_bw = [int(np.bitwise_or.reduce(v[c * 512:(c + 1) * 512])).bit_length() for c in range(8)]
    assert f[25] == pytest.approx(np.mean(or_bw) / 32)


def test_stats_mean_width():
    """Feature 30 is the bit width of floor(mean): values 0 and 2^20 in equal numbers have
    mean 2^19 (width 20); one more zero pulls the mean just below it (width 19)."""
    v = np.tile(np.array([0, 1 << 20], np.uint32), 2048)
    assert O.stats(v)[30] == pytest.approx(20 / 32)
    v = np.concatenate([v, np.zeros(1, np.uint32)])
    assert O.stats(v)[30] == pytest.approx(19 / 32)


def test_stats_sampled_chunks():
    """Above 65536 values the statistics read 128 chunks: chunk floor(s * C / 128) for
    s < 128, C = floor(n / 512).  Chunk c holds the constant c when it is one of those and
    0xFFFFFFFF otherwise: every read chunk is constant, the largest value read is the last
    sampled index, and the unread chunks (which hold the maximum uint32) never show."""
    C = 1000
    n = 512 * C + 77
    sampled = sorted({(s * C) // 128 for s in range(128)})
    v = np.full(n, 0xFFFFFFFF, np.uint32)
    for c in sampled:
        v[512 * c:512 * (c + 1)] = c
    f = O.stats(v)
    assert f[31] == 1.0                                   # every sampled chunk is constant
    assert f[29] == pytest.approx(max(sampled).bit_length() / 32)   # 992 -> 10 bits
    assert f[28] == 0.0                                   # chunk 0 is read
    mean = sum((s * C) // 128 for s in range(128)) * 512 // (128 * 512)
    assert f[30] == pytest.approx(int(mean).bit_length() / 32)
    assert f[23] == pytest.approx(np.log2(max(sampled) + 1) / 32)
    assert f[20] == 1.0 and f[12] == 1.0                  # constant chunks: differences 0


# ----------------------------------------------------------------------------- selector network
def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.3, O.MLP_NPARAM)
    x = rng.normal(0, 1, (5, 32))
    t = rng.normal(0, 1, (5, 6))
    loss, g = O.mlp_loss_grad(p, x, t)
    y = O.mlp_forward(p, x)
    assert loss == pytest.approx(np.mean((y - t) ** 2))
    idx = rng.choice(O.MLP_NPARAM, 300, replace=False)
    for i in idx:
        h = 1e-6
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (O.mlp_loss_grad(pp, x, t)[0] - O.mlp_loss_grad(pm, x, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_mlp_forward_is_affine_relu_chain():
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.3, O.MLP_NPARAM)
    x = rng.normal(0, 1, (7, 32))
    W1 = p[:2048].reshape(64, 32); b1 = p[2048:2112]
    W2 = p[2112:6208].reshape(64, 64); b2 = p[6208:6272]
    W3 = p[6272:6656].reshape(6, 64); b3 = p[6656:6662]
    h = np.maximum(x @ W1.T + b1, 0)
    h = np.maximum(h @ W2.T + b2, 0)
    np.testing.assert_allclose(O.mlp_forward(p, x), h @ W3.T + b3, rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    m = np.zeros(100); v = np.zeros(100)
    p0 = p.copy()
    O.adam_step(p, g, m, v, 1, 0.01)
    # after one step the bias-corrected moments are g and g^2: the update is lr * g / (|g| + eps)
    np.testing.assert_allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ----------------------------------------------------------------------------- query plans
def test_q1_plan_matches_numpy():
    import oracle.queries as OQ
    a = datagen.uniform_bits(41, 50_000, 10)
    b = datagen.uniform_bits(42, 50_000, 20)
    r = OQ.q1(a, b, 103)
    np.testing.assert_array_equal(r["P"], np.nonzero(a < 103)[0])
    np.testing.assert_array_equal(r["Bp"], b[a < 103])
    assert r["sum"] == int(b[a < 103].astype(np.uint64).sum())


def test_q3_plan_matches_numpy():
    """The star plan as one numpy expression: a fact row qualifies when every foreign key
    points at a dimension row passing its filter; group by floor(fk3 / 10)."""
    import oracle.queries as OQ
    dims = (2000, 30_000, 20_000, 2500)
    n = 60_000
    cols = datagen.star_columns(9, n, dims)
    thr = datagen.star_thresholds((0.2, 0.3, 0.5, 0.4))
    r = OQ.q3(cols, thr, dims)
    ok = np.ones(n, bool)
    for d in range(4):
        ok &= (cols[f"dimattr{d}"] < thr[d])[cols[f"fk{d}"]]
    g = cols["fk3"][ok] // 10
    np.testing.assert_array_equal(r["intermediates"]["P"], np.nonzero(ok)[0])
    np.testing.assert_array_equal(r["out1"], np.bincount(g, weights=cols["m1"][ok], minlength=250).astype(np.uint64))
    np.testing.assert_array_equal(r["out2"], np.bincount(g, weights=cols["m2"][ok], minlength=250).astype(np.uint64))
    assert ok.sum() > 100


# --------------------------------------------------------------------- selection labels (section 5.2)
def test_size_targets_closed_form():
    """bits per value = 2^j - 1 gives the target j / 6 exactly: bytes = n (2^j - 1) / 8."""
    n = np.array([8, 64, 4096, 0], np.float64)
    for j in range(7):
        F = np.outer(np.where(n > 0, n, 8.0) * (2 ** j - 1) / 8, np.ones(6))
        F[-1] = (2 ** j - 1) / 8 * 8  # n = 0 counts as n = 1: bytes = (2^j - 1) / 8 per value
        t = O.size_targets(F, n)
        np.testing.assert_array_equal(t[:-1], np.full((3, 6), j / 6.0))
        np.testing.assert_allclose(t[-1], np.log2(1 + 8 * F[-1]) / 6, rtol=0, atol=0)


def test_cost_targets_closed_form():
    """picoseconds per value = 2^j - 1 gives j / 16: ns = n (2^j - 1) / 1000; negative times
    count as zero."""
    n = np.array([1000, 5000], np.float64)
    for j in range(0, 24, 3):
        C = np.outer(n * (2 ** j - 1) / 1000.0, np.ones(6))
        np.testing.assert_allclose(O.cost_targets(C, n), np.full((2, 6), j / 16.0), rtol=1e-15, atol=1e-15)
    assert np.all(O.cost_targets(np.full(6, -5.0), [10]) == 0.0)


def test_exhaustive_choice_hand_cases():
    rows = np.array([[5, 5, 5, 5, 5, 5], [9, 3, 3, 7, 1, 1], [0, 0, 1, 2, 3, 4], [7, 6, 5, 4, 3, 2]], np.uint64)
    np.testing.assert_array_equal(O.exhaustive_choice(rows), [0, 4, 0, 5])


def test_exhaustive_choice_is_the_smallest_encoding():
    """On tiny columns the choice names the format whose actual encoding is the smallest
    (the encoder's own footprint, not the closed-form one) at the lowest such kind."""
    for seed in range(40):
        n = int(datagen.stream(seed, 0, 1)[0] % 1500)
        v = (datagen.stream(seed + 100, 0, n) >> np.uint64(60 - seed % 20)).astype(np.uint32)
        if seed % 3 == 0:
            v = np.sort(v)
        sizes = [O.footprint(O.encode(v, k)) for k in O.KINDS]
        k = int(O.exhaustive_choice(O.footprints(v))[0])
        assert sizes[k] == min(sizes) and all(s > sizes[k] for s in sizes[:k]), (seed, sizes, k)


# --------------------------------------------------------------------- calc, join pairs, group-by
def test_calc_wraps_modulo_2_32():
    a = np.array([0xFFFFFFFF, 0, 0x10000, 3, 7, 0x80000000], np.uint32)
    b = np.array([1, 1, 0x10000, 0x55555556, 5, 2], np.uint32)
    np.testing.assert_array_equal(O.calc(a, b, O.CALC_ADD), [0, 1, 0x20000, 0x55555559, 12, 0x80000002])
    np.testing.assert_array_equal(O.calc(a, b, O.CALC_SUB), [0xFFFFFFFE, 0xFFFFFFFF, 0, 0xAAAAAAAD, 2, 0x7FFFFFFE])
    np.testing.assert_array_equal(O.calc(a, b, O.CALC_MUL), [0xFFFFFFFF, 0, 0, 2, 35, 0])
    v = datagen.uniform_bits(1, 5000, 32)
    w = datagen.uniform_bits(2, 5000, 32)
    np.testing.assert_array_equal(O.calc(O.calc(v, w, O.CALC_ADD), w, O.CALC_SUB), v)  # inverse operations
    np.testing.assert_array_equal(O.calc(v, np.ones(5000, np.uint32), O.CALC_MUL), v)
    with pytest.raises(O.OracleError):
        O.calc(v, w[:10], O.CALC_ADD)


def test_join_pairs_brute_force():
    for seed in range(30):
        D = 1 + int(datagen.stream(seed, 0, 1)[0] % 200)
        n = int(datagen.stream(seed, 1, 1)[0] % 400)
        keys = datagen.uniform_range(seed + 50, n, 0, D + 20)
        dim = datagen.uniform_range(seed + 90, D, 0, 10)
        s = O.select(dim, O.LT, 4)
        left, right = O.join_pairs(keys, O.bitmap_from_positions(s, D), D)
        pairs = [(i, j) for i in range(n) for j in s if keys[i] == j]
        assert [(int(a), int(b)) for a, b in zip(left, right)] == pairs
        # the left side is the semi-join
        np.testing.assert_array_equal(left, O.semijoin(keys, O.bitmap_from_positions(s, D), D))


def test_group_by_brute_force():
    for seed in range(30):
        n = int(datagen.stream(seed, 2, 1)[0] % 500)
        keys = datagen.uniform_range(seed + 7, n, 0, 1 + seed * 37)
        ids, distinct = O.group_by(keys)
        for i in range(n):
            assert ids[i] == sum(1 for d in set(int(x) for x in keys) if d < keys[i])
        assert all(distinct[j] < distinct[j + 1] for j in range(distinct.size - 1))
        np.testing.assert_array_equal(distinct[ids.astype(np.int64)] if n else distinct[:0], keys)
        assert ids.size == n and (n == 0 or ids.max() == distinct.size - 1)
