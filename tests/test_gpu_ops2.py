"""GPU parity of the wider operator set against the oracle: calc (every operation, input
and output format), the join emitting position pairs, and the group-by that assigns its
own group ids, followed by a group-sum over those ids.  Column results are compared block
by block with the oracle's encoding of the expected values."""
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


SIZES = [0, 1, 511, 513, 100_003, 1_000_123]


@pytest.mark.parametrize("n", SIZES)
def test_calc_all_formats(M, n):
    a = datagen.uniform_bits(301, n, 20)
    b = datagen.runs(302, n)
    for op in (O.CALC_ADD, O.CALC_SUB, O.CALC_MUL):
        want = O.calc(a, b, op)
        for ka in O.KINDS:
            ca = M.encode(a, M.fmt(ka))
            cb = M.encode(b, M.fmt((ka + 2) % 6))
            kouts = O.KINDS if (ka == O.STATIC_BP or n == 100_003) else (O.STATIC_BP, O.DELTA_DYN_BP)
            for kout in kouts:
                assert_column(M.calc(ca, cb, op, M.fmt(kout)), want, kout)
    M.sync()


def test_calc_length_mismatch(M):
    a = M.encode(datagen.uniform_bits(1, 1000, 8), M.fmt(M.STATIC_BP))
    b = M.encode(datagen.uniform_bits(2, 999, 8), M.fmt(M.STATIC_BP))
    with pytest.raises(M.MorphError):
        M.calc(a, b, M.CALC_ADD)
    with pytest.raises(M.MorphError):
        M.calc(a, a, 7)


@pytest.mark.parametrize("n", [0, 1, 4097, 1_000_123])
@pytest.mark.parametrize("D", [1, 2500, 3_000_000])
def test_join_pairs(M, n, D):
    keys = datagen.uniform_range(310 + D % 97, n, 0, D + D // 10 + 1)  # some keys beyond the domain
    dim = datagen.uniform_range(311, D, 0, 100)
    s = O.select(dim, O.LT, 20)
    bm_h = O.bitmap_from_positions(s, D)
    want_l, want_r = O.join_pairs(keys, bm_h, D)
    bm = M.bitmap_from_positions(M.encode(s, M.fmt(M.DELTA_DYN_BP)), D)
    for kin in (O.STATIC_BP, O.DYN_BP, O.RLE):
        ck = M.encode(keys, M.fmt(kin))
        for kl, kr in ((O.DELTA_DYN_BP, O.STATIC_BP), (O.UNCOMPR, O.FOR_DYN_BP), (O.RLE, O.DYN_BP)):
            left, right = M.join(ck, bm, D, M.fmt(kl), M.fmt(kr))
            assert_column(left, want_l, kl)
            assert_column(right, want_r, kr)
    M.sync()


@pytest.mark.parametrize("n", [0, 1, 600, 100_003, 2_000_017])
@pytest.mark.parametrize("domain", [1, 250, 70_000, 1 << 24])
def test_group_by_and_group_sum(M, n, domain):
    keys = datagen.uniform_range(320 + domain % 13, n, 0, min(domain, 1 << 20))
    vals = datagen.uniform_bits(321, n, 17)
    ids_w, distinct_w = O.group_by(keys)
    ck = M.encode(keys, M.fmt(M.DYN_BP))
    for ki, kd in ((O.STATIC_BP, O.DELTA_DYN_BP), (O.UNCOMPR, O.STATIC_BP), (O.RLE, O.UNCOMPR), (O.FOR_DYN_BP,
                                                                                                 O.RLE)):
        ids, distinct = M.group_by(ck, domain, M.fmt(ki), M.fmt(kd))
        assert_column(ids, ids_w, ki)
        assert_column(distinct, distinct_w, kd)
    G = max(1, distinct_w.size)
    got = M.u64(M.group_sum(ids, M.encode(vals, M.fmt(M.STATIC_BP)), G))
    np.testing.assert_array_equal(got, O.group_sum(ids_w, vals, G))
    M.sync()


def test_group_by_key_out_of_domain(M):
    ck = M.encode(np.array([1, 5, 9, 2], np.uint32), M.fmt(M.UNCOMPR))
    ids, distinct = M.group_by(ck, 8)
    with pytest.raises(M.MorphError) as e:
        M.sync()
    assert e.value.status == "OUT_OF_RANGE"
    with pytest.raises(M.MorphError):
        M.group_by(ck, 0)
    with pytest.raises(M.MorphError):
        M.group_by(ck, (1 << 28) + 1)
