"""Host-side logic of the package that runs without a GPU."""
import numpy as np
import pytest


def test_selector_targets_and_regret():
    from paper_2004_09350_amd import selector as S
    fp = np.array([[4000, 1250, 1300, 400, 900, 8000], [0, 0, 0, 0, 0, 0]], np.uint64)
    n = np.array([1000, 0])
    t = S.targets(fp, n)
    # bits per value 32, 10, 10.4, 3.2, 7.2, 64 -> log2(1 + b) / 6
    np.testing.assert_allclose(t[0], np.log2(1 + np.array([32, 10, 10.4, 3.2, 7.2, 64])) / 6, rtol=1e-6)
    assert (t[1] == 0).all()
    assert S.regret(fp[:1], np.array([3])) == 0.0
    assert S.regret(fp[:1], np.array([1])) == pytest.approx(1250 / 400 - 1)
    # regret sums footprints over intermediates before dividing
    F = np.array([[100, 50, 60, 70, 80, 90], [10, 20, 30, 40, 5, 60]], np.uint64)
    assert S.regret(F, np.array([1, 0])) == pytest.approx((50 + 10) / (50 + 5) - 1)


def test_plan_step_layout():
    import ctypes
    from paper_2004_09350_amd import morphgpu as M
    assert ctypes.sizeof(M.Step) == 40 and ctypes.sizeof(M.Tune) == 8
    s = M.step(M.OP_SELECT, a=M.inp(2), cmp=M.LT, c0=103, out=M.fmt(M.DELTA_DYN_BP))
    assert (s.op, s.a, s.cmp, s.c0, s.out.kind) == (M.OP_SELECT, -3, M.LT, 103, M.DELTA_DYN_BP)


def test_generator_at_indices_matches_stream():
    from paper_2004_09350_amd import datagen
    idx = np.array([0, 1, 7, 999, 123456])
    full = datagen.uniform_range(17, 200_000, 5, 1000)
    np.testing.assert_array_equal(datagen.uniform_range_at(17, idx, 5, 1000), full[idx])
    np.testing.assert_array_equal(datagen.stream_at(3, idx), datagen.stream(3, 0, 200_000)[idx])
