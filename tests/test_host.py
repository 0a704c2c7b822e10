"""Host-side logic of the package that runs without a GPU."""
import numpy as np
import pytest


def test_selector_struct_layout():
    """ms_train_cfg as the header lays it out: six 4-byte fields, then the 8-byte seed."""
    import ctypes
    from paper_2004_09350_amd import morphgpu as M
    assert ctypes.sizeof(M.TrainCfg) == 32 and M.TrainCfg.seed.offset == 24
    assert (M.NET_SIZE, M.NET_COST, M.OBJ_FOOTPRINT, M.OBJ_DECODE) == (0, 1, 0, 1)


def test_plan_step_layout():
    import ctypes
    from paper_2004_09350_amd import morphgpu as M
    assert ctypes.sizeof(M.Step) == 40 and ctypes.sizeof(M.Tune) == 16
    s = M.step(M.OP_SELECT, a=M.inp(2), cmp=M.LT, c0=103, out=M.fmt(M.DELTA_DYN_BP))
    assert (s.op, s.a, s.cmp, s.c0, s.out.kind) == (M.OP_SELECT, -3, M.LT, 103, M.DELTA_DYN_BP)


def test_generator_at_indices_matches_stream():
    from paper_2004_09350_amd import datagen
    idx = np.array([0, 1, 7, 999, 123456])
    full = datagen.uniform_range(17, 200_000, 5, 1000)
    np.testing.assert_array_equal(datagen.uniform_range_at(17, idx, 5, 1000), full[idx])
    np.testing.assert_array_equal(datagen.stream_at(3, idx), datagen.stream(3, 0, 200_000)[idx])
