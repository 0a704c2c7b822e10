"""Helpers that compare GPU columns with the oracle (used by the GPU tests)."""
import numpy as np

import oracle as O


def expected_sections(values, kind, bit_width=O.BW_AUTO):
    return O.encode(np.asarray(values, np.uint32), kind, bit_width)


def assert_column(col, values, kind, bit_width=O.BW_AUTO, canonical=False):
    """GPU column == oracle encoding of `values`: decoded contents, per-block widths,
    bases and payload words, remainder, runs and footprint.  With canonical=True the
    whole payload must match word for word (count-known producers after shrink)."""
    values = np.asarray(values, np.uint32)
    got = col.sections()
    exp = expected_sections(values, kind, bit_width)
    assert got["kind"] == kind
    assert got["n"] == values.size, (got["n"], values.size)
    dec = O.decode(got)
    if not np.array_equal(dec, values):
        bad = np.nonzero(dec != values)[0]
        raise AssertionError(f"decoded contents differ at {bad.size} places, first {bad[:5]}: "
                             f"got {dec[bad[:5]]} want {values[bad[:5]]}")
    assert got["footprint"] == exp["footprint"], (got["footprint"], exp["footprint"])
    if kind == O.STATIC_BP:
        assert got["bit_width"] == exp["bit_width"]
        w = exp["payload_words"]
        np.testing.assert_array_equal(got["payload"][:w], exp["payload"])
        np.testing.assert_array_equal(got["rem"], exp["rem"])
    elif kind in (O.DYN_BP, O.DELTA_DYN_BP, O.FOR_DYN_BP):
        np.testing.assert_array_equal(got["widths"], exp["widths"])
        if kind != O.DYN_BP:
            np.testing.assert_array_equal(got["bases"], exp["bases"])
        np.testing.assert_array_equal(got["rem"], exp["rem"])
        w = exp["widths"].astype(np.int64) * 16
        if w.size:
            # gather each block's words through both directories
            rel = np.arange(int(w.max()) if w.max() else 0)
            for k in np.nonzero(w)[0][:: max(1, w.size // 4096)] if w.size > 4096 else np.nonzero(w)[0]:
                g0, e0 = int(got["offsets"][k]), int(exp["offsets"][k])
                np.testing.assert_array_equal(got["payload"][g0:g0 + w[k]], exp["payload"][e0:e0 + w[k]],
                                              err_msg=f"block {k}")
            del rel
        if canonical:
            np.testing.assert_array_equal(got["offsets"], exp["offsets"])
            np.testing.assert_array_equal(got["payload"][: exp["payload_words"]], exp["payload"])
    elif kind == O.RLE:
        np.testing.assert_array_equal(got["rvalues"], exp["rvalues"])
        np.testing.assert_array_equal(got["rstarts"], exp["rstarts"])
    else:
        np.testing.assert_array_equal(got["payload"][: values.size], values)
    return got
