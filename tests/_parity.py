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
        if int(w.sum()):
            # every block's words, gathered through both directories
            go, eo = got["offsets"].astype(np.int64), exp["offsets"].astype(np.int64)
            blk = np.repeat(np.arange(w.size), w)
            within = np.arange(blk.size) - np.repeat(np.cumsum(w) - w, w)
            gw, ew = got["payload"][go[blk] + within], exp["payload"][eo[blk] + within]
            if not np.array_equal(gw, ew):
                bad = np.nonzero(gw != ew)[0]
                raise AssertionError(f"payload words differ in {np.unique(blk[bad]).size} blocks, first block "
                                     f"{blk[bad[0]]} word {within[bad[0]]}")
        if canonical:
            np.testing.assert_array_equal(got["offsets"], exp["offsets"])
            np.testing.assert_array_equal(got["payload"][: exp["payload_words"]], exp["payload"])
    elif kind == O.RLE:
        np.testing.assert_array_equal(got["rvalues"], exp["rvalues"])
        np.testing.assert_array_equal(got["rstarts"], exp["rstarts"])
    else:
        np.testing.assert_array_equal(got["payload"][: values.size], values)
    return got
