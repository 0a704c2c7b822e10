"""The chunked evaluation of the oracle's star query (used by the full-size GPU parity
test) equals the whole-table evaluation: chunks that cut the table unevenly, both filter
settings."""
import numpy as np
import pytest

import oracle.queries as OQ
from paper_2004_09350_amd import datagen
from tests._oracle_star import oracle_star


@pytest.mark.parametrize("sel", [datagen.STAR_WIDE, datagen.STAR_NARROW])
def test_oracle_star_chunking_is_exact(sel):
    n = 1_000_003
    thr = datagen.star_thresholds(sel)
    whole = OQ.q3(datagen.star_columns(3, n), thr, datagen.STAR_DIM_SIZES)
    P, o1, o2 = oracle_star(3, n, thr, chunk=300_007)
    np.testing.assert_array_equal(P, whole["intermediates"]["P"])
    np.testing.assert_array_equal(o1, whole["out1"])
    np.testing.assert_array_equal(o2, whole["out2"])
    assert P.size > 0
