"""The learned format selector end to end on the GPU: training data produced by the
engine (statistics + exact footprints of star-plan intermediates), training with the
library's own kernels, and its picks on star plans with other seeds compared with
exhaustive selection, an untrained network and the naive all-static-BP plan."""
import numpy as np
import pytest

import oracle as O
import oracle.queries as OQ
from paper_2004_09350_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu, selector
    morphgpu.init()
    return selector


def test_collect_labels_match_oracle(S):
    X, F, N, names = S.collect(2, seed0=20_000, n_lo=2e5, n_hi=4e5)
    assert X.shape == (len(names), 32) and F.shape == (len(names), 6)
    # recompute the first plan's intermediates with the oracle and compare labels
    u = datagen.stream(20_000 * 7919, 0, 5).astype(np.float64) / 2.0 ** 64
    n_fact = int(np.exp(np.log(2e5) + u[0] * (np.log(4e5) - np.log(2e5))))
    sel = [0.01 + 0.19 * x for x in u[1:5]]
    cols = datagen.star_columns(20_000 * 100 + 1, n_fact)
    want = OQ.q3(cols, datagen.star_thresholds(sel), datagen.STAR_DIM_SIZES)
    k = len(want["intermediates"])  # the first plan's intermediates come first
    assert names[:k] == list(want["intermediates"])  # same order as the oracle's plan
    for i, name in enumerate(names[:k]):
        inter = want["intermediates"][name]
        np.testing.assert_array_equal(F[i], O.footprints(inter), err_msg=name)
        np.testing.assert_allclose(X[i].astype(np.float64), O.stats(inter), atol=1e-6, err_msg=name)
        assert N[i] == inter.size


def test_learned_selector_gain(S):
    import torch
    X, F, N, _ = S.collect(48, seed0=30_000, n_lo=1e5, n_hi=2e6)
    T = S.targets(F, N)
    p = S.train(X, T, epochs=80, batch=256, lr=2e-3)
    p0 = torch.from_numpy(datagen.mlp_init(77)).cuda()
    # evaluation: star plans with the evaluation seeds (wide and narrow filters)
    Xe, Fe = [], []
    from paper_2004_09350_amd.queries import Q3
    for seed, sel in ((1, datagen.STAR_WIDE), (2, datagen.STAR_NARROW)):
        cols, _ = S.star_inputs(seed, 1_000_000)
        q = Q3(cols, datagen.star_thresholds(sel), datagen.STAR_DIM_SIZES, 1_000_000, extra=("stats", "footprints"))
        q.plan.run()
        for name in q.names:
            Xe.append(q.plan.read(q.stats_step[name]))
            Fe.append(q.plan.read(q.fp_step[name]))
        q.plan.close()
    Xe, Fe = np.stack(Xe), np.stack(Fe)
    learned = S.regret(Fe, S.pick(p, Xe))
    untrained = S.regret(Fe, S.pick(p0, Xe))
    static = S.regret(Fe, np.full(len(Fe), 1))
    uncompr = S.regret(Fe, np.zeros(len(Fe), int))
    print(f"regret: learned {learned:.4f} untrained {untrained:.4f} all-static {static:.4f} "
          f"all-uncompressed {uncompr:.4f}")
    assert learned <= 0.05
    assert learned < untrained and learned < static and learned < uncompr
