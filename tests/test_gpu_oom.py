"""Allocation failure: an allocator callback that returns NULL at one chosen allocation.

Every operator, the column encoder and both plan paths are called with the k-th device
allocation failing, for every k until the call succeeds.  A failing call must raise OOM,
hand nothing back, and free every allocation it made before the failure (the live set of
callback allocations is unchanged); the call that succeeds must give the oracle's result,
and the library must keep working with the ordinary allocator afterwards."""
import numpy as np
import pytest

import oracle as O
import oracle.queries as OQ
from paper_2004_09350_amd import datagen
from tests._parity import assert_column

pytestmark = pytest.mark.gpu

MAX_ALLOCS = 64  # no single operator call makes more device allocations than this
MAX_PLAN_ALLOCS = 400  # nor an eager run of the star plan


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09350_amd import morphgpu
    morphgpu.init()
    return morphgpu


class FailingAllocator:
    """Callbacks that count allocations and fail allocation number `fail_at` (0-based)."""

    def __init__(self, M):
        import torch
        self.M, self.torch = M, torch
        self.fail_at, self.count, self.live, self.ever, self.double_frees = None, 0, set(), set(), []

        @M._ALLOC_T
        def alloc(nbytes, stream, ctx):
            i = self.count
            self.count += 1
            if self.fail_at is not None and i == self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
            self.live.add(p)
            self.ever.add(p)
            return p

        @M._FREE_T
        def free(ptr, nbytes, stream, ctx):
            if not ptr:
                return
            if ptr in self.live:
                self.live.discard(ptr)
            elif ptr in self.ever:
                self.double_frees.append(ptr)  # freed before and not handed out again since
                return
            torch.cuda.caching_allocator_delete(ptr)  # else: allocated before these callbacks

        self.alloc, self.free = alloc, free

    def __enter__(self):
        assert self.M.lib().ms_init(self.alloc, self.free, None) == 0
        return self

    def __exit__(self, *exc):
        self.M.sync()
        assert self.M.lib().ms_init(self.M._torch_alloc, self.M._torch_free, None) == 0
        assert not self.double_frees, f"{len(self.double_frees)} buffers freed twice"

    def sweep(self, call, check, limit=MAX_ALLOCS):
        """Runs call() with allocation k failing for k = 0, 1, ... until it succeeds."""
        for k in range(limit):
            before = set(self.live)
            self.fail_at, self.count = k, 0
            try:
                out = call()
            except self.M.MorphError as e:
                self.fail_at = None
                assert e.status == "OOM", f"allocation {k} failing raised {e}"
                self.M.sync()
                assert self.live == before, f"allocation {k} failing leaked {len(self.live - before)} buffers"
                continue
            self.fail_at = None
            assert self.count <= k, "the call succeeded although an allocation failed"
            self.M.sync()
            check(out)
            return k
        raise AssertionError(f"the call still fails with {limit} allocations allowed")


def test_operators_report_oom_and_leak_nothing(M):
    n = 70_001
    v = datagen.uniform_bits(501, n, 14)
    g = datagen.uniform_range(502, n, 0, 300)
    pa = O.select(datagen.uniform_bits(503, n, 10), O.LT, 300)
    pb = O.select(datagen.uniform_bits(504, n, 10), O.LT, 700)
    D = 5_000
    keys = datagen.uniform_range(505, n, 0, D)
    s_dim = O.select(datagen.uniform_range(506, D, 0, 100), O.LT, 40)
    pos = datagen.uniform_range(507, n // 3, 0, n)
    with FailingAllocator(M) as fa:
        cols = {}
        for kind in O.KINDS:  # the encoder itself, every format
            fa.sweep(lambda: M.encode(v, M.fmt(kind)), lambda c, kind=kind: assert_column(c, v, kind))
            cols[kind] = M.encode(v, M.fmt(kind))
        cg = M.encode(g, M.fmt(M.STATIC_BP))
        ca, cb = M.encode(pa, M.fmt(M.DELTA_DYN_BP)), M.encode(pb, M.fmt(M.DYN_BP))
        ck = M.encode(keys, M.fmt(M.FOR_DYN_BP))
        cpos = M.encode(pos, M.fmt(M.STATIC_BP))
        bm = M.bitmap_from_positions(M.encode(s_dim, M.fmt(M.DELTA_DYN_BP)), D)
        want_sel = O.select(v, O.LT, 5000)
        for kin in O.KINDS:
            for kout in (M.STATIC_BP, M.RLE, M.DELTA_DYN_BP):
                fa.sweep(lambda: M.select(cols[kin], M.LT, 5000, f=M.fmt(kout)),
                         lambda c, kout=kout: assert_column(c, want_sel, kout))
                fa.sweep(lambda: M.morph(cols[kin], M.fmt(kout)), lambda c, kout=kout: assert_column(c, v, kout))
                fa.sweep(lambda: M.project(cols[kin], cpos, M.fmt(kout)),
                         lambda c, kout=kout: assert_column(c, O.project(v, pos), kout))
        for kout in (M.UNCOMPR, M.FOR_DYN_BP, M.RLE):
            fa.sweep(lambda: M.intersect(ca, cb, n, M.fmt(kout)),
                     lambda c, kout=kout: assert_column(c, O.intersect(pa, pb), kout))
            fa.sweep(lambda: M.semijoin(ck, bm, D, M.fmt(kout)),
                     lambda c, kout=kout: assert_column(c, O.semijoin(keys, O.bitmap_from_positions(s_dim, D), D),
                                                        kout))
        fa.sweep(lambda: M.group_sum(cg, cols[M.DYN_BP], 300),
                 lambda r: np.testing.assert_array_equal(M.u64(r), O.group_sum(g, v, 300)))
        fa.sweep(lambda: M.group_sum(cg, cols[M.RLE], 300_000),
                 lambda r: np.testing.assert_array_equal(M.u64(r), O.group_sum(g, v, 300_000)))
        ids_w, distinct_w = O.group_by(g)
        fa.sweep(lambda: M.group_by(cg, 300, M.fmt(M.STATIC_BP), M.fmt(M.RLE)),
                 lambda r: (assert_column(r[0], ids_w, M.STATIC_BP), assert_column(r[1], distinct_w, M.RLE)))
        fa.sweep(lambda: M.calc(cols[M.DYN_BP], cols[M.RLE], M.CALC_MUL, M.fmt(M.FOR_DYN_BP)),
                 lambda c: assert_column(c, O.calc(v, v, O.CALC_MUL), M.FOR_DYN_BP))
    # the ordinary allocator again
    assert_column(M.select(cols[M.STATIC_BP], M.LT, 5000, f=M.fmt(M.DYN_BP)), want_sel, M.DYN_BP)
    M.sync()


def test_plan_run_and_launch_report_oom(M):
    from paper_2004_09350_amd import queries
    dims = (2_000, 30_000, 20_000, 250)
    n = 150_001
    cols = datagen.star_columns(77, n, dims)
    thr = datagen.star_thresholds(datagen.STAR_WIDE)
    want = OQ.q3(cols, thr, dims)

    def check(_):
        o1, o2 = q.results()
        np.testing.assert_array_equal(o1, want["out1"])
        np.testing.assert_array_equal(o2, want["out2"])

    with FailingAllocator(M) as fa:
        enc = {k: M.encode(v, M.fmt(M.STATIC_BP)) for k, v in cols.items()}
        live0 = set(fa.live)
        q = queries.Q3(enc, thr, dims, n)
        k_run = fa.sweep(lambda: q.plan.run(), check, MAX_PLAN_ALLOCS)
        q.plan.set_tune(2, 0)
        k_launch = fa.sweep(lambda: q.plan.launch(), check)
        assert k_run > 0 and k_launch > 0
        q.plan.launch()  # a replay of the graph captured last
        M.sync()
        check(None)
        q.plan.close()
        assert fa.live == live0, "plan results or the arena outlived the plan"
    q = queries.Q3(enc, thr, dims, n)  # the ordinary allocator again
    q.plan.run()
    M.sync()
    check(None)
    q.plan.close()
