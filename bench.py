"""Benchmark on one MI355X.

Default: the fused star query (6e8 fact rows, static-BP base columns) under six format
policies -- plain uncompressed execution (uncompressed base columns and intermediates),
uncompressed intermediates, all static BP, exhaustive selection, and the learned
selector's picks for footprint and for decode time -- each run eagerly and as an
autotuned captured graph, every run timed cold (a 2 GiB write evicts the caches between
runs); the value is the uncompressed-equivalent GB/s of the learned plan's graph.  The
line also carries the footprint regret against exhaustive selection, the roofline of
the dominant kernel, measured copy bandwidth, the CPU oracle (one thread and all cores)
and, under "sweep", the operator/format sweep:

One sweep step = one pass of the whole sweep (every row of the hot path that applies to
single operators): for each of six value distributions (uniform 4/12/24/32-bit,
sorted with small gaps, runs of mean length 64), each stored in each of the six
formats:
  * select at 1 %, 10 % and 50 % selectivity, each emitting every output format;
  * project of the column at P = select(U12, 10 %), emitting every output format;
  * sum;
plus intersect of two delta-compressed position lists (10 % and 50 %) emitting
every format, and morph between every ordered pair of formats.

Printed: one JSON line with the uncompressed-equivalent throughput of the step
(value), the fraction of HBM peak on compressed bytes, the roofline of the
dominant kernel (per-launch HIP events on the launch stream) and the CPU oracle
timed on a bounded sample of the same sweep.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LDS_BITMAP_BITS = 1 << 18  # semi-join bitmaps up to this many bits sit whole in a workgroup's dynamic LDS
DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")
SELECTIVITIES = (0.01, 0.10, 0.50)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="star", choices=("sweep", "star", "batch", "q1"),
                    help="star: the fused star query under every format policy (default; the operator/format "
                         "sweep rides along unless --no-sweep); sweep: operator/format sweep alone; batch: 512 "
                         "mixed tasks, one graph vs one launch sequence per task; q1: the simple "
                         "select-project-sum query")
    ap.add_argument("--no-sweep", action="store_true", help="star: skip the operator/format sweep")
    ap.add_argument("--greedy", action="store_true",
                    help="star: add the greedy runtime search policy (hundreds of full-size plan captures)")
    ap.add_argument("--star-tune", default=None,
                    help="star: fixed launch shape 'branches,wg_per_cu,chunks_per_wg,batch' (default: STAR_TUNE)")
    ap.add_argument("--star-autotune", action="store_true",
                    help="star: autotune every policy's plan at full size instead of the fixed launch shape")
    ap.add_argument("--sweep-steps", type=int, default=2)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=None, help="rows per column (default per workload)")
    ap.add_argument("--seeds", default="1", help="star: comma-separated instance seeds")
    ap.add_argument("--tasks", type=int, default=512, help="batch: number of tasks")
    ap.add_argument("--weights", default=None, help="star: selector weights (.npy); default: the packaged ones")
    ap.add_argument("--cpu-rows", type=int, default=None,
                    help="rows of the CPU oracle sample (default per workload: sweep 1.2e6, star 4e7, batch 1e6 per task)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="fewer operators (for profiling runs)")
    ap.add_argument("--dump", default=None, help="write per-operator kernel timings (JSON) to this file")
    ap.add_argument("--calib-copy", action="store_true",
                    help="decode one uncompressed column first (k_decode: 4 B read + 4 B written per row), the "
                         "known-size reference for scaling HBM counters")
    return ap.parse_args()


def source_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_09350_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".inc")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def thresholds(dist: str, values_sorted_probe=None):
    """Constant c of `v < c` per selectivity (value quantiles of each distribution)."""
    out = []
    for s in SELECTIVITIES:
        if dist.startswith("U"):
            b = int(dist[1:])
            out.append(max(1, int(round(s * (1 << b)))) if b < 32 else int(s * (1 << 32)))
        elif dist == "RUNS":
            out.append(int(s * (1 << 16)))
        else:
            out.append(int(values_sorted_probe(s)))
    return out


class Sweep:
    """The operator list of one step plus the byte accounting of every operator."""

    def __init__(self, M, gen, n: int, quick: bool = False, log=print):
        self.M, self.n = M, n
        self.cols = {}      # (dist, kind) -> Column
        self.thr = {}
        self.log = log
        t0 = time.time()
        for di, d in enumerate(DISTS):
            raw = gen.sweep_column(d, 7000 + di, n)
            if d == "SORTED":
                probe = lambda s, raw=raw: int(raw[min(n - 1, int(s * n))].item()) & 0xFFFFFFFF
            else:
                probe = None
            self.thr[d] = thresholds(d, probe)
            for k in M.KINDS:
                self.cols[(d, k)] = M.encode(raw, M.fmt(k))
            del raw
            M.sync()
        # positions for project and intersect
        u12b = M.encode(gen.uniform_bits(7100, n, 12), M.fmt(M.STATIC_BP, 12))
        self.P = M.select(self.cols[("U12", M.STATIC_BP)], M.LT, self.thr["U12"][1], 0, M.fmt(M.DELTA_DYN_BP))
        self.Pa = self.P
        self.Pb = M.select(u12b, M.LT, self.thr["U12"][2], 0, M.fmt(M.DELTA_DYN_BP))
        del u12b
        M.sync()
        self.ops = self._ops(quick)
        log(f"setup {time.time() - t0:.1f}s, {len(self.ops)} operators per step")

    def _ops(self, quick):
        M = self.M
        ops = []
        kinds = M.KINDS
        for d in DISTS:
            for kin in kinds:
                for si, c in enumerate(self.thr[d]):
                    for kout in kinds:
                        ops.append(("select", (d, kin), c, kout))
                for kout in kinds:
                    ops.append(("project", (d, kin), None, kout))
                ops.append(("sum", (d, kin), None, None))
            for kin in kinds:
                for kout in kinds:
                    if kin != kout:
                        ops.append(("morph", (d, kin), None, kout))
        for kout in kinds:
            ops.append(("intersect", None, None, kout))
        if quick:
            ops = ops[::7]
        return ops

    def run_op(self, op):
        M = self.M
        name, key, c, kout = op
        if name == "select":
            return M.select(self.cols[key], M.LT, c, 0, M.fmt(kout))
        if name == "project":
            return M.project(self.cols[key], self.P, M.fmt(kout))
        if name == "sum":
            return M.sum_(self.cols[key], out=self._sum_out)
        if name == "morph":
            return M.morph(self.cols[key], M.fmt(kout))
        if name == "intersect":
            return M.intersect(self.Pa, self.Pb, self.n, M.fmt(kout))
        raise ValueError(name)

    def step(self):
        for op in self.ops:
            out = self.run_op(op)
            del out

    def account(self):
        """Run each operator once, synchronously, and record its uncompressed-equivalent
        bytes and its algorithmic compressed bytes split over the kernels it launches."""
        M = self.M
        self._sum_out = __import__("torch").empty(1, dtype=__import__("torch").int64, device="cuda")
        info = {k: c.info() for k, c in self.cols.items()}
        pinfo = self.P.info()
        pa, pb = self.Pa.info(), self.Pb.info()
        n = self.n
        # fraction of 64-byte sectors of a 4-byte column touched by the project positions
        pos = M.u32(self.P.decode())
        frac = np.unique(pos >> 4).size / ((n + 15) // 16)
        self.acct = []
        M.prof_enable(True)
        M.prof_reset()
        for op in self.ops:
            r0 = M.prof_count()
            out = self.run_op(op)
            M.sync()
            recs = M.prof_records(r0)
            name, key, c, kout = op
            oi = out.info() if hasattr(out, "info") else None
            fin = info[key]["footprint"] if key else None
            if name == "select":
                ue = 4 * (n + oi["n"])
                alg = {"k_pred": fin, "k_emit": oi["footprint"]}
            elif name == "project":
                ue = 4 * (2 * pinfo["n"]) + int(4 * 16 * frac * ((n + 15) // 16))
                data = int(frac * fin)
                alg = {"k_project": pinfo["footprint"] + oi["footprint"] + data,
                       "k_project_rle": pinfo["footprint"] + oi["footprint"] + data,
                       "k_rle_count_proj": pinfo["footprint"] + data, "k_rle_emit_proj": oi["footprint"]}
            elif name == "sum":
                ue = 4 * n + 8
                alg = {"k_sum": fin}
            elif name == "morph":
                ue = 8 * n
                alg = {"k_morph": fin + oi["footprint"], "k_rle_count": fin, "k_rle_emit": oi["footprint"]}
            else:
                ue = 4 * (pa["n"] + pb["n"] + oi["n"])
                probe, build = (pa, pb) if pa["n"] <= pb["n"] else (pb, pa)
                alg = {"k_bitmap": build["footprint"], "k_pred": probe["footprint"],
                       "k_emit_vals": probe["footprint"] + oi["footprint"]}
            kernels = [r[0] for r in recs]
            alg_k = {}
            for k in set(kernels):
                base = k.split("<")[0]  # template instances share their family's byte accounting
                if base in alg:
                    alg_k[k] = alg[base]
            self.acct.append(dict(op=op, ue=ue, alg=sum(alg_k.values()), alg_by_kernel=alg_k, recs=recs,
                                  out_fp=oi["footprint"] if oi else 0))
            del out
        M.prof_enable(False)
        M.prof_reset()


def roofline(acct, kernel_times=None):
    """Dominant kernel by total time; achieved = its algorithmic bytes / its time."""
    tot_t, tot_b, cnt = {}, {}, {}
    for a in acct:
        seen = set()
        for k, ms in a["recs"]:
            tot_t[k] = tot_t.get(k, 0.0) + ms
            cnt[k] = cnt.get(k, 0) + 1
            if k not in seen:
                tot_b[k] = tot_b.get(k, 0) + a["alg_by_kernel"].get(k, 0)
                seen.add(k)
    dom = max(tot_t, key=tot_t.get)
    avg_ms = tot_t[dom] / cnt[dom]
    bytes_per_launch = tot_b.get(dom, 0) / cnt[dom]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    share = tot_t[dom] / sum(tot_t.values())
    return dom, dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None), dict(
        kernel=dom, launches=cnt[dom], avg_ms=round(avg_ms, 4), bytes_per_launch=int(bytes_per_launch),
        share_of_step=round(share, 3), per_kernel_ms={k: round(v, 2) for k, v in sorted(tot_t.items())})


def cpu_baseline(rows: int):
    """The oracle on the same sweep over the first `rows` rows (single thread)."""
    import oracle as O
    from paper_2004_09350_amd import datagen
    cols = {}
    for di, d in enumerate(DISTS):
        cols[d] = datagen.sweep_column(d, 7000 + di, rows)
    enc = {(d, k): O.encode(cols[d], k) for d in DISTS for k in O.KINDS}
    thr = {}
    for d in DISTS:
        thr[d] = thresholds(d, (lambda s, v=cols[d]: int(v[min(rows - 1, int(s * rows))])) if d == "SORTED" else None)
    u12b = datagen.uniform_bits(7100, rows, 12)
    ue = 0
    t0 = time.perf_counter()
    P = O.select(O.decode(enc[("U12", O.STATIC_BP)]), O.LT, thr["U12"][1])
    Pb = O.select(u12b, O.LT, thr["U12"][2])
    for d in DISTS:
        for kin in O.KINDS:
            for c in thr[d]:
                v = O.decode(enc[(d, kin)])
                p = O.select(v, O.LT, c)
                for kout in O.KINDS:
                    O.encode(p, kout)
                    ue += 4 * (rows + p.size)
            v = O.decode(enc[(d, kin)])
            pr = O.project(v, P)
            for kout in O.KINDS:
                O.encode(pr, kout)
                ue += 8 * P.size
            O.sum_(O.decode(enc[(d, kin)]))
            ue += 4 * rows + 8
        for kin in O.KINDS:
            v = O.decode(enc[(d, kin)])
            for kout in O.KINDS:
                if kin != kout:
                    O.encode(v, kout)
                    ue += 8 * rows
    r = O.intersect(P, Pb)
    for kout in O.KINDS:
        O.encode(r, kout)
        ue += 4 * (P.size + Pb.size + r.size)
    dt = time.perf_counter() - t0
    return dict(value=round(ue / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample=f"the same sweep on the first {rows} rows of each column, single thread, "
                       f"{dt:.1f} s", seconds=round(dt, 2))


KIND_NAMES = ("UNCOMPR", "STATIC_BP", "DYN_BP", "DELTA_DYN_BP", "FOR_DYN_BP", "RLE")


def calib_copy(M, log, col, rows):
    """Decode an uncompressed column once: the known-size reference (4 B read + 4 B
    written per row) that scales the HBM counters."""
    dst = col.decode()
    M.sync()
    log(f"calibration copy: k_decode of {rows} rows ({4 * rows} B read, {4 * rows} B written)")
    del dst


def traffic_for(kernel: str, name: str = "traffic"):
    """HBM bytes per launch of `kernel` from the committed counter summary of the same
    workload (profiles/<name>.json), while its source hash matches the kernels being
    measured (else None)."""
    f = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(f):
        return None
    try:
        t = json.load(open(f))
        if t.get("source_sha") == source_sha() and kernel in t.get("kernels", {}):
            return t["kernels"][kernel]["bytes_per_launch"]
    except Exception:
        pass
    return None


def base_line(args, metric, value, unit, dt, workload, extra_config=None):
    cfg = {"workload": workload}
    cfg.update(extra_config or {})
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic", "config": cfg}


def run_sweep(args, M, gen, torch, log):
    rows = args.rows or 100_000_000
    sw = Sweep(M, gen, rows, args.quick, log)
    if args.calib_copy:
        calib_copy(M, log, sw.cols[("U32", M.UNCOMPR)], rows)
    sw.account()
    log("accounting pass done")
    if args.dump:
        KN = M.KIND_NAMES
        rows_ = []
        for a in sw.acct:
            name, key, c, kout = a["op"]
            rows_.append(dict(op=name, dist=key[0] if key else None, kin=KN[key[1]] if key else None, c=c,
                              kout=KN[kout] if kout is not None else None, recs=a["recs"], alg=a["alg"],
                              ue=a["ue"], out_fp=a["out_fp"]))
        json.dump(rows_, open(args.dump, "w"))
    for _ in range(args.warmup):
        sw.step()
    M.sync()
    log("warmup done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sw.step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} {time.perf_counter() - t0:.2f}s")
    M.sync()
    dt = (time.perf_counter() - t0) / args.steps
    ue = sum(a["ue"] for a in sw.acct)
    alg = sum(a["alg"] for a in sw.acct)
    dom, roof, dominfo = roofline(sw.acct)
    res = base_line(args, "uncompressed-equivalent GB/s of the fused operator sweep (plus %HBM roofline on "
                          "compressed bytes)", round(ue / dt / 1e9, 2), "GB/s", dt,
                    "operator/format sweep: 6 distributions x 6 formats of 1e8-row uint32 columns; select "
                    "1/10/50 % -> 6 formats, project at a 10 % position list -> 6 formats, sum, intersect -> 6 "
                    "formats, morph between all 30 format pairs", {"rows": rows, "operators_per_step": len(sw.ops)})
    res.update(hbm_frac_step=round(alg / dt / 1e9 / HBM_PEAK_GBS, 4), roofline=roof, dominant_kernel=dominfo,
               source_sha=source_sha())
    res["roofline"]["traffic"] = traffic_for(dom)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.cpu_rows or 1_200_000)
    return res


# ------------------------------------------------------------------------------ plans
def sectors_touched(M, pos_col) -> int:
    """Distinct 64-byte sectors of a 4-byte column touched by a position list."""
    import torch
    p = pos_col.decode().to(torch.int64) & 0xFFFFFFFF
    return int(torch.unique(p >> 4).numel()) if p.numel() else 0


def plan_account(M, plan, inputs, log=None):
    """Uncompressed-equivalent and algorithmic bytes of every step of a plan's last run,
    the latter split over the kernels each step launches (same rules as the sweep)."""
    steps = plan.steps
    info = {}

    def col(ref):
        return inputs[-1 - ref] if ref < 0 else plan.column(ref)

    def inf(ref):
        if ref not in info:
            info[ref] = col(ref).info()
        return info[ref]

    ue_total, alg = 0, {}

    def add(k, b):
        alg[k] = alg.get(k, 0) + int(b)

    for i, s in enumerate(steps):
        op = s.op
        if op in (M.OP_MORPH, M.OP_SELECT, M.OP_SEMIJOIN, M.OP_PROJECT, M.OP_INTERSECT):
            out = inf(i)
            kout = KIND_NAMES[s.out.kind]
        if op == M.OP_MORPH:
            a = inf(s.a)
            ue_total += 8 * a["n"]
            if s.out.kind == M.RLE:
                add("k_rle_count", a["footprint"]); add("k_rle_emit", out["footprint"])
            else:
                add(f"k_morph<{kout}>", a["footprint"] + out["footprint"])
        elif op in (M.OP_SELECT, M.OP_SEMIJOIN):
            a = inf(s.a)
            ue_total += 4 * (a["n"] + out["n"])
            if op == M.OP_SELECT:
                kpred = "k_pred<0>"
            else:  # bitmaps beyond the workgroup's dynamic LDS go to the 1024-thread wide-LDS kernel
                kpred = "k_semijoin_wide" if s.param > LDS_BITMAP_BITS and a["kind"] != M.RLE else "k_pred<1>"
            add(kpred, a["footprint"])
            add("k_emit", out["footprint"])
        elif op == M.OP_BITMAP:
            a = inf(s.a)
            ue_total += 4 * a["n"]
            add("k_bitmap", a["footprint"])
        elif op == M.OP_INTERSECT:
            a, b = inf(s.a), inf(s.b)
            ue_total += 4 * (a["n"] + b["n"] + out["n"])
            probe, build = (a, b) if a["capacity_bytes"] <= b["capacity_bytes"] else (b, a)
            add("k_bitmap", build["footprint"]); add("k_pred<2>", probe["footprint"])
            add("k_emit_vals", probe["footprint"] + out["footprint"])  # decodes the probe list again
        elif op == M.OP_PROJECT:
            d, p = inf(s.a), inf(s.b)
            sec = sectors_touched(M, col(s.b))
            nsec = max((d["n"] + 15) // 16, 1)
            data = int(d["footprint"] * sec / nsec)
            ue_total += 8 * p["n"] + 64 * sec
            if s.out.kind == M.RLE:
                add("k_rle_count_proj", p["footprint"] + data); add("k_rle_emit_proj", out["footprint"])
            else:
                kname = "k_project_rle" if d["kind"] == M.RLE else "k_project"
                add(f"{kname}<{kout}>", p["footprint"] + out["footprint"] + data)
        elif op == M.OP_SUM:
            a = inf(s.a)
            ue_total += 4 * a["n"] + 8
            add("k_sum", a["footprint"])
        elif op == M.OP_GROUP_SUM:
            g, v = inf(s.a), inf(s.b)
            ue_total += 4 * (g["n"] + v["n"]) + 8 * s.param
            add("k_group_sum", g["footprint"] + v["footprint"] + 8 * s.param)
    return ue_total, alg


def plan_roofline(M, plan, alg, workload: str):
    """Dominant kernel of one profiled eager run; achieved = its algorithmic bytes per
    launch / its mean launch time; traffic from the workload's own counter summary."""
    M.sync()
    tune = plan.tune()
    plan.set_tune(1, tune[1], tune[2])  # one branch: concurrent kernels would inflate each launch's events
    M.prof_enable(True)
    M.prof_reset()
    plan.run()
    M.sync()
    recs = M.prof_records(0)
    M.prof_enable(False)
    M.prof_reset()
    plan.set_tune(*tune)
    tot, cnt = {}, {}
    for k, ms in recs:
        tot[k] = tot.get(k, 0.0) + ms
        cnt[k] = cnt.get(k, 0) + 1
    dom = max(tot, key=tot.get)
    avg_ms = tot[dom] / cnt[dom]
    bpl = alg.get(dom, 0) / cnt[dom]
    ach = bpl / (avg_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_for(dom, "traffic_" + workload))
    info = dict(kernel=dom, launches=cnt[dom], avg_ms=round(avg_ms, 4), bytes_per_launch=int(bpl),
                share_of_run=round(tot[dom] / sum(tot.values()), 3),
                per_kernel_ms={k: round(v, 3) for k, v in sorted(tot.items())})
    return roof, info


def time_graph(torch, plan, reps):
    plan.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.launch()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def time_eager(torch, plan, reps):
    plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


# ------------------------------------------------------------------------------ star query
# Format policies: base columns x intermediates.  "plain" is plain uncompressed execution
# (uncompressed base columns and intermediates); the others keep the base columns in static
# BP (the paper's base-data compression) and choose the intermediates' formats.
POLICIES = ("plain", "uncompr_inter", "static", "exhaustive", "learned", "learned_decode", "greedy")
FLUSH_BYTES = 2 << 30  # written between timed runs: evicts the 256 MB MALL and the L2s
# Launch shape of the full-size star plans (two branches, each operator's default grid and
# chunks per workgroup): re-capturing a full-size star plan many times in one process (the
# autotuner's trials, the greedy search) is kept out of the default run; --star-autotune
# and --greedy turn it on.
STAR_TUNE = (2, 0, 0)


def cold_times(torch, fn, reps, flush):
    """Per-run GPU times (s) of `reps` runs of fn, each bracketed by events on the current
    stream and preceded by a 2 GiB write that evicts the caches (not timed)."""
    ts = []
    for _ in range(reps):
        flush.fill_(len(ts) + 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    return ts


def copy_bandwidth(M, torch, log):
    """Achievable HBM bandwidth: a 4 GiB device-to-device copy (torch) and the library's
    decode of a 1e9-value uncompressed column (4 B read + 4 B written per value)."""
    n = 1 << 30
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    col = M.wrap(src)
    out = {}
    for name, fn in (("torch_copy", lambda: dst.copy_(src)), ("k_decode", lambda: col.decode(n=n))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        e1.synchronize()
        out[name] = round(8.0 * n * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
    del col, src, dst
    log(f"copy bandwidth (read + write GB/s): {out}")
    return out


def run_star(args, M, gen, torch, log):
    from paper_2004_09350_amd import datagen, queries, selector
    n = args.rows or 600_000_000
    star_tune = tuple(int(x) for x in args.star_tune.split(",")) if args.star_tune else STAR_TUNE
    wpath = args.weights or selector.WEIGHTS
    sel = selector.load(wpath)
    wsrc = os.path.relpath(wpath, ROOT)
    if args.calib_copy:
        calib_copy(M, log, M.encode(gen.uniform_bits(3, n, 32), M.fmt(M.UNCOMPR)), n)
    flush = torch.empty(FLUSH_BYTES // 4, dtype=torch.int32, device="cuda")
    copy_bw = copy_bandwidth(M, torch, log)
    settings = (("wide", datagen.STAR_WIDE), ("narrow", datagen.STAR_NARROW))
    cache = os.path.join(tempfile.gettempdir(), "ms_plan_tune_cache.txt")
    results, ue_sum, t_sum, t_all = [], 0, 0.0, []
    roof = dom = None
    for seed in [int(x) for x in args.seeds.split(",")]:
        t0 = time.time()
        cols, _ = selector.star_inputs(seed, n)
        plain_cols, _ = selector.star_inputs(seed, n, fact_fmt=M.fmt(M.UNCOMPR))
        for k in ("dimattr0", "dimattr1", "dimattr2", "dimattr3", "dimgroup3"):
            plain_cols[k] = M.morph(cols[k], M.fmt(M.UNCOMPR))
        torch.cuda.synchronize()
        base_fp = sum(c.info()["footprint"] for c in cols.values())
        plain_fp = sum(c.info()["footprint"] for c in plain_cols.values())
        log(f"seed {seed}: base columns {base_fp / 1e9:.2f} GB static BP, {plain_fp / 1e9:.2f} GB uncompressed, "
            f"{time.time() - t0:.1f}s")
        for sname, sel_s in settings:
            thr = datagen.star_thresholds(sel_s)
            log(f"  {sname}: probe run (statistics and footprints of every intermediate)")
            probe = queries.Q3(cols, thr, datagen.STAR_DIM_SIZES, n, extra=("stats", "footprints"))
            probe.plan.run()
            names = list(probe.names)
            fps = np.stack([probe.plan.read(probe.fp_step[k]) for k in names]).astype(np.uint64)
            feats = np.stack([probe.plan.read(probe.stats_step[k]) for k in names])
            ref = probe.results()
            probe.plan.close()
            kinds = {"uncompr_inter": np.zeros(len(names), int), "static": np.full(len(names), M.STATIC_BP),
                     "exhaustive": selector.exhaustive(fps), "learned": selector.pick(sel, feats),
                     "learned_decode": selector.pick(sel, feats, M.OBJ_DECODE)}
            kinds["plain"] = kinds["uncompr_inter"]
            log(f"  {sname}: formats picked")
            row = dict(seed=seed, setting=sname, rows_final=0, policies={})
            for pol in POLICIES:
                if pol == "greedy" and not args.greedy:
                    continue
                greedy_inputs, t_search = {}, 0.0
                log(f"  {sname}: policy {pol}")
                if pol == "greedy":
                    # the paper's greedy runtime search from plain uncompressed execution: base
                    # columns first, then the intermediates in plan order
                    ts0 = time.time()
                    gcols, gfmt, _, n_trials = queries.greedy_runtime_formats(
                        plain_cols, thr, datagen.STAR_DIM_SIZES, n, {k: M.fmt(M.UNCOMPR) for k in names}, reps=3)
                    t_search = time.time() - ts0
                    greedy_inputs = gcols
                    kinds["greedy"] = [gfmt[k].kind for k in names]
                    q = queries.Q3(gcols, thr, datagen.STAR_DIM_SIZES, n, formats=gfmt)
                else:
                    fm = {k: M.fmt(int(kk)) for k, kk in zip(names, kinds[pol])}
                    q = queries.Q3(plain_cols if pol == "plain" else cols, thr, datagen.STAR_DIM_SIZES, n,
                                   formats=fm)
                # eager runs and graph runs on separate plan objects (see the executor notes)
                qcols = [c for c in q.plan.inputs]
                mk = lambda: queries.Q3(dict(zip(queries.Q3_INPUTS, qcols)), thr, datagen.STAR_DIM_SIZES, n,
                                        formats={k: M.fmt(int(q.plan.steps[q.names[k]].out.kind)) for k in names})
                qe = mk()
                te = cold_times(torch, qe.plan.run, max(2, args.steps // 2), flush)
                qe.plan.close()
                del qe
                if args.star_autotune:
                    log(f"  {sname}: {pol} autotune")
                    tune, _ = q.plan.autotune(reps=2, cache=cache)
                else:
                    q.plan.set_tune(*star_tune)
                    tune = q.plan.tune()
                q.plan.launch()
                torch.cuda.synchronize()
                tg = cold_times(torch, q.plan.launch, args.steps, flush)
                arena = q.plan.arena_bytes()  # device bytes the graph holds (worst-case output capacities, scratch)
                o1, o2 = q.results()
                if not (np.array_equal(o1, ref[0]) and np.array_equal(o2, ref[1])):
                    raise SystemExit(f"star query answers differ under policy {pol}")
                fp = int(sum(int(fps[i][kinds[pol][i]]) for i in range(len(names))))
                ue, alg = plan_account(M, q.plan, q.plan.inputs)
                row["rows_final"] = int(q.plan.column(q.names["P"]).info()["n"])
                tgm = float(np.mean(tg))
                row["policies"][pol] = dict(
                    graph_ms_mean=round(tgm * 1e3, 3), graph_ms_median=round(float(np.median(tg)) * 1e3, 3),
                    eager_ms_mean=round(float(np.mean(te)) * 1e3, 3),
                    eager_ms_median=round(float(np.median(te)) * 1e3, 3), tune=list(tune),
                    intermediates_bytes=fp, arena_bytes=int(arena),
                    base_bytes=(plain_fp if pol == "plain" else base_fp if pol != "greedy" else
                                sum(c.info()["footprint"] for c in q.plan.inputs)),
                    ue_gbs=round(ue / tgm / 1e9, 1), hbm_frac=round(sum(alg.values()) / tgm / 1e9 / HBM_PEAK_GBS, 4))
                if pol == "learned":
                    ue_sum += ue
                    t_sum += tgm
                    t_all += tg
                    if roof is None:
                        qr = mk()
                        qr.plan.set_tune(*tune)
                        roof, dom = plan_roofline(M, qr.plan, alg, "star")
                        qr.plan.close()
                        del qr
                if pol == "greedy":
                    row["policies"][pol].update(
                        search_s=round(t_search, 1), trials=n_trials,
                        base_kinds={queries.Q3_INPUTS[j]: KIND_NAMES[int(c.info()["kind"])]
                                    for j, c in enumerate(q.plan.inputs)},
                        intermediate_kinds={k: KIND_NAMES[int(kk)] for k, kk in zip(names, kinds["greedy"])})
                q.plan.close()
                del q, greedy_inputs
            P = row["policies"]
            ex = P["exhaustive"]["intermediates_bytes"]
            row["regret_learned"] = round(P["learned"]["intermediates_bytes"] / ex - 1, 5)
            row["regret_learned_decode"] = round(P["learned_decode"]["intermediates_bytes"] / ex - 1, 5)
            row["learned_vs_plain_graph"] = round(P["plain"]["graph_ms_mean"] / P["learned"]["graph_ms_mean"], 3)
            row["learned_vs_plain_eager"] = round(P["plain"]["eager_ms_mean"] / P["learned"]["eager_ms_mean"], 3)
            if "greedy" in P:
                row["time_regret_vs_greedy"] = {k: round(P[k]["graph_ms_mean"] / P["greedy"]["graph_ms_mean"] - 1, 4)
                                                for k in P if k != "greedy"}
            row["footprint_learned_vs_plain"] = round(
                (P["learned"]["intermediates_bytes"] + base_fp) / (P["plain"]["intermediates_bytes"] + plain_fp), 4)
            results.append(row)
            log(json.dumps(row))
        del cols, plain_cols
    del flush
    res = base_line(args, "uncompressed-equivalent GB/s of the fused star query (learned formats, captured graph, "
                          "cold) + %HBM roofline; footprint vs exhaustive",
                    round(ue_sum / t_sum / 1e9, 2), "GB/s", t_sum / len(results),
                    f"star query: {n}-row fact table, 4 foreign keys over dimensions of "
                    f"{'/'.join(str(d) for d in datagen.STAR_DIM_SIZES)} rows, 2 measures, static-BP base columns, "
                    "semi-joins via dimension bitmaps, intersect of 4 position lists, group-sum into 250 groups; "
                    "wide and narrow filters", {"rows": n, "selector": wsrc})
    res.update(ms_per_step_median=round(float(np.median(t_all)) * 1e3, 3), roofline=roof, dominant_kernel=dom,
               runs=results, copy_bandwidth_gbs=copy_bw, source_sha=source_sha(),
               protocol="each timed run preceded by a 2 GiB device write (not timed); HIP events per run",
               launch_shape=("autotuned per plan" if args.star_autotune else
                             f"fixed {list(star_tune)} (branches, wg/CU, chunks/wg, batch)"))
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_star(min(n, args.cpu_rows or 40_000_000))
    return res


def _sectors(pos) -> int:
    return int(np.unique(np.asarray(pos, np.int64) >> 4).size)


def _star_ue(it, rows) -> int:
    """Uncompressed-equivalent bytes of one star query over `rows` fact rows (the rules of
    plan_account)."""
    from paper_2004_09350_amd import datagen
    D = datagen.STAR_DIM_SIZES
    ue = 0
    for d in range(4):
        s, pd = it[f"S{d}"].size, it[f"P{d}"].size
        ue += 4 * (D[d] + s) + 4 * s + 4 * (rows + pd)
    ue += 4 * (it["P0"].size + it["P1"].size + it["P01"].size)
    ue += 4 * (it["P01"].size + it["P2"].size + it["P012"].size)
    ue += 4 * (it["P012"].size + it["P3"].size + it["P"].size)
    P = it["P"]
    ue += 3 * (8 * P.size + 64 * _sectors(P)) + 8 * it["kp"].size + 64 * _sectors(it["kp"])
    ue += 2 * (4 * 2 * P.size + 8 * 250)
    return ue


def cpu_baseline_star(rows: int):
    """The oracle's star query (wide filters) on a bounded fact table: single thread, then
    over fact-row slices on all host cores (the plan is row-local up to its additive
    group-sums, and the C oracle releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle.queries as OQ
    from paper_2004_09350_amd import datagen
    cols = datagen.star_columns(1, rows)
    thr = datagen.star_thresholds(datagen.STAR_WIDE)
    t0 = time.perf_counter()
    r = OQ.q3(cols, thr, datagen.STAR_DIM_SIZES)
    dt1 = time.perf_counter() - t0
    ue = _star_ue(r["intermediates"], rows)
    nproc = os.cpu_count() or 1
    workers = max(1, min(16, nproc))  # the GPU machine's CPU share is 16 cores
    bounds = [(r0, min(rows, r0 + -(-rows // workers))) for r0 in range(0, rows, -(-rows // workers))]

    def part(b):
        sub = {k: (v[b[0]:b[1]] if not k.startswith("dim") else v) for k, v in cols.items()}
        return OQ.q3(sub, thr, datagen.STAR_DIM_SIZES)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(part, bounds))
    dtn = time.perf_counter() - t0
    with np.errstate(over="ignore"):
        tot = np.sum(np.stack([p["out1"] for p in parts]), axis=0, dtype=np.uint64)
    if not np.array_equal(tot, r["out1"]):
        raise SystemExit("sliced oracle star query differs from the whole one")
    return dict(value=round(ue / dtn / 1e9, 4), unit="GB/s", cores=workers, kind="oracle",
                single_thread_value=round(ue / dt1 / 1e9, 4), nproc=nproc,
                sample=f"the star query (wide filters) on a {rows}-row fact table: {dt1:.2f} s on one thread, "
                       f"{dtn:.2f} s over {len(bounds)} row slices on {workers} threads (nproc {nproc})",
                seconds=round(dt1 + dtn, 2))


# ------------------------------------------------------------------------------ batch
BATCH_OPS = ("select", "project", "intersect", "sum", "morph")


def batch_spec(T: int, seed: int = 4242):
    """T tasks: rows log-uniform in [1e4, 5e7]; operator, distribution, formats and
    selectivity uniform over the sweep's sets."""
    from paper_2004_09350_amd import datagen
    u = (datagen.stream(seed, 0, 8 * T).astype(np.float64) / 2.0 ** 64).reshape(T, 8)
    out = []
    for t in range(T):
        n_t = int(np.exp(np.log(1e4) + u[t, 0] * (np.log(5e7) - np.log(1e4))))
        kin, kout = int(u[t, 3] * 6), int(u[t, 4] * 6)
        op = BATCH_OPS[int(u[t, 1] * 5)]
        if op == "morph" and kout == kin:
            kout = (kin + 1) % 6
        out.append(dict(n=n_t, op=op, dist=DISTS[int(u[t, 2] * 6)], kin=kin, kout=kout,
                        si=int(u[t, 5] * 3), seed=50_000 + t))
    return out


def run_batch(args, M, gen, torch, log):
    T = args.tasks
    spec = batch_spec(T)
    inputs, steps = [], []
    t0 = time.time()
    for t, sp in enumerate(spec):
        n_t = sp["n"]
        raw = gen.sweep_column(sp["dist"], sp["seed"], n_t)
        if sp["op"] in ("select", "sum", "morph", "project"):
            inputs.append(M.encode(raw, M.fmt(sp["kin"])))
            j = len(inputs) - 1
        if sp["op"] == "select":
            probe = (lambda s, raw=raw: int(raw[min(n_t - 1, int(s * n_t))].item()) & 0xFFFFFFFF)
            c = thresholds(sp["dist"], probe if sp["dist"] == "SORTED" else None)[sp["si"]]
            steps.append(M.step(M.OP_SELECT, a=M.inp(j), cmp=M.LT, c0=c, out=M.fmt(sp["kout"])))
        elif sp["op"] == "sum":
            steps.append(M.step(M.OP_SUM, a=M.inp(j)))
        elif sp["op"] == "morph":
            steps.append(M.step(M.OP_MORPH, a=M.inp(j), out=M.fmt(sp["kout"])))
        elif sp["op"] == "project":
            u12 = M.encode(gen.uniform_bits(sp["seed"] + 100_000, n_t, 12), M.fmt(M.STATIC_BP))
            inputs.append(M.select(u12, M.LT, 410, 0, M.fmt(M.DELTA_DYN_BP)))
            steps.append(M.step(M.OP_PROJECT, a=M.inp(j), b=M.inp(j + 1), out=M.fmt(sp["kout"])))
        else:  # intersect of a 10 % and a 50 % position list over n_t rows
            a = M.encode(gen.uniform_bits(sp["seed"] + 200_000, n_t, 12), M.fmt(M.STATIC_BP))
            b = M.encode(gen.uniform_bits(sp["seed"] + 300_000, n_t, 12), M.fmt(M.STATIC_BP))
            inputs.append(M.select(a, M.LT, 410, 0, M.fmt(sp["kin"] if sp["kin"] != M.RLE else M.DELTA_DYN_BP)))
            inputs.append(M.select(b, M.LT, 2048, 0, M.fmt(M.DELTA_DYN_BP)))
            steps.append(M.step(M.OP_INTERSECT, a=M.inp(len(inputs) - 2), b=M.inp(len(inputs) - 1), param=n_t,
                                out=M.fmt(sp["kout"])))
        del raw
    M.sync()
    rows = sum(sp["n"] for sp in spec)
    log(f"batch: {T} tasks, {rows} rows, inputs ready in {time.time() - t0:.1f}s")
    reps = max(1, args.steps)
    # eager runs and graph runs on separate plan objects (see the executor notes)
    pe = M.Plan(steps, inputs)
    te1 = time_eager(torch, pe, reps)
    pe.set_tune(8, 8)
    te8 = time_eager(torch, pe, reps)
    pe.close()
    log(f"eager one stream {te1 * 1e3:.2f} ms, eager 8 streams {te8 * 1e3:.2f} ms")
    plan = M.Plan(steps, inputs)
    cache = os.path.join(tempfile.gettempdir(), "ms_plan_tune_cache.txt")
    best, best_ms = plan.autotune(reps=2, cache=cache)
    tg = time_graph(torch, plan, reps)
    arena = plan.arena_bytes()
    log(f"autotuned {best} ({best_ms:.2f} ms in tuning), graph {tg * 1e3:.2f} ms")
    # batched persistent launches (one launch per kernel kind and phase of each plan level)
    pb = M.Plan(steps, inputs)
    pb.set_tune(best[0], best[1], best[2], 1)
    tbe = time_eager(torch, pb, reps)
    pb.close()
    pb = M.Plan(steps, inputs)
    pb.set_tune(best[0], best[1], best[2], 1)
    tbg = time_graph(torch, pb, reps)
    pb.close()
    log(f"batched persistent launches: eager {tbe * 1e3:.2f} ms, graph {tbg * 1e3:.2f} ms")
    ue, alg = plan_account(M, plan, inputs)
    pr = M.Plan(steps, inputs)
    pr.set_tune(*best)
    roof, dom = plan_roofline(M, pr, alg, "batch")
    pr.close()
    res = base_line(args, "uncompressed-equivalent GB/s of 512 mixed column-operator tasks in one captured graph",
                    round(ue / tg / 1e9, 2), "GB/s", tg,
                    f"batch: {T} tasks, rows log-uniform in [1e4, 5e7] ({rows} rows), operator "
                    "(select/project/intersect/sum/morph), distribution and formats uniform over the sweep's sets",
                    {"tasks": T, "rows_total": rows})
    res.update(graph_ms=round(tg * 1e3, 3), eager_one_stream_ms=round(te1 * 1e3, 3),
               eager_8_streams_ms=round(te8 * 1e3, 3), speedup_vs_one_launch_sequence_per_task=round(te1 / tg, 3),
               tune={"branches": best[0], "wg_per_cu": best[1], "chunks_per_wg": best[2], "batch": best[3]},
               batched_graph_ms=round(tbg * 1e3, 3), batched_eager_ms=round(tbe * 1e3, 3),
               speedup_batched_graph_vs_one_launch_sequence_per_task=round(te1 / tbg, 3),
               arena_gb=round(arena / 1e9, 2),
               roofline=roof, dominant_kernel=dom, source_sha=source_sha())
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batch(spec, cap=args.cpu_rows or 1_000_000, max_tasks=len(spec))
    plan.close()
    return res


def cpu_baseline_batch(spec, cap: int, max_tasks: int):
    """The oracle on the first tasks of the batch, each cut to at most `cap` rows."""
    import oracle as O
    from paper_2004_09350_amd import datagen
    ue, dt = 0, 0.0
    for sp in spec[:max_tasks]:
        n_t = min(sp["n"], cap)
        v = datagen.sweep_column(sp["dist"], sp["seed"], n_t)
        enc = O.encode(v, sp["kin"])
        t0 = time.perf_counter()
        if sp["op"] == "select":
            c = thresholds(sp["dist"], (lambda s: int(v[min(n_t - 1, int(s * n_t))])))[sp["si"]]
            p = O.select(O.decode(enc), O.LT, c)
            O.encode(p, sp["kout"])
            ue += 4 * (n_t + p.size)
        elif sp["op"] == "sum":
            O.sum_(O.decode(enc))
            ue += 4 * n_t + 8
        elif sp["op"] == "morph":
            O.encode(O.decode(enc), sp["kout"])
            ue += 8 * n_t
        elif sp["op"] == "project":
            pos = O.select(datagen.uniform_bits(sp["seed"] + 100_000, n_t, 12), O.LT, 410)
            O.encode(O.project(O.decode(enc), pos), sp["kout"])
            ue += 8 * pos.size + 64 * _sectors(pos)
        else:
            pa = O.select(datagen.uniform_bits(sp["seed"] + 200_000, n_t, 12), O.LT, 410)
            pb = O.select(datagen.uniform_bits(sp["seed"] + 300_000, n_t, 12), O.LT, 2048)
            r = O.intersect(pa, pb)
            O.encode(r, sp["kout"])
            ue += 4 * (pa.size + pb.size + r.size)
        dt += time.perf_counter() - t0
    return dict(value=round(ue / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample=f"the first {max_tasks} batch tasks cut to at most {cap} rows each, single thread, "
                       f"{dt:.1f} s", seconds=round(dt, 2))


# ------------------------------------------------------------------------------ Q1
def run_q1(args, M, gen, torch, log):
    from paper_2004_09350_amd import queries
    n = args.rows or 1_000_000
    A = M.encode(gen.uniform_bits(1, n, 10), M.fmt(M.STATIC_BP, 10))
    B = M.encode(gen.uniform_bits(2, n, 20), M.fmt(M.STATIC_BP, 20))
    reps = max(10, args.steps)
    pe = queries.q1_plan(A, B, 103)  # eager runs and graph runs on separate plan objects
    te = time_eager(torch, pe, reps)
    pe.close()
    plan = queries.q1_plan(A, B, 103)
    tg = time_graph(torch, plan, reps)
    ue, alg = plan_account(M, plan, [A, B])
    pr = queries.q1_plan(A, B, 103)
    roof, dom = plan_roofline(M, pr, alg, "q1")
    pr.close()
    res = base_line(args, "uncompressed-equivalent GB/s of Q1 (select -> project -> sum, captured graph)",
                    round(ue / tg / 1e9, 2), "GB/s", tg,
                    f"Q1: {n} rows, A uniform 10-bit static BP, B uniform 20-bit static BP, positions of A < 103 "
                    "as delta+DynBP, project B (static BP auto), sum", {"rows": n})
    res.update(graph_ms=round(tg * 1e3, 4), eager_ms=round(te * 1e3, 4), sum=int(plan.read(2)[0]),
               roofline=roof, dominant_kernel=dom, source_sha=source_sha())
    if not args.no_cpu_baseline:
        import oracle.queries as OQ
        from paper_2004_09350_amd import datagen
        a, b = datagen.uniform_bits(1, n, 10), datagen.uniform_bits(2, n, 20)
        t0 = time.perf_counter()
        reps_c = 0
        while time.perf_counter() - t0 < 10.0:
            r = OQ.q1(a, b, 103)
            reps_c += 1
        dt = (time.perf_counter() - t0) / reps_c
        ue_c = 4 * (n + r["P"].size) + 8 * r["P"].size + 64 * _sectors(r["P"]) + 4 * r["Bp"].size + 8
        res["cpu_baseline"] = dict(value=round(ue_c / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                                   sample=f"Q1 on the same {n} rows, {reps_c} runs, single thread",
                                   seconds=round(dt, 3))
    plan.close()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (the row-wise sharding "
                                   "of the columns over several GPUs is designed, not built)"}))
        sys.exit(2)
    import torch

    from paper_2004_09350_amd import gen_gpu as gen
    from paper_2004_09350_amd import morphgpu as M

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    M.init()
    if args.workload == "sweep":
        res = run_sweep(args, M, gen, torch, log)
    elif args.workload == "star":
        res = run_star(args, M, gen, torch, log)
        if not args.no_sweep:
            sargs = argparse.Namespace(**vars(args))
            sargs.steps, sargs.warmup, sargs.rows, sargs.no_cpu_baseline = args.sweep_steps, 1, None, True
            sargs.calib_copy = False
            sw = run_sweep(sargs, M, gen, torch, log)
            res["sweep"] = {k: sw[k] for k in ("metric", "value", "unit", "ms_per_step", "hbm_frac_step", "roofline",
                                               "dominant_kernel", "config")}
    elif args.workload == "batch":
        res = run_batch(args, M, gen, torch, log)
    else:
        res = run_q1(args, M, gen, torch, log)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
