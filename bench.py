"""Benchmark: the operator/format sweep over 1e8-row uint32 columns on one MI355X.

One step = one pass of the whole sweep (every row of the hot path that applies to
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
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DISTS = ("U4", "U12", "U24", "U32", "SORTED", "RUNS")
SELECTIVITIES = (0.01, 0.10, 0.50)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=100_000_000)
    ap.add_argument("--cpu-rows", type=int, default=600_000)
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
                       "k_rle_count": pinfo["footprint"] + data, "k_rle_emit": oi["footprint"]}
            elif name == "sum":
                ue = 4 * n + 8
                alg = {"k_sum": fin}
            elif name == "morph":
                ue = 8 * n
                alg = {"k_morph": fin + oi["footprint"], "k_rle_count": fin, "k_rle_emit": oi["footprint"]}
            else:
                ue = 4 * (pa["n"] + pb["n"] + oi["n"])
                probe, build = (pa, pb) if pa["n"] <= pb["n"] else (pb, pa)
                alg = {"k_bitmap": build["footprint"], "k_pred": probe["footprint"], "k_emit": oi["footprint"]}
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        sys.exit(2)
    import torch

    from paper_2004_09350_amd import gen_gpu as gen
    from paper_2004_09350_amd import morphgpu as M

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    M.init()
    sw = Sweep(M, gen, args.rows, args.quick, log)
    if args.calib_copy:
        dst = sw.cols[("U32", M.UNCOMPR)].decode()
        M.sync()
        log(f"calibration copy: k_decode of {args.rows} rows ({4 * args.rows} B read, {4 * args.rows} B written)")
        del dst
    sw.account()
    log("accounting pass done")
    if args.dump:
        KN = M.KIND_NAMES
        rows = []
        for a in sw.acct:
            name, key, c, kout = a["op"]
            rows.append(dict(op=name, dist=key[0] if key else None, kin=KN[key[1]] if key else None, c=c,
                             kout=KN[kout] if kout is not None else None, recs=a["recs"], alg=a["alg"],
                             ue=a["ue"], out_fp=a["out_fp"]))
        json.dump(rows, open(args.dump, "w"))
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
    res = {
        "metric": "uncompressed-equivalent GB/s of the fused operator sweep (plus %HBM roofline on compressed bytes)",
        "value": round(ue / dt / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "operator/format sweep: 6 distributions x 6 formats of 1e8-row uint32 columns; "
                               "select 1/10/50 % -> 6 formats, project at a 10 % position list -> 6 formats, "
                               "sum, intersect -> 6 formats, morph between all 30 format pairs",
                   "rows": args.rows, "operators_per_step": len(sw.ops)},
        "hbm_frac_step": round(alg / dt / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "dominant_kernel": dominfo,
        "source_sha": source_sha(),
    }
    traffic_file = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(traffic_file):
        try:
            t = json.load(open(traffic_file))
            if t.get("source_sha") == res["source_sha"] and dom in t.get("kernels", {}):
                res["roofline"]["traffic"] = t["kernels"][dom]["bytes_per_launch"]
        except Exception:
            pass
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.cpu_rows)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
