"""Query plans on the GPU (section 3.3: operator-at-a-time plans whose intermediates are
materialised in the format chosen for each of them; final results uncompressed).

* Q1, the simple query of section 5.1 with a range predicate: positions of A < c,
  project B at them, sum.
* Q3, a star-style plan: per dimension select -> bitmap -> semi-join of the fact
  table's foreign key, intersect the four position lists, project the measures and the
  group key, group-sum both measures.

Format policies for the intermediates (section 5.2): all uncompressed, all static BP
(the "naive" choice), exhaustive (the least exact footprint per intermediate: footprints
add up, so the per-column minimum is the plan optimum; ties to the lower format number)
and learned (the selector network's pick from the 32 statistics).
"""
from __future__ import annotations

import numpy as np

from . import morphgpu as M

POSITION_DEFAULT = M.DELTA_DYN_BP


def q1_plan(A, B, threshold: int = 103, fmt_p=None, fmt_b=None) -> M.Plan:
    fmt_p = fmt_p if fmt_p is not None else M.fmt(M.DELTA_DYN_BP)
    fmt_b = fmt_b if fmt_b is not None else M.fmt(M.STATIC_BP)
    steps = [
        M.step(M.OP_SELECT, a=M.inp(0), cmp=M.LT, c0=threshold, out=fmt_p),   # 0: P
        M.step(M.OP_PROJECT, a=M.inp(1), b=0, out=fmt_b),                     # 1: B'
        M.step(M.OP_SUM, a=1),                                                # 2: sum
    ]
    return M.Plan(steps, [A, B])


Q1_INTERMEDIATES = {"P": 0, "Bp": 1}

# Q3 inputs, in order
Q3_INPUTS = ("fk0", "fk1", "fk2", "fk3", "m1", "m2", "dimattr0", "dimattr1", "dimattr2", "dimattr3", "dimgroup3")


class Q3:
    """The star plan over the columns named in Q3_INPUTS.  `names` maps every column
    intermediate to its step; `out1`/`out2` are the group-sum steps."""

    def __init__(self, cols: dict, thresholds, dim_sizes, n_fact: int, groups: int = 250, formats: dict | None = None,
                 extra=None):
        I = {name: M.inp(j) for j, name in enumerate(Q3_INPUTS)}
        steps, names = [], {}
        pos = M.fmt(POSITION_DEFAULT)
        val = M.fmt(M.STATIC_BP)

        def add(st, name=None):
            steps.append(st)
            if name:
                names[name] = len(steps) - 1
            return len(steps) - 1

        pd = []
        for d in range(4):
            s = add(M.step(M.OP_SELECT, a=I[f"dimattr{d}"], cmp=M.LT, c0=thresholds[d], out=pos), f"S{d}")
            bm = add(M.step(M.OP_BITMAP, a=s, param=dim_sizes[d]))
            pd.append(add(M.step(M.OP_SEMIJOIN, a=I[f"fk{d}"], b=bm, param=dim_sizes[d], out=pos), f"P{d}"))
        p = add(M.step(M.OP_INTERSECT, a=pd[0], b=pd[1], param=n_fact, out=pos), "P01")
        p = add(M.step(M.OP_INTERSECT, a=p, b=pd[2], param=n_fact, out=pos), "P012")
        p = add(M.step(M.OP_INTERSECT, a=p, b=pd[3], param=n_fact, out=pos), "P")
        m1p = add(M.step(M.OP_PROJECT, a=I["m1"], b=p, out=val), "m1p")
        m2p = add(M.step(M.OP_PROJECT, a=I["m2"], b=p, out=val), "m2p")
        kp = add(M.step(M.OP_PROJECT, a=I["fk3"], b=p, out=val), "kp")
        gp = add(M.step(M.OP_PROJECT, a=I["dimgroup3"], b=kp, out=val), "gp")
        self.out1 = add(M.step(M.OP_GROUP_SUM, a=gp, b=m1p, param=groups))
        self.out2 = add(M.step(M.OP_GROUP_SUM, a=gp, b=m2p, param=groups))
        self.names = names
        # optional per-intermediate statistics / footprints (selector training and labels)
        self.stats_step, self.fp_step = {}, {}
        if extra:
            for name, i in list(names.items()):
                if "stats" in extra:
                    self.stats_step[name] = add(M.step(M.OP_STATS, a=i))
                if "footprints" in extra:
                    self.fp_step[name] = add(M.step(M.OP_FOOTPRINTS, a=i))
        if formats:
            for name, f in formats.items():
                steps[names[name]].out = f
        self.groups = groups
        self.plan = M.Plan(steps, [cols[k] for k in Q3_INPUTS])

    def set_formats(self, formats: dict):
        for name, f in formats.items():
            self.plan.set_format(self.names[name], f)

    def results(self):
        return self.plan.read(self.out1), self.plan.read(self.out2)

    def footprint(self) -> int:
        """Bytes of all intermediates as stored in the last run."""
        return sum(self.plan.column(i).info()["footprint"] for i in self.names.values())


def uniform_formats(names, kind) -> dict:
    return {n: M.fmt(kind) for n in names}


def exhaustive_formats(plan: M.Plan, names: dict) -> tuple[dict, dict]:
    """Least-footprint format of every intermediate of the plan's last run (the library's
    exhaustive selection: exact footprints from one pass each, ties to the lower format);
    also returns the footprint vectors."""
    chosen, fps = {}, {}
    for n, i in names.items():
        k, b = M.select_exhaustive(plan.column(i))
        chosen[n] = M.fmt(int(k.cpu()[0]))
        fps[n] = M.u64(b)
    return chosen, fps


def learned_formats(plan: M.Plan, names: dict, params) -> dict:
    """The selector network's pick for every intermediate of the plan's last run."""
    import torch
    feats = torch.stack([M.stats(plan.column(i)) for i in names.values()])
    _, pick = M.mlp_forward(params, feats.contiguous(), want_y=False)
    picks = pick.cpu().numpy()
    return {n: M.fmt(int(k)) for n, k in zip(names, picks)}


def _replay_ms(plan: M.Plan, reps: int) -> float:
    """Mean time (ms) of `reps` graph replays after a capture and a warm replay."""
    import torch
    plan.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.launch()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def greedy_runtime_formats(cols: dict, thresholds, dim_sizes, n_fact: int, formats: dict, reps: int = 3,
                           tune=(2, 0, 0), search_inputs: bool = True, log=None):
    """Section 5.2's greedy runtime search: starting at the base data, one column at a time
    (the star plan's input columns, then its intermediates in plan order), every format is
    tried, the query is timed (captured graph, mean of `reps` replays) and the column keeps
    its fastest format for the rest of the search.  Returns (input columns, intermediate
    formats, final mean ms, number of trials); input columns in a new format are morphed
    copies (the given columns are not changed)."""
    cur_cols = dict(cols)
    cur_fmt = dict(formats)

    def trial(cs, fm):
        q = Q3(cs, thresholds, dim_sizes, n_fact, formats=fm)
        q.plan.set_tune(*tune)
        t = _replay_ms(q.plan, reps)
        q.plan.close()
        return t

    best_t = trial(cur_cols, cur_fmt)
    trials = 1
    if search_inputs:
        for name in Q3_INPUTS:
            given = cur_cols[name]
            k0 = given.info()["kind"]
            for k in M.KINDS:
                if k == k0:
                    continue
                cand = M.morph(given, M.fmt(k))
                t = trial(dict(cur_cols, **{name: cand}), cur_fmt)
                trials += 1
                if t < best_t:
                    best_t, cur_cols[name] = t, cand
                del cand
            if log:
                log(f"greedy: {name} -> {M.KIND_NAMES[cur_cols[name].info()['kind']]} ({best_t:.3f} ms)")
    for name in formats:
        k0 = cur_fmt[name].kind
        for k in M.KINDS:
            if k == k0:
                continue
            fm = dict(cur_fmt, **{name: M.fmt(k)})
            t = trial(cur_cols, fm)
            trials += 1
            if t < best_t:
                best_t, cur_fmt = t, fm
        if log:
            log(f"greedy: {name} -> {M.KIND_NAMES[cur_fmt[name].kind]} ({best_t:.3f} ms)")
    return cur_cols, cur_fmt, best_t, trials
