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
    """Least-footprint format of every intermediate of the plan's last run (exact
    footprints from one pass each); also returns the footprint vectors."""
    fps = {n: M.u64(M.footprints(plan.column(i))) for n, i in names.items()}
    return {n: M.fmt(int(np.argmin(f))) for n, f in fps.items()}, fps


def learned_formats(plan: M.Plan, names: dict, params) -> dict:
    """The selector network's pick for every intermediate of the plan's last run."""
    import torch
    feats = torch.stack([M.stats(plan.column(i)) for i in names.values()])
    _, pick = M.mlp_forward(params, feats.contiguous(), want_y=False)
    picks = pick.cpu().numpy()
    return {n: M.fmt(int(k)) for n, k in zip(names, picks)}
