"""Query plans composed from the oracle's plain operators (TEST INFRASTRUCTURE ONLY).

Operator-at-a-time execution with every intermediate fully materialised
(paper section 3 and 3.3): each operator runs to completion before the next.
Compression is lossless, so the answer of a plan does not depend on the
formats; the formats only change footprints, which ``plan_footprints`` reports.
"""
from __future__ import annotations

import numpy as np

from . import (BETWEEN, EQ, GE, GT, LE, LT, NE, bitmap_from_positions, footprints, group_sum, intersect,
               project, select, semijoin, sum_)


def q1(a, b, threshold=103):
    """SUM(B) WHERE A < threshold: select -> project -> sum (the paper's simple query shape,
    section 5.1, with a range predicate)."""
    p = select(a, LT, threshold)
    bp = project(b, p)
    return dict(P=p, Bp=bp, sum=sum_(bp))


def q3(cols: dict, thresholds, dim_sizes, groups=250):
    """Star-style plan: per dimension select -> bitmap -> semi-join, intersect the four
    position lists, project the measures and the group key, group-sum both measures."""
    inter = {}
    plist = []
    for d in range(4):
        s = select(cols[f"dimattr{d}"], LT, thresholds[d])
        bm = bitmap_from_positions(s, dim_sizes[d])
        pd = semijoin(cols[f"fk{d}"], bm, dim_sizes[d])
        inter[f"S{d}"] = s
        inter[f"P{d}"] = pd
        plist.append(pd)
    p = intersect(plist[0], plist[1])
    inter["P01"] = p
    p = intersect(p, plist[2])
    inter["P012"] = p
    p = intersect(p, plist[3])
    inter["P"] = p
    m1p = project(cols["m1"], p)
    m2p = project(cols["m2"], p)
    kp = project(cols["fk3"], p)
    gp = project(cols["dimgroup3"], kp)
    inter.update(m1p=m1p, m2p=m2p, kp=kp, gp=gp)
    out1 = group_sum(gp, m1p, groups)
    out2 = group_sum(gp, m2p, groups)
    return dict(intermediates=inter, out1=out1, out2=out2)


def plan_footprints(intermediates: dict) -> dict:
    """Exact footprint of every intermediate in each of the six formats."""
    return {k: footprints(v) for k, v in intermediates.items()}


def exhaustive_choice(intermediates: dict) -> dict:
    """Per intermediate, the format of least footprint (ties to the lowest format number).
    Footprints add up over columns, so the per-column minimum is the plan optimum
    (section 5.2)."""
    return {k: int(np.argmin(f)) for k, f in plan_footprints(intermediates).items()}
