"""Table 3's set-up (Section 4.5) on the oracle: the 21 x 21 cubic-steel grid at 0 degrees,
source at the centre, the subgrid study's nested source grids, and the mean absolute
relative percentage error at the original nodes against straight-ray times.

`group` chooses the group speed of the straight rays, both those that start the march
near the source and those that give the true times: "exact" (the oracle's own reading), or
"paper" (Section 3.2's run-time inversion, which takes the phase angle whose polarisation
points along the group direction).  `table` switches the stencil and straight-ray speeds
to the velocity table (exact speeds at whole degrees, linearly interpolated); the true
times then keep the group rule of the run-time row.  `variant` selects alternative
readings of the update (oracle.VAR_* bits) for the thread that runs the case.
"""
import functools
import json
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import synthmedia as sm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table3_subgrid.json")))
SUBGRIDS = GOLD["subgrid_size"]
PRINTED = dict(zip(SUBGRIDS, GOLD["ali_fmm_christoffel_percent"]))
PRINTED_TABLE = dict(zip(SUBGRIDS, GOLD["ali_fmm_table_percent"]))


def levels(s):
    if s == 1:
        return [tuple(x) for x in GOLD["levels_subgrid_1"]], 0.5
    return [(d, r * s) for d, r in GOLD["levels_subgrid_s_original_cells"]], 0.5 * s


def error(orc, s, group="paper", table=False, variant=0):
    n, h, mat = GOLD["grid"], 1e-3, sm.CUBIC_STEEL
    c = n // 2
    mats = orc.with_paper_group([mat]) if group == "paper" and not table else [mat]
    if table:
        mats = orc.as_table(mats)
    truth_speed = orc.qp_group_speed_paper if group == "paper" else orc.qp_group_speed
    mid, ori = orc.refine_medium(np.zeros((n, n), np.uint8), np.zeros((n, n)), s)
    lv, half = levels(s)
    orc.set_reading_variant(variant)
    try:
        T = orc.solve_refined(h / s, mats, mid, ori, (c * s, c * s), lv, half)[::s, ::s]
    finally:
        orc.set_reading_variant(0)
    e = []
    for j in range(n):
        for i in range(n):
            if i == c and j == c:
                continue
            phi = math.atan2(j - c, i - c) - 0.5 * math.pi
            t = math.hypot(i - c, j - c) * h / truth_speed(mat, phi)
            e.append(abs(T[j, i] - t) / t)
    return 100.0 * float(np.mean(e))


@functools.lru_cache(maxsize=None)
def _row(orc, group, table, variant):
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        vals = list(ex.map(lambda s: error(orc, s, group, table, variant), SUBGRIDS))
    return tuple(vals)


def row(orc, group="paper", table=False, variant=0):
    """{subgrid size: error} over every printed subgrid size (cases on a thread pool,
    each row computed once per session)."""
    return dict(zip(SUBGRIDS, _row(orc, group, table, variant)))

