"""Pins for the oracle's nested fine grids around the source (Section 4.4) and the
whole-grid refinement of the subgrid study (Section 4.5, Table 3).

  - without fine grids the driver reduces to the straight-ray box (exactly);
  - a fine level that covers the whole domain equals solving the s-times refined medium
    directly and keeping every s-th node (exactly); this checks the level extents, the
    nearest-node material of the fine grids (computed by a second, numpy route) and the
    hand-over of known nodes between levels;
  - levels that run to the domain's edge hand every node over unchanged;
  - Table 3 with the oracle's own reading (exact group speed for the straight rays): with
    the paper's levels the error on the 21 x 21 cubic-steel grid at 0 degrees is within
    10 % of the printed 1.083 %; for subgrid sizes 3-7 it decreases and stays below the
    printed values; the straight-ray box alone is about four times worse.
  - Table 3 as printed: the printed errors follow Section 3.2's run-time group speed (the
    phase angle whose polarisation points along the group direction, up to 0.43 % faster
    than the exact group speed for this steel) in the straight rays near the source and
    in the true times.  Under that reading every printed value of the run-time row is
    reproduced to a factor 1.02-1.10 (s >= 3; 1.05-1.16 at s = 1) that varies by at most
    0.05 over s = 3..21; under the exact group speed the same ratio falls from 0.95 to
    0.45, which no change of the field can produce.  The pin rejects a close node keeping
    the smaller of its old and new estimates (errors a third of the printed ones) and a
    strict priority of the side-1 squares over the side-sqrt(2) squares (ratios 0.87-0.98,
    varying by 0.11); the first-member triangle score read literally and dropping the
    causality filter leave this symmetric case unchanged (not decided by Table 3).
"""
import json
import math
import os

import numpy as np
import pytest

import synthmedia as sm
import table3

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_table3_subgrid.json")


def test_no_levels_is_the_straight_ray_box(orc):
    m = sm.random_medium(23, 19, 0.2e-3, seed=5, n_mats=3)
    src = m.sources[0]
    for R, half in ((0, 0.5), (2, 2.5), (3, 3.5)):
        a = orc.solve_refined(m.h, m.mats, m.mat_id, m.orient, src, levels=(), vor_half=half)
        b = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient, src, R)
        assert np.array_equal(a, b), R


@pytest.mark.parametrize("s,seed", [(3, 2), (5, 6)])
def test_level_covering_the_domain_is_the_refined_grid(orc, s, seed):
    m = sm.random_medium(13, 11, 0.3e-3, seed=seed, n_mats=3, smooth=False)
    src = m.sources[0]
    a = orc.solve_refined(m.h, m.mats, m.mat_id, m.orient, src, levels=((s, 50),), vor_half=0.5)
    mid, ori = orc.refine_medium(m.mat_id, m.orient, s)
    b = orc.solve_refined(m.h / s, m.mats, mid, ori, (src[0] * s, src[1] * s), levels=(), vor_half=0.5 * s)
    assert np.array_equal(a, b[::s, ::s])
    # a finer level in front of it, also covering everything, changes nothing
    c = orc.solve_refined(m.h, m.mats, m.mat_id, m.orient, src, levels=((3 * s, 50), (s, 50)), vor_half=0.5)
    d = orc.solve_refined(m.h / s, m.mats, mid, ori, (src[0] * s, src[1] * s), levels=((3, 50),),
                          vor_half=0.5 * s)
    assert np.array_equal(c, d[::s, ::s])


def test_refine_medium_nearest_node(orc):
    mid = np.arange(12, dtype=np.uint8).reshape(3, 4)
    ori = np.arange(12, dtype=np.float64).reshape(3, 4) * 0.1
    rm, ro = orc.refine_medium(mid, ori, 3)
    assert rm.shape == (7, 10)
    # node k of the fine grid sits at k / 3 of the original: nearest original index
    for j in range(7):
        for i in range(10):
            assert rm[j, i] == mid[int(math.floor(j / 3 + 0.5)), int(math.floor(i / 3 + 0.5))]
            assert ro[j, i] == ori[int(math.floor(j / 3 + 0.5)), int(math.floor(i / 3 + 0.5))]


def _table3_error(orc, s, levels, half):
    gold = json.load(open(GOLD))
    n = gold["grid"]
    mat, h = sm.CUBIC_STEEL, 1e-3
    mid, ori = orc.refine_medium(np.zeros((n, n), np.uint8), np.zeros((n, n)), s)
    c = n // 2
    if levels is None:
        T = orc.solve_fmm(h / s, [mat], mid, ori, (c * s, c * s), 2)
    else:
        T = orc.solve_refined(h / s, [mat], mid, ori, (c * s, c * s), levels, half)
    T = T[::s, ::s]
    err = []
    for j in range(n):
        for i in range(n):
            if i == c and j == c:
                continue
            phi = math.atan2(j - c, i - c) - 0.5 * math.pi
            t = math.hypot(i - c, j - c) * h / orc.qp_group_speed(mat, phi)
            err.append(abs(T[j, i] - t) / t)
    return 100.0 * float(np.mean(err))


def test_table3_subgrid_errors(orc):
    gold = json.load(open(GOLD))
    printed = dict(zip(gold["subgrid_size"], gold["ali_fmm_christoffel_percent"]))
    e1 = _table3_error(orc, 1, [tuple(x) for x in gold["levels_subgrid_1"]], 0.5)
    print("subgrid 1: %.3f %% (printed %.3f)" % (e1, printed[1]))
    assert abs(e1 - printed[1]) <= 0.1 * printed[1]
    box = _table3_error(orc, 1, None, 0.5)
    assert box > 3.0 * e1
    prev = e1
    for s in (3, 5, 7):
        lv = [(d, r * s) for d, r in gold["levels_subgrid_s_original_cells"]]
        e = _table3_error(orc, s, lv, 0.5 * s)
        print("subgrid %d: %.3f %% (printed %.3f)" % (s, e, printed[s]))
        assert e < prev and e < printed[s] and e > 0.6 * printed[s]
        prev = e


def test_refinement_reduces_error_in_ti_steel(orc):
    mat, h, n = sm.TI_STEEL, 1e-3, 25
    c = n // 2
    for th in (0.3, 1.1):
        mid, ori = np.zeros((n, n), np.uint8), np.full((n, n), th)
        Tb = orc.solve_fmm(h, [mat], mid, ori, (c, c), 2)
        Tr = orc.solve_refined(h, [mat], mid, ori, (c, c))
        eb, er = [], []
        for j in range(n):
            for i in range(n):
                if max(abs(i - c), abs(j - c)) <= 2:
                    continue
                phi = math.atan2(j - c, i - c) - (th + 0.5 * math.pi)
                t = math.hypot(i - c, j - c) * h / orc.qp_group_speed(mat, phi)
                eb.append(abs(Tb[j, i] - t) / t)
                er.append(abs(Tr[j, i] - t) / t)
        assert np.mean(er) < 0.5 * np.mean(eb), (th, np.mean(er), np.mean(eb))


def _ratios(vals):
    return {s: vals[s] / table3.PRINTED[s] for s in table3.SUBGRIDS}


def test_table3_printed_row_follows_the_papers_group_speed(orc):
    r = _ratios(table3.row(orc, group="paper"))
    print("paper group speed, oracle / printed:", " ".join("%d:%.3f" % kv for kv in r.items()))
    assert 1.05 <= r[1] <= 1.16
    later = [r[s] for s in table3.SUBGRIDS if s >= 3]
    assert all(1.02 <= x <= 1.10 for x in later)
    assert max(later) - min(later) <= 0.05
    # the exact group speed everywhere: the ratio to the printed values keeps falling
    rx = _ratios(table3.row(orc, group="exact"))
    print("exact group speed, oracle / printed:", " ".join("%d:%.3f" % kv for kv in rx.items()))
    assert rx[3] > 0.85 and rx[21] < 0.5 and all(rx[a] > rx[b] for a, b in zip(table3.SUBGRIDS[1:], table3.SUBGRIDS[2:]))


@pytest.mark.parametrize("variant,decided", [("VAR_MIN_UPDATE", True), ("VAR_UNIT_SQUARES_FIRST", True),
                                             ("VAR_TRIANGLE_LITERAL", False), ("VAR_NO_CAUSALITY", False)])
def test_table3_alternative_readings(orc, variant, decided):
    base = table3.row(orc, group="paper")
    alt = table3.row(orc, group="paper", variant=getattr(orc, variant))
    r = _ratios(alt)
    later = [r[s] for s in table3.SUBGRIDS if s >= 3]
    print(variant, " ".join("%d:%.3f" % kv for kv in r.items()))
    ok = all(1.02 <= x <= 1.10 for x in later) and max(later) - min(later) <= 0.05
    if decided:
        assert not ok
    else:
        # the reading changes nothing in this symmetric set-up
        assert all(alt[s] == base[s] for s in table3.SUBGRIDS)
