"""Pin of the oracle's gradient with the velocity table (Sections 3.2 and 4.2: speeds at
whole degrees, linearly interpolated).  The table's interpolants are piecewise linear in the
angle, so the derivative of every estimate and straight ray uses the slope of the whole-degree
interval it lies in; the gradient of a receiver functional must then match central
differences of the oracle's own table forward in every node's orientation (steps far smaller
than a degree rarely cross an interval end)."""
import numpy as np

import synthmedia as sm


def _cos(a, b):
    return float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_table_gradient_matches_central_differences(orc):
    m = sm.random_medium(14, 12, 0.2e-3, seed=9, n_mats=3)
    tm = orc.as_table(m.mats)
    sources = [(7, 0), (2, 5)]
    receivers = [(0, 11), (13, 11), (7, 11), (13, 4)]
    w = np.random.default_rng(3).normal(size=(len(sources), len(receivers)))

    def functional(orient):
        tot = 0.0
        for s, src in enumerate(sources):
            T = orc.solve_fmm(m.h, tm, m.mat_id, orient, src, 2)
            tot += sum(w[s, r] * T[rj, ri] for r, (ri, rj) in enumerate(receivers))
        return tot

    G = np.zeros((m.nz, m.nx))
    for s, src in enumerate(sources):
        g = np.zeros((m.nz, m.nx))
        for r, (ri, rj) in enumerate(receivers):
            g[rj, ri] += w[s, r]
        G += orc.adjoint(m.h, tm, m.mat_id, m.orient, src, g)[1]
    step = 1e-7
    fd = np.zeros_like(G)
    base = m.orient.astype(np.float64)
    for j in range(m.nz):
        for i in range(m.nx):
            op = base.copy()
            op[j, i] += step
            lp = functional(op)
            op[j, i] -= 2 * step
            lm = functional(op)
            fd[j, i] = (lp - lm) / (2 * step)
    rel = np.abs(G - fd) / np.abs(fd).max()
    print("table gradient vs central differences (%d nodes): cos %.9f, median rel %.3g, max rel %.3g"
          % (fd.size, _cos(G, fd), np.median(rel), rel.max()))
    assert _cos(G, fd) >= 0.99999
    assert rel.max() <= 1e-4


def test_table_stiffness_gradient_refused(orc):
    import pytest
    m = sm.random_medium(8, 8, 0.2e-3, seed=1, n_mats=2)
    with pytest.raises(ValueError):
        orc.adjoint(m.h, orc.as_table(m.mats), m.mat_id, m.orient, (4, 0), np.ones((8, 8)), with_A=True)
