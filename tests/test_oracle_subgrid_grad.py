"""Pin of the misfit gradient on the s-fold refined medium (Section 4.5's subgrid size): the
oracle composition (fine-grid adjoint carried back through the nearest-node refinement) must
match central differences of the oracle's own s-fold forward in every node's orientation.
A step that changed a stencil choice on the fine grid would leave that node without a
derivative; on this medium none does, and every node is held to the bar."""
import numpy as np

import synthmedia as sm
from subgrid_grad import misfit, misfit_gradient


def _cos(a, b):
    return float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_subgrid_gradient_matches_central_differences(orc):
    m = sm.random_medium(9, 8, 0.3e-3, seed=4, n_mats=2)
    s = 3
    sources = [(4, 0), (1, 2)]
    receivers = [(0, 7), (8, 7), (4, 7), (8, 3)]
    _, t0 = misfit(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers, np.zeros((2, 4)), s)
    obs = t0 * (1.0 + 0.02 * np.random.default_rng(0).normal(size=t0.shape))
    L, trec, G = misfit_gradient(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers, obs, s)
    assert np.allclose(trec, t0, rtol=1e-15, atol=0)
    step = 1e-6
    fd = np.zeros_like(G)
    for j in range(m.nz):
        for i in range(m.nx):
            op = m.orient.astype(np.float64).copy()
            op[j, i] += step
            lp, _ = misfit(orc, m.h, m.mats, m.mat_id, op, sources, receivers, obs, s)
            op[j, i] -= 2 * step
            lm, _ = misfit(orc, m.h, m.mats, m.mat_id, op, sources, receivers, obs, s)
            fd[j, i] = (lp - lm) / (2 * step)
    scale = np.abs(fd).max()
    rel = np.abs(G - fd) / scale
    print("subgrid 3 gradient vs central differences (%d nodes): cos %.8f, median rel %.3g, max rel %.3g"
          % (fd.size, _cos(G, fd), np.median(rel), rel.max()))
    # measured: cosine 1 - 1e-15, largest error 3.2e-9 of the largest entry
    assert _cos(G, fd) >= 0.99999
    assert rel.max() <= 1e-5


def test_subgrid_one_is_the_plain_gradient(orc):
    m = sm.random_medium(12, 10, 0.2e-3, seed=2, n_mats=2)
    sources = [(6, 0)]
    receivers = [(0, 9), (11, 9)]
    obs = np.zeros((1, 2))
    L, trec, G = misfit_gradient(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers, obs, 1)
    T = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient, sources[0], 2)
    g = np.zeros((m.nz, m.nx))
    for r, (ri, rj) in enumerate(receivers):
        g[rj, ri] += T[rj, ri]
    ref = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, sources[0], g)[1]
    assert np.array_equal(G, ref)
