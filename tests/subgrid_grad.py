"""Misfit and its orientation gradient on the medium refined s-fold (Section 4.5's subgrid
size with the straight-ray source box), composed from the oracle for the tests: the medium
is refined by nearest node, every source's field is solved and differentiated on the fine
grid with the sources and receivers on the nodes (s i, s j), and the fine gradient is
carried back to the nodes through the transpose of the nearest-node gather (each node's
orientation reaches the fine nodes nearest to it)."""
import numpy as np


def _maps(nz, nx, s):
    """Node each fine row / column takes its medium from (as oracle.refine_medium)."""
    jz = (np.arange((nz - 1) * s + 1) + s // 2) // s
    ix = (np.arange((nx - 1) * s + 1) + s // 2) // s
    return jz, ix


def misfit(orc, h, mats, mat_id, orient, sources, receivers, obs, s, R=2):
    """L = 1/2 sum over (source, receiver) of (T - obs)^2 on the s-fold grid, and the
    modelled times [n_src, n_rec]."""
    mid, ori = orc.refine_medium(mat_id, orient, s)
    L, trec = 0.0, np.zeros((len(sources), len(receivers)))
    for k, (si, sj) in enumerate(sources):
        T = orc.solve_fmm(h / s, mats, mid, ori, (si * s, sj * s), R)
        for r, (ri, rj) in enumerate(receivers):
            trec[k, r] = T[rj * s, ri * s]
            L += 0.5 * (trec[k, r] - obs[k, r]) ** 2
    return L, trec


def misfit_gradient(orc, h, mats, mat_id, orient, sources, receivers, obs, s, R=2):
    """(L, modelled times, dL/dtheta [nz, nx]) on the s-fold grid."""
    nz, nx = np.shape(mat_id)
    mid, ori = orc.refine_medium(mat_id, orient, s)
    L, trec = 0.0, np.zeros((len(sources), len(receivers)))
    gf = np.zeros(mid.shape)
    for k, (si, sj) in enumerate(sources):
        src = (si * s, sj * s)
        T = orc.solve_fmm(h / s, mats, mid, ori, src, R)
        g = np.zeros(mid.shape)
        for r, (ri, rj) in enumerate(receivers):
            trec[k, r] = T[rj * s, ri * s]
            d = trec[k, r] - obs[k, r]
            L += 0.5 * d * d
            g[rj * s, ri * s] += d
        gf += orc.adjoint(h / s, mats, mid, ori, src, g, R)[1]
    jz, ix = _maps(nz, nx, s)
    G = np.zeros((nz, nx))
    np.add.at(G, (jz[:, None], ix[None, :]), gf)
    return L, trec, G
