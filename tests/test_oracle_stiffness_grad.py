"""Pins for the oracle's gradient with respect to the stiffness of every node.

The parameters are the density-normalised stiffnesses A = C / rho of each node (A11, A13,
A33, A55; the in-plane qP speeds depend on A only).  A stencil estimate (Section 4.2)
depends on A_D through the phase speed at the normal's angle, a straight ray (fallback
and source box, Sections 4.3-4.4) through the group speed of its node.  Pins:
  - the phase-speed derivative against its closed forms along the two symmetry directions
    (v^2 = A11 and v^2 = A33), against central differences, and against Euler's identity
    (v is homogeneous of degree 1/2 in A);
  - the group-speed derivative against the envelope theorem (at the phase angle that
    carries a group angle, dV/dA = V / v dv/dA) and Euler's identity;
  - the stencil partials against central differences of the stencil estimate;
  - the adjoint against central differences of the frozen-choice field under a change of
    one node's stiffness, and of the full solver under a change of one material;
  - the whole-field identity sum over nodes of A . dL/dA = -1/2 sum g T (every travel time
    is homogeneous of degree -1/2 in the stiffnesses of all nodes together).
"""
import math

import numpy as np
import pytest

import synthmedia as sm

KEYS = ("c11", "c13", "c33", "c55")


def _A(mat):
    return np.array([mat[k] for k in KEYS]) / mat["rho"]


def _bump(mat, k, dA):
    m = dict(mat)
    m[KEYS[k]] += dA * mat["rho"]
    return m


MATS = (sm.TI_STEEL, sm.CUBIC_STEEL, sm.PARENT_STEEL, sm.elliptic(3.6e7, 2.2e7, 1.1e7))


def test_phase_speed_dA_symmetry_directions(orc):
    for mat in MATS:
        A = _A(mat)
        # along the c22 axis v^2 = A11, along the symmetry axis v^2 = A33
        for th, k in ((0.0, 0), (math.pi, 0), (0.5 * math.pi, 2), (-0.5 * math.pi, 2)):
            d = orc.qp_phase_speed_dA(mat, th)
            want = np.zeros(4)
            want[k] = 0.5 / math.sqrt(A[k])
            assert np.allclose(d, want, rtol=1e-12, atol=1e-12 * want[k]), (th, d, want)


def test_phase_speed_dA_differences_and_euler(orc):
    for mat in MATS:
        A = _A(mat)
        for th in np.linspace(-3.0, 3.0, 31):
            d = orc.qp_phase_speed_dA(mat, th)
            v = orc.qp_phase_speed(mat, th)
            assert abs(A @ d - 0.5 * v) <= 1e-12 * v
            for k in range(4):
                e = 1e-4 * A.mean()
                fd = (orc.qp_phase_speed(_bump(mat, k, e), th) - orc.qp_phase_speed(_bump(mat, k, -e), th)) / (2 * e)
                assert abs(d[k] - fd) <= 1e-6 * np.abs(d).max(), (th, k, d[k], fd)


def test_group_speed_dA_envelope_and_euler(orc):
    for mat in MATS:
        A = _A(mat)
        for psi in np.linspace(0.02, 1.55, 23):
            phi, V = orc.qp_group_from_phase(mat, psi)
            v = orc.qp_phase_speed(mat, psi)
            want = V / v * orc.qp_phase_speed_dA(mat, psi)
            for ang in (phi, -phi, math.pi - phi, phi + math.pi):
                d = orc.qp_group_speed_dA(mat, ang)
                assert np.allclose(d, want, rtol=0, atol=1e-8 * np.abs(want).max()), (psi, ang, d, want)
                assert abs(A @ d - 0.5 * V) <= 1e-10 * V


def _plane_wave_times(rng, off, h, v=6000.0):
    ang = rng.uniform(-math.pi, math.pi)
    n = np.array([math.cos(ang), math.sin(ang)])
    return [float(n @ np.array(p)) * h / v + 1e-5 + rng.normal(0, 2e-10) for p in off]


def test_stencil_partials_dA_vs_central_differences(orc):
    rng = np.random.default_rng(5)
    h = 1e-4
    checked = 0
    for it in range(900):
        mat = MATS[it % 3]
        A = _A(mat)
        s = int(rng.integers(0, 32))
        off = orc.stencil_offsets(s)
        th = rng.uniform(-3, 3)
        t = _plane_wave_times(rng, off, h)
        if not (t[0] < t[1] <= t[2]):
            continue
        U = orc.stencil_estimate(mat, th, h, off, *t)
        if not U > t[2]:
            continue
        d = orc.stencil_partials(mat, th, h, off, *t, with_A=True)
        dA = d[4]
        # dU/dA . A = -(U - tau_B) / 2: the increment is homogeneous of degree -1/2 in A
        assert abs(A @ dA + 0.5 * (U - t[1])) <= 1e-10 * (U - t[1])
        for k in range(4):
            e = 1e-4 * A.mean()
            fd = (orc.stencil_estimate(_bump(mat, k, e), th, h, off, *t)
                  - orc.stencil_estimate(_bump(mat, k, -e), th, h, off, *t)) / (2 * e)
            assert abs(dA[k] - fd) <= 1e-6 * np.abs(dA).max(), (s, k, dA[k], fd)
        checked += 1
    assert checked > 100


def _misfit(T, rec, d):
    return 0.5 * sum((T[r[1], r[0]] - d[k]) ** 2 for k, r in enumerate(rec))


def _g(T, rec, d):
    g = np.zeros_like(T)
    for k, r in enumerate(rec):
        g[r[1], r[0]] += T[r[1], r[0]] - d[k]
    return g


@pytest.mark.parametrize("seed", [4, 7])
def test_adjoint_dA_vs_frozen_choice_differences(orc, seed):
    m = sm.random_medium(24, 20, 0.2e-3, seed=seed, n_mats=3)
    src = m.sources[0]
    T, pops, choice = orc.frozen_setup(m.h, m.mats, m.mat_id, m.orient, src)
    rec = [(23, 19), (0, 19), (12, 0), (5, 13)]
    d = [T[r[1], r[0]] * 0.97 for r in rec]
    T2, _, dA = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, _g(T, rec, d), with_A=True)
    assert np.array_equal(T, T2)
    nz_nodes = np.argwhere(np.abs(dA).sum(axis=2) > 0)
    rng = np.random.default_rng(seed)
    nodes = [(src[1], src[0])] + [tuple(v) for v in nz_nodes[rng.permutation(len(nz_nodes))[:8]]]
    scale = np.abs(dA).max()
    for (j, i) in nodes:
        base = m.mats[m.mat_id[j, i]]
        A = _A(base)
        for k in range(4):
            e = 1e-5 * A.mean()
            mid = m.mat_id.copy()
            mid[j, i] = len(m.mats)
            Lp = _misfit(orc.frozen_field(m.h, list(m.mats) + [_bump(base, k, e)], mid, m.orient, src, choice, pops),
                         rec, d)
            Lm = _misfit(orc.frozen_field(m.h, list(m.mats) + [_bump(base, k, -e)], mid, m.orient, src, choice, pops),
                         rec, d)
            fd = (Lp - Lm) / (2 * e)
            assert abs(dA[j, i, k] - fd) <= 1e-6 * scale, (i, j, k, dA[j, i, k], fd)


def test_adjoint_dA_material_vs_full_solver(orc):
    # changing one material's A_k everywhere it is used: dT(r)/dA_k is the sum of dA over
    # that material's nodes (full solver, choices free to switch; none for so small a step)
    m = sm.random_medium(28, 24, 0.2e-3, seed=9, n_mats=3)
    src = m.sources[0]
    for r in [(27, 23), (0, 23), (14, 0)]:
        g = np.zeros((m.nz, m.nx))
        g[r[1], r[0]] = 1.0
        _, _, dA = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g, with_A=True)
        for mi in range(len(m.mats)):
            sel = m.mat_id == mi
            if not sel.any():
                continue
            A = _A(m.mats[mi])
            for k in range(4):
                e = 1e-6 * A.mean()
                mp, mm = list(m.mats), list(m.mats)
                mp[mi] = _bump(m.mats[mi], k, e)
                mm[mi] = _bump(m.mats[mi], k, -e)
                Tp = orc.solve_fmm(m.h, mp, m.mat_id, m.orient, src, 2)
                Tm = orc.solve_fmm(m.h, mm, m.mat_id, m.orient, src, 2)
                fd = (Tp[r[1], r[0]] - Tm[r[1], r[0]]) / (2 * e)
                got = dA[sel][:, k].sum()
                assert abs(got - fd) <= 1e-5 * np.abs(dA).sum(axis=(0, 1)).max() + 1e-25, (r, mi, k, got, fd)


@pytest.mark.parametrize("seed", [3, 11])
def test_adjoint_dA_euler_identity(orc, seed):
    m = sm.random_medium(26, 22, 0.2e-3, seed=seed, n_mats=3)
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(m.nz, m.nx))
    T, _, dA = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], g, with_A=True)
    Anode = np.stack([_A(m.mats[k]) for k in range(len(m.mats))])[m.mat_id]
    lhs = float((Anode * dA).sum())
    rhs = -0.5 * float((g * T).sum())
    assert abs(lhs - rhs) <= 1e-10 * float(np.abs(g * T).sum()), (lhs, rhs)


def test_adjoint_without_A_unchanged(orc):
    m = sm.random_medium(20, 18, 0.2e-3, seed=11)
    g = np.random.default_rng(1).normal(size=(18, 20))
    T1, d1 = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], g)
    T2, d2, _ = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], g, with_A=True)
    assert np.array_equal(T1, T2) and np.array_equal(d1, d2)
