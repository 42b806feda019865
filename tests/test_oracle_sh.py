"""Pins for the oracle's SH mode (the shear wave polarised normal to the plane; the paper
names S waves as an extension in Section 6).

The SH Christoffel entry is c66 n1^2 + c44 n3^2, an elliptical slowness curve:
  - phase speeds along the two symmetry directions are sqrt(c66/rho) and sqrt(c44/rho);
  - the closed-form group speed (an elliptical wave surface) equals the support-function
    route max cos(phi - psi) / v(psi) computed from the SH phase speed;
  - the derivatives match central differences;
  - a qP material with an exactly elliptical qP curve of the same axes (A11 = c66/rho,
    A33 = c44/rho) has the same phase and group speeds by a different formula (the
    Christoffel root and the polarisation-vector group velocity), so every solver must give
    the same result for it in qP mode as for the SH material in SH mode;
  - homogeneous SH media: straight-ray box exact, field within the discretisation error of
    the exact ellipse times, and the nested source grids reduce that error.
"""
import math

import numpy as np
import pytest

import synthmedia as sm

SH_MATS = [sm.TI_STEEL, dict(sm.CUBIC_STEEL, c66=60e9), dict(sm.PARENT_STEEL, c66=40e9)]


def _equivalent_qp(mat):
    """qP record whose qP curve is the SH ellipse of mat (a55 below both axes)."""
    a66, a44 = mat["c66"] / mat["rho"], mat["c44"] / mat["rho"]
    return sm.elliptic(a66, a44, 0.5 * min(a66, a44), mat["rho"])


def test_sh_speeds_closed_forms(orc):
    for mat in orc.as_sh(SH_MATS):
        assert math.isclose(orc.phase_speed(mat, 0.0), math.sqrt(mat["c66"] / mat["rho"]), rel_tol=1e-15)
        assert math.isclose(orc.phase_speed(mat, 0.5 * math.pi), math.sqrt(mat["c44"] / mat["rho"]), rel_tol=1e-15)
        for ang in (0.0, 0.5 * math.pi, math.pi):
            assert math.isclose(orc.group_speed(mat, ang), orc.phase_speed(mat, ang), rel_tol=1e-14)
        for phi in np.linspace(-3.0, 3.0, 41):
            assert math.isclose(orc.group_speed(mat, phi), orc.group_speed_support(mat, phi), rel_tol=1e-11)


def test_sh_derivatives(orc):
    for mat in orc.as_sh(SH_MATS):
        for a in np.linspace(-3.0, 3.0, 29):
            e = 1e-5
            fd = (orc.phase_speed(mat, a + e) - orc.phase_speed(mat, a - e)) / (2 * e)
            assert abs(orc.phase_speed_deriv(mat, a) - fd) <= 1e-6 * max(abs(fd), 1.0)
            fd = (orc.group_speed(mat, a + e) - orc.group_speed(mat, a - e)) / (2 * e)
            assert abs(orc.group_speed_deriv(mat, a) - fd) <= 1e-6 * max(abs(fd), 1.0)


def test_sh_speeds_equal_elliptic_qp(orc):
    for mat in SH_MATS:
        sh, qp = orc.as_sh([mat])[0], _equivalent_qp(mat)
        for a in np.linspace(-3.0, 3.0, 37):
            assert math.isclose(orc.phase_speed(sh, a), orc.qp_phase_speed(qp, a), rel_tol=1e-13)
            assert math.isclose(orc.group_speed(sh, a), orc.qp_group_speed(qp, a), rel_tol=1e-12)


@pytest.mark.parametrize("seed", [2, 9])
def test_sh_solvers_equal_elliptic_qp(orc, seed):
    m = sm.random_medium(31, 27, 0.2e-3, seed=seed, n_mats=3)
    sh = orc.as_sh(SH_MATS)
    qp = [_equivalent_qp(x) for x in SH_MATS]
    src = m.sources[0]
    Ts = orc.solve_fmm(m.h, sh, m.mat_id, m.orient, src, 2)
    Tq = orc.solve_fmm(m.h, qp, m.mat_id, m.orient, src, 2)
    assert np.allclose(Ts, Tq, rtol=1e-12, atol=0)
    Ts = orc.solve_refined(m.h, sh, m.mat_id, m.orient, src)
    Tq = orc.solve_refined(m.h, qp, m.mat_id, m.orient, src)
    assert np.allclose(Ts, Tq, rtol=1e-12, atol=0)
    g = np.random.default_rng(seed).normal(size=(m.nz, m.nx))
    _, ds = orc.adjoint(m.h, sh, m.mat_id, m.orient, src, g)
    _, dq = orc.adjoint(m.h, qp, m.mat_id, m.orient, src, g)
    assert np.abs(ds - dq).max() <= 1e-8 * np.abs(dq).max()
    p1, t1, ok1 = orc.trace_ray(m.h, sh, m.mat_id, m.orient, Ts, src, (30, 26))
    p2, t2, ok2 = orc.trace_ray(m.h, qp, m.mat_id, m.orient, Tq, src, (30, 26))
    assert ok1 and ok2 and len(p1) == len(p2)
    assert np.allclose(p1, p2, atol=1e-9) and math.isclose(t1, t2, rel_tol=1e-12)


def test_sh_stiffness_gradient_is_refused(orc):
    m = sm.random_medium(12, 12, 0.2e-3, seed=1)
    with pytest.raises(ValueError):
        orc.adjoint(m.h, orc.as_sh(m.mats), m.mat_id, m.orient, m.sources[0], np.ones((12, 12)), with_A=True)


def test_sh_homogeneous_accuracy(orc):
    mat = orc.as_sh([sm.TI_STEEL])[0]
    h, n = 1e-3, 31
    c = n // 2
    for th in (0.0, 0.6):
        mid, ori = np.zeros((n, n), np.uint8), np.full((n, n), th)
        Tb = orc.solve_fmm(h, [mat], mid, ori, (c, c), 2)
        Tr = orc.solve_refined(h, [mat], mid, ori, (c, c))
        eb, er = [], []
        for j in range(n):
            for i in range(n):
                if i == c and j == c:
                    continue
                t = math.hypot(i - c, j - c) * h / orc.group_speed(mat, math.atan2(j - c, i - c) - (th + 0.5 * math.pi))
                if max(abs(i - c), abs(j - c)) <= 2:
                    assert math.isclose(Tb[j, i], t, rel_tol=1e-14)
                eb.append(abs(Tb[j, i] - t) / t)
                er.append(abs(Tr[j, i] - t) / t)
        # box: about 4 % (the qP cubic-steel box gives the same); the source grids: about 1 %
        assert np.mean(eb) < 0.06 and np.mean(er) < 0.02 and np.mean(er) < 0.5 * np.mean(eb), (th, np.mean(eb), np.mean(er))
