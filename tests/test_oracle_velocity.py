"""Pins for the oracle's velocities (paper Section 3) against closed forms that do not
go through the oracle's own formulas."""
import math

import numpy as np
import pytest

import synthmedia as sm


def a_of(mat):
    r = mat["rho"]
    return mat["c11"] / r, mat["c13"] / r, mat["c33"] / r, mat["c55"] / r


def test_axis_values(orc):
    # Section 3.2: on the c22 axis lambda = c22, on the symmetry axis lambda = c33
    for mat in (sm.TI_STEEL, sm.CUBIC_STEEL):
        a11, _, a33, _ = a_of(mat)
        assert orc.qp_phase_speed(mat, 0.0) == pytest.approx(math.sqrt(a11), rel=1e-15)
        assert orc.qp_phase_speed(mat, math.pi / 2) == pytest.approx(math.sqrt(a33), rel=1e-15)


def test_hand_computed_values(orc):
    # phase speeds at 0, 45 and 90 degrees worked out by hand from the closed-form roots of
    # the 2 x 2 Christoffel matrix (to 0.1 m/s): TI steel 5454.6 / 6210.3 / 5164.0, cubic
    # steel 5092.8 / 6164.9 / 5092.8
    got = [orc.qp_phase_speed(sm.TI_STEEL, math.radians(a)) for a in (0, 45, 90)]
    assert [round(v, 1) for v in got] == [5454.6, 6210.3, 5164.0]
    got = [orc.qp_phase_speed(sm.CUBIC_STEEL, math.radians(a)) for a in (0, 45, 90)]
    assert [round(v, 1) for v in got] == [5092.8, 6164.9, 5092.8]


def test_isotropic_constant(orc):
    # Section 3.2: isotropic media need no Christoffel solve, v is constant
    mat = sm.isotropic(5900.0, 3200.0, 8100.0)
    for a in np.linspace(-3, 3, 37):
        assert orc.qp_phase_speed(mat, a) == pytest.approx(5900.0, rel=1e-14)
        assert orc.qp_group_speed(mat, a) == pytest.approx(5900.0, rel=1e-12)


def test_elliptic_closed_form(orc):
    # (c13 + c55)^2 = (c11 - c55)(c33 - c55): v^2 = a11 cos^2 + a33 sin^2 (phase angle from
    # the c22 axis) and the group curve is the ellipse 1/V^2 = cos^2/a11 + sin^2/a33.
    a11, a33, a55 = 3.6e7, 2.2e7, 1.1e7
    mat = sm.elliptic(a11, a33, a55)
    for a in np.linspace(-1.5, 3.0, 41):
        v2 = a11 * math.cos(a) ** 2 + a33 * math.sin(a) ** 2
        assert orc.qp_phase_speed(mat, a) == pytest.approx(math.sqrt(v2), rel=1e-13)
        V = 1.0 / math.sqrt(math.cos(a) ** 2 / a11 + math.sin(a) ** 2 / a33)
        assert orc.qp_group_speed(mat, a) == pytest.approx(V, rel=1e-11)


@pytest.mark.parametrize("name", ["ti", "cubic"])
def test_group_two_routes(orc, name):
    # polarisation-vector group velocity inverted by bisection vs the slowness support function
    mat = sm.TI_STEEL if name == "ti" else sm.CUBIC_STEEL
    for a in np.linspace(0.0, math.pi, 46):
        g1 = orc.qp_group_speed(mat, a)
        g2 = orc.qp_group_speed_support(mat, a)
        assert g1 == pytest.approx(g2, rel=1e-11)


def test_group_equals_phase_on_axes(orc):
    # Section 3.2: for angles that are multiples of 90 deg group and phase coincide
    for mat in (sm.TI_STEEL, sm.CUBIC_STEEL):
        for a in (0.0, math.pi / 2, math.pi):
            ga, gs = orc.qp_group_from_phase(mat, a)
            assert gs == pytest.approx(orc.qp_phase_speed(mat, a), rel=1e-14)
            assert abs(math.remainder(ga - a, math.pi)) < 1e-12


def test_group_angle_monotone_and_bound(orc):
    # the phase->group angle map is monotone on [0, 90 deg] (bisection relies on it) and
    # |V| = |v| / cos(theta') with theta' the group-phase angle (Section 3.1)
    for mat in (sm.TI_STEEL, sm.CUBIC_STEEL):
        prev = -1.0
        for a in np.linspace(0.0, math.pi / 2, 181):
            ga, gs = orc.qp_group_from_phase(mat, a)
            assert ga >= prev - 1e-15
            prev = ga
            v = orc.qp_phase_speed(mat, a)
            assert gs == pytest.approx(v / math.cos(ga - a), rel=1e-12)


def test_symmetries(orc):
    # 180 deg symmetry and mirror symmetry of an orthotropic curve
    mat = sm.TI_STEEL
    for a in np.linspace(0.05, 1.5, 9):
        v = orc.qp_phase_speed(mat, a)
        assert orc.qp_phase_speed(mat, -a) == pytest.approx(v, rel=1e-15)
        assert orc.qp_phase_speed(mat, a + math.pi) == pytest.approx(v, rel=1e-14)
        assert orc.qp_group_speed(mat, math.pi - a) == pytest.approx(orc.qp_group_speed(mat, a), rel=1e-13)
