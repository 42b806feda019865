"""Pins for the oracle's stencil table (Tables 1-2) and single-stencil estimate
(Sections 4.1-4.2)."""
import math

import numpy as np
import pytest

import synthmedia as sm

D4 = [lambda x, y: (x, y), lambda x, y: (-x, y), lambda x, y: (x, -y), lambda x, y: (-x, -y),
      lambda x, y: (y, x), lambda x, y: (-y, x), lambda x, y: (y, -x), lambda x, y: (-y, -x)]


def table(orc):
    return [tuple(orc.stencil_offsets(s)) for s in range(32)]


def test_table_shape(orc):
    t = table(orc)
    assert len(set(t)) == 32
    for s, (A, B, C) in enumerate(t):
        for p in (A, B, C):
            assert 0 < abs(p[0]) + abs(p[1]) <= 2          # inside the 12-node diamond
        # pairs share A (and D) and swap B and C (Section 4.1)
        if s % 2 == 0:
            A2, B2, C2 = t[s + 1]
            assert A2 == A and B2 == C and C2 == B
        # B and C are neighbours of A (the stencil is a square or a triangle with D)
        assert max(abs(A[0] - B[0]), abs(A[1] - B[1])) == 1
        assert max(abs(A[0] - C[0]), abs(A[1] - C[1])) == 1


def test_table_classes(orc):
    t = table(orc)
    for s, (A, B, C) in enumerate(t):
        if s < 8:     # small squares: A diagonal, B and C axial
            assert abs(A[0]) == abs(A[1]) == 1
            assert abs(B[0]) + abs(B[1]) == 1 and abs(C[0]) + abs(C[1]) == 1
        elif s < 16:  # big squares: A at distance 2 on an axis, B and C diagonal
            assert abs(A[0]) + abs(A[1]) == 2 and 0 in A
            assert abs(B[0]) == abs(B[1]) == 1 and abs(C[0]) == abs(C[1]) == 1
        else:         # triangles: first member B axial / C diagonal, second swapped
            assert abs(A[0]) + abs(A[1]) == 2 and 0 in A
            ax, dg = (B, C) if s % 2 == 0 else (C, B)
            assert abs(ax[0]) + abs(ax[1]) == 1 and abs(dg[0]) == abs(dg[1]) == 1


def test_table_d4_closed(orc):
    # with the two printing errors corrected, the family is closed under the symmetry
    # group of the square (an uncorrected row breaks this)
    t = set(table(orc))
    for (A, B, C) in t:
        for g in D4:
            assert (g(*A), g(*B), g(*C)) in t


def plane_wave(orc, mat, ang, th_ax, h, offsets, t0=0.0):
    """Times of the support points for the plane wave tau = n.x / v(n) (closed form for
    an elliptic medium, independent of the oracle's velocity code)."""
    r = mat["rho"]
    a11, a33 = mat["c11"] / r, mat["c33"] / r
    psi = ang - th_ax                              # normal vs symmetry axis
    v = math.sqrt(a33 * math.cos(psi) ** 2 + a11 * math.sin(psi) ** 2)
    n = (math.cos(ang), math.sin(ang))
    return [t0 + (n[0] * p[0] + n[1] * p[1]) * h / v for p in offsets], v


def test_plane_wave_exact(orc):
    # linear interpolation and the normal of EB are exact for a linear field, and the phase
    # speed is exact: every usable stencil reproduces tau_D of a plane wave
    mat = sm.elliptic(3.6e7, 2.2e7, 1.1e7)
    rng = np.random.default_rng(0)
    h = 1e-3
    used = 0
    for _ in range(300):
        ang = rng.uniform(-math.pi, math.pi)
        th_ax = rng.uniform(-math.pi, math.pi)
        for s in range(32):
            off = orc.stencil_offsets(s)
            t, v = plane_wave(orc, mat, ang, th_ax, h, off)
            if not (t[0] < t[1] <= t[2]):
                continue
            U = orc.stencil_estimate(mat, th_ax, h, off, *t)
            if U > t[2]:
                used += 1
                assert abs(U - 0.0) <= 1e-12 * (h / v)
    assert used > 300


def test_plane_wave_exact_anisotropic(orc):
    # same for the TI steel with the exact phase speed from an independent 2x2 eigen-solve
    mat = sm.TI_STEEL
    r = mat["rho"]
    a11, a13, a33, a55 = mat["c11"] / r, mat["c13"] / r, mat["c33"] / r, mat["c55"] / r
    rng = np.random.default_rng(1)
    h = 1e-4
    for _ in range(200):
        ang = rng.uniform(-math.pi, math.pi)
        th_ax = rng.uniform(-math.pi, math.pi)
        ax = np.array([math.cos(th_ax), math.sin(th_ax)])
        pe = np.array([-ax[1], ax[0]])
        n = np.array([math.cos(ang), math.sin(ang)])
        c, s = n @ ax, n @ pe                     # components along / across the axis
        G = np.array([[a11 * s * s + a55 * c * c, (a13 + a55) * s * c],
                      [(a13 + a55) * s * c, a55 * s * s + a33 * c * c]])
        v = math.sqrt(np.linalg.eigvalsh(G).max())
        for k in range(32):
            off = orc.stencil_offsets(k)
            t = [(n[0] * p[0] + n[1] * p[1]) * h / v for p in off]
            if not (t[0] < t[1] <= t[2]):
                continue
            U = orc.stencil_estimate(mat, th_ax, h, off, *t)
            if U > t[2]:
                assert abs(U) <= 1e-11 * (h / v)


def test_estimate_example_by_hand(orc):
    # stencil 1-1 in an isotropic medium, worked by hand: A=(-1,-1), B=(0,-1), C=(-1,0),
    # tau = 0, 0.5, 1 (units of h/v) -> a = 0.5, E = (-1,-0.5), line EB from (-1,-0.5) to
    # (0,-1); distance of D=(0,0) from it = |(-0.5)(1) + (1)(0.5)... | computed below
    mat = sm.isotropic(1.0, 0.5, 1.0)
    xE, yE = -1.0, -0.5
    xB, yB = 0.0, -1.0
    num = abs((yE - yB) * (0 - xE) + (xB - xE) * (0 - yE))
    den = math.hypot(xB - xE, yB - yE)
    expect = 0.5 + num / den
    U = orc.stencil_estimate(mat, 0.3, 1.0, orc.stencil_offsets(0), 0.0, 0.5, 1.0)
    assert U == pytest.approx(expect, rel=1e-15)
    # = 0.5 + 1/sqrt(1.25) * 1 ... the closed value
    assert U == pytest.approx(0.5 + 1.0 / math.sqrt(1.25), rel=1e-15)
