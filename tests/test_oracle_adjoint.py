"""Pins for the oracle's orientation gradient (frozen choices, reverse pop order).

The gradient is not in the paper; it differentiates the paper's local update
(Section 4.2: point E, foot point F, |FD| over the phase speed at the normal's angle),
its straight-ray fallback and its source box (Section 4.4).  Pins:
  - the velocity derivatives against central differences of the pinned speeds;
  - the hand-derived stencil partials against central differences of the stencil
    estimate, and the shift invariance dU/dta + dU/dtb + dU/dtc = 1;
  - the adjoint against central differences of the frozen-choice field (tight), and of
    the full solver (choices free to switch) under a uniform rotation of every node;
  - isotropic media give a zero gradient; the gradient is linear in dL/dT;
  - the ray-path gradient (the time along the traced ray, path held fixed) is a different
    discretisation of the same derivative: projected onto a smooth control grid the two
    agree better as the grid is refined, cosine at least 0.95 at 128 x 128.
"""
import math

import numpy as np
import pytest

import synthmedia as sm


def test_phase_speed_derivative(orc):
    for mat in (sm.TI_STEEL, sm.CUBIC_STEEL, sm.elliptic(3.6e7, 2.2e7, 1.1e7)):
        for th in np.linspace(-3.0, 3.0, 37):
            e = 1e-5
            fd = (orc.qp_phase_speed(mat, th + e) - orc.qp_phase_speed(mat, th - e)) / (2 * e)
            d = orc.qp_phase_speed_deriv(mat, th)
            assert abs(d - fd) <= 1e-6 * max(abs(fd), 1.0)


def test_group_speed_derivative(orc):
    for mat in (sm.TI_STEEL, sm.CUBIC_STEEL):
        for phi in np.linspace(-3.0, 3.0, 25):
            e = 1e-4
            fd = (orc.qp_group_speed(mat, phi + e) - orc.qp_group_speed(mat, phi - e)) / (2 * e)
            assert abs(orc.qp_group_speed_deriv(mat, phi) - fd) <= 1e-4 * max(abs(fd), 1.0)
    # isotropic: constant speed
    assert abs(orc.qp_group_speed_deriv(sm.PARENT_STEEL, 0.7)) < 1e-6


def _plane_wave_times(rng, off, h, v=6000.0):
    ang = rng.uniform(-math.pi, math.pi)
    n = np.array([math.cos(ang), math.sin(ang)])
    return [float(n @ np.array(p)) * h / v + 1e-5 + rng.normal(0, 2e-10) for p in off]


def test_stencil_partials_vs_central_differences(orc):
    rng = np.random.default_rng(0)
    mat, h = sm.TI_STEEL, 1e-4
    checked = 0
    for _ in range(1200):
        s = int(rng.integers(0, 32))
        off = orc.stencil_offsets(s)
        th = rng.uniform(-3, 3)
        t = _plane_wave_times(rng, off, h)
        if not (t[0] < t[1] <= t[2]):
            continue
        U = orc.stencil_estimate(mat, th, h, off, *t)
        if not U > t[2]:
            continue
        d = orc.stencil_partials(mat, th, h, off, *t)
        fd = []
        for k in range(3):
            eps = 1e-13
            tp, tm = list(t), list(t)
            tp[k] += eps
            tm[k] -= eps
            fd.append((orc.stencil_estimate(mat, th, h, off, *tp) - orc.stencil_estimate(mat, th, h, off, *tm)) / (2 * eps))
        e = 1e-6
        fd.append((orc.stencil_estimate(mat, th + e, h, off, *t) - orc.stencil_estimate(mat, th - e, h, off, *t)) / (2 * e))
        for k in range(3):
            assert abs(d[k] - fd[k]) <= 2e-5 * max(abs(fd[k]), 1.0)
        assert abs(d[3] - fd[3]) <= 1e-5 * abs(fd[3]) + 1e-15
        # adding a constant to all three known times adds it to the estimate
        assert abs(d[0] + d[1] + d[2] - 1.0) <= 1e-9
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
def test_adjoint_vs_frozen_choice_differences(orc, seed):
    m = sm.random_medium(24, 20, 0.2e-3, seed=seed)
    src = m.sources[0]
    T, pops, choice = orc.frozen_setup(m.h, m.mats, m.mat_id, m.orient, src)
    rec = [(23, 19), (0, 19), (12, 0), (5, 13)]
    d = [T[r[1], r[0]] * 0.97 for r in rec]
    T2, dth = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, _g(T, rec, d))
    assert np.array_equal(T, T2)
    # frozen recomputation reproduces the field exactly
    assert np.array_equal(orc.frozen_field(m.h, m.mats, m.mat_id, m.orient, src, choice, pops), T)
    rng = np.random.default_rng(seed)
    nodes = [(src[1], src[0])] + [tuple(v) for v in np.argwhere(np.abs(dth) > 0)[rng.permutation(
        int((np.abs(dth) > 0).sum()))[:10]]]
    for (j, i) in nodes:
        e = 1e-6
        op, om = m.orient.copy(), m.orient.copy()
        op[j, i] += e
        om[j, i] -= e
        fd = (_misfit(orc.frozen_field(m.h, m.mats, m.mat_id, op, src, choice, pops), rec, d)
              - _misfit(orc.frozen_field(m.h, m.mats, m.mat_id, om, src, choice, pops), rec, d)) / (2 * e)
        assert abs(dth[j, i] - fd) <= 1e-6 * np.abs(dth).max(), (i, j, dth[j, i], fd)


def test_adjoint_uniform_rotation_vs_full_solver(orc):
    # rotating every node by the same angle: d T(r) / d angle = sum of the gradient for
    # g = unit at r; the full solver is differenced (choices may switch, none expected
    # for so small a step in this medium)
    for nm, seed in ((1, 9), (3, 9), (3, 12)):
        _uniform_rotation_case(orc, sm.random_medium(28, 24, 0.2e-3, seed=seed, n_mats=nm))


def _uniform_rotation_case(orc, m):
    src = m.sources[0]
    for r in [(27, 23), (0, 23), (14, 0)]:
        g = np.zeros((m.nz, m.nx))
        g[r[1], r[0]] = 1.0
        _, dth = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g)
        e = 1e-7
        Tp = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient + e, src, 2)
        Tm = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient - e, src, 2)
        fd = (Tp[r[1], r[0]] - Tm[r[1], r[0]]) / (2 * e)
        # FD noise: rounding of T (~1e-22 s) over the step
        assert abs(dth.sum() - fd) <= 1e-5 * abs(fd) + 1e-13, (m.name, r, dth.sum(), fd)


def test_isotropic_gradient_is_zero(orc):
    m = sm.homogeneous(20, 20, 1e-3, sm.PARENT_STEEL, 10.0, (4, 6))
    rng = np.random.default_rng(2)
    g = rng.normal(size=(20, 20))
    T, dth = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, (4, 6), g)
    # zero up to the rounding of the numerical group-speed derivative
    assert np.abs(dth).max() < 1e-12 * np.abs(g).sum() * T.max()


def test_gradient_linear_in_g(orc):
    m = sm.random_medium(20, 18, 0.2e-3, seed=11)
    rng = np.random.default_rng(3)
    g1, g2 = rng.normal(size=(18, 20)), rng.normal(size=(18, 20))
    _, a = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], g1)
    _, b = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], g2)
    _, c = orc.adjoint(m.h, m.mats, m.mat_id, m.orient, m.sources[0], 2.0 * g1 - g2)
    assert np.allclose(c, 2.0 * a - b, rtol=0, atol=1e-12 * np.abs(c).max())


def test_control_gradient_vs_full_differences(orc):
    # misfit over a small bilinear control grid (the tomography setting): adjoint
    # gradient through the bilinear transpose against central differences of the full
    # solver on each control value, with steps 1e-5 and 1e-3 rad
    n, nc, h = 24, 4, 0.2e-3
    W = sm.bilinear_weights(n, nc)
    ctrl_true = sm.bilinear_controls(nc, 1)
    ctrl = sm.bilinear_controls(nc, 2)
    mats, mid = [sm.TI_STEEL], np.zeros((n, n), np.uint8)
    srcs = [(4, 0), (12, 0), (19, 0)]
    recs = [(3, n - 1), (11, n - 1), (20, n - 1)]
    th_true = W @ ctrl_true @ W.T
    dobs = [[orc.solve_fmm(h, mats, mid, th_true, s, 2)[r[1], r[0]] for r in recs] for s in srcs]

    def loss(c):
        th = W @ c @ W.T
        return sum(_misfit(orc.solve_fmm(h, mats, mid, th, s, 2), recs, dobs[k]) for k, s in enumerate(srcs))

    th = W @ ctrl @ W.T
    dth = np.zeros((n, n))
    for k, s in enumerate(srcs):
        T = orc.solve_fmm(h, mats, mid, th, s, 2)
        dth += orc.adjoint(h, mats, mid, th, s, _g(T, recs, dobs[k]))[1]
    grad = W.T @ dth @ W
    for e in (1e-5, 1e-3):
        fd = np.zeros_like(ctrl)
        for a in range(nc):
            for b in range(nc):
                cp, cm = ctrl.copy(), ctrl.copy()
                cp[a, b] += e
                cm[a, b] -= e
                fd[a, b] = (loss(cp) - loss(cm)) / (2 * e)
        cos = float((grad * fd).sum() / (np.linalg.norm(grad) * np.linalg.norm(fd)))
        rel = np.abs(grad - fd) / np.abs(fd).max()
        if e < 1e-4:
            # small step: no stencil switch, the full solver is locally the frozen map
            assert rel.max() <= 1e-6, rel.max()
        else:
            # 1e-3 rad: a switch moves single entries by a few percent
            assert cos >= 0.99, cos
            assert np.median(rel) <= 1e-2, np.median(rel)


def test_adjoint_vs_ray_path_gradient(orc):
    # One source, six receivers with random weights, TI steel with a smooth orientation
    # (6 x 6 bilinear controls) on the same physical square at 32, 64 and 128 nodes per side.
    # Both gradients are projected onto the controls (W^T G W).  Measured: cosine 0.825 /
    # 0.898 / 0.963, norm ratio adjoint / ray 0.61 / 0.68 / 0.76: the field's discretisation
    # error varies with the orientation, and that variation shrinks with the cell size.
    from raypath_grad import cosine, ray_path_gradient
    rng = np.random.default_rng(3)
    nc = 6
    ctrl = rng.uniform(-0.8, 0.8, size=(nc, nc))
    src63, recs63 = (20, 0), [(5, 63), (30, 63), (50, 63), (63, 40), (63, 20), (40, 63)]
    w = rng.normal(size=len(recs63))
    mats = [sm.TI_STEEL]
    cos, ratio = [], []
    for n in (32, 64, 128):
        h = 0.5e-3 * 64 / n
        W = sm.bilinear_weights(n, nc)
        th = W @ ctrl @ W.T
        mid = np.zeros((n, n), np.uint8)

        def at(p):
            return (int(round(p[0] * (n - 1) / 63)), int(round(p[1] * (n - 1) / 63)))

        src = at(src63)
        T = orc.solve_fmm(h, mats, mid, th, src, 2)
        g = np.zeros((n, n))
        ray = np.zeros((n, n))
        for r63, wk in zip(recs63, w):
            r = at(r63)
            g[r[1], r[0]] += wk
            pts, t, ok = orc.trace_ray(h, mats, mid, th, T, src, r)
            assert ok
            ray += wk * ray_path_gradient(orc, h, mats, mid, th, pts)
        adj = orc.adjoint(h, mats, mid, th, src, g)[1]
        ga, gr = W.T @ adj @ W, W.T @ ray @ W
        cos.append(cosine(ga, gr))
        ratio.append(float(np.linalg.norm(ga) / np.linalg.norm(gr)))
    print("control-space cosine", cos, "norm ratio", ratio)
    assert cos[0] < cos[1] < cos[2] and cos[2] >= 0.95
    assert ratio[0] < ratio[1] < ratio[2] <= 1.0 and ratio[2] >= 0.7
