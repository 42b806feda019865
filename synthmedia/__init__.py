"""Seeded synthetic media for the anisotropic travel-time solver.

This module only draws inputs: grids, stiffness records, per-node material ids and
symmetry-axis orientations, source and receiver nodes.  It holds none of the solver's
arithmetic and is shared by the tests, the benchmark and the CPU oracle runs.

Orientation arrays are returned as float32 values (the GPU path's input precision) held
in float64 arrays, so that the FP64 oracle and the FP32 kernels solve exactly the same
problem.  Random numbers come from numpy's PCG64 generator with the seeds listed here.

Workloads (the paper's EBSD weld and finite-element data are not available; the
synthetic V-weld stands in for them):
  tiny_ti        64x64, h = 0.5 mm, homogeneous TI steel, axis at 30 deg, centre source.
  weld           512x512, h = 0.1 mm, isotropic parent steel (5900 m/s) around a V-shaped
                 TI weld (40 mm top width tapering to 4 mm) whose axis follows
                 atan2(z + 15 mm, |x| + 1 mm) plus N(0, 5 deg) noise per node (seed 0).
  weld_multi     the weld with 64 top-surface sources and 64 bottom-surface receivers.
  adjoint_grid   256x256, h = 0.2 mm, TI everywhere, orientation bilinear from a 32x32
                 control grid with values U(-45, 45) deg (seed 1 = true, 2 = evaluation).
  batch          128 media, square sides U{256..1024} (seed 3), orientations as
                 adjoint_grid with seed 1000 + b, 32 top sources and 32 bottom receivers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GPA = 1.0e9

# TI steel-like weld metal (C12 = 97 GPa -> C66 = (C11 - C12) / 2 = 72 GPa)
TI_STEEL = dict(c11=241 * GPA, c13=138 * GPA, c33=216 * GPA, c55=129 * GPA, c44=129 * GPA,
                c66=72 * GPA, rho=8100.0)
# the paper's austenitic steel (cubic): c11 = 203.6, c12 = 133.5, c44 = 129.8 GPa, rho 7850
CUBIC_STEEL = dict(c11=203.6 * GPA, c13=133.5 * GPA, c33=203.6 * GPA, c55=129.8 * GPA,
                   c44=129.8 * GPA, c66=129.8 * GPA, rho=7850.0)


def isotropic(vp, vs, rho):
    """Isotropic stiffness record with P speed vp and S speed vs."""
    c11 = rho * vp * vp
    c55 = rho * vs * vs
    return dict(c11=c11, c13=c11 - 2 * c55, c33=c11, c55=c55, c44=c55, c66=c55, rho=rho)


PARENT_STEEL = isotropic(5900.0, 3200.0, 8100.0)


def elliptic(a11, a33, a55, rho=1000.0):
    """TI record with an exactly elliptical qP curve: (c13 + c55)^2 = (c11 - c55)(c33 - c55)."""
    c11, c33, c55 = a11 * rho, a33 * rho, a55 * rho
    c13 = math.sqrt((c11 - c55) * (c33 - c55)) - c55
    return dict(c11=c11, c13=c13, c33=c33, c55=c55, c44=c55, c66=c55, rho=rho)


def f32(a):
    """Round to float32 and hold in float64 (the GPU input precision)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclass
class Medium:
    nx: int
    nz: int
    h: float
    mats: list
    mat_id: np.ndarray          # uint8 [nz][nx]
    orient: np.ndarray          # float64 holding float32 values [nz][nx], radians
    sources: list = field(default_factory=list)     # [(i, j)]
    receivers: list = field(default_factory=list)   # [(i, j)]
    name: str = ""


def homogeneous(nx, nz, h, mat, theta_deg, src=None, name="homogeneous"):
    mat_id = np.zeros((nz, nx), np.uint8)
    orient = f32(np.full((nz, nx), math.radians(theta_deg)))
    src = src if src is not None else (nx // 2, nz // 2)
    return Medium(nx, nz, h, [mat], mat_id, orient, [tuple(src)], [], name)


def tiny_ti():
    """64x64, 0.5 mm, homogeneous TI steel with the axis at 30 deg, source at (32, 32)."""
    return homogeneous(64, 64, 0.5e-3, TI_STEEL, 30.0, (32, 32), "tiny_ti")


def weld(n=512, h=0.1e-3, seed=0, n_src=1, n_rec=0):
    """V-shaped TI weld in isotropic parent steel (see module docstring)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    j = np.arange(n)
    x = (i - (n - 1) / 2.0) * h            # centred lateral coordinate
    z = j * h                              # depth
    X, Z = np.meshgrid(x, z)
    zmax = (n - 1) * h
    half_width = 20e-3 - 18e-3 * Z / zmax  # 40 mm wide at the top, 4 mm at the bottom
    inside = np.abs(X) <= half_width
    theta = np.arctan2(Z + 15e-3, np.abs(X) + 1e-3) + np.radians(5.0) * rng.standard_normal((n, n))
    mat_id = np.where(inside, 1, 0).astype(np.uint8)
    orient = f32(np.where(inside, theta, 0.0))
    if n_src == 1:
        sources = [(n // 2, 0)]
    else:
        step = n // n_src
        sources = [(step * k + step // 2, 0) for k in range(n_src)]
    receivers = []
    if n_rec:
        step = n // n_rec
        receivers = [(step * k + step // 2, n - 1) for k in range(n_rec)]
    return Medium(n, n, h, [PARENT_STEEL, TI_STEEL], mat_id, orient, sources, receivers,
                  "weld%d" % n)


def weld_multi():
    """The 512x512 weld with 64 top sources (8k + 4, 0) and 64 bottom receivers."""
    return weld(512, 0.1e-3, 0, n_src=64, n_rec=64)


def bilinear_controls(nc, seed, lo_deg=-45.0, hi_deg=45.0):
    """nc x nc control orientations (radians), uniform in [lo, hi] degrees."""
    rng = np.random.default_rng(seed)
    return np.radians(rng.uniform(lo_deg, hi_deg, size=(nc, nc)))


def bilinear_weights(n, nc):
    """Interpolation matrix W [n][nc] of a 1-D linear interpolant whose nc control points
    span the n nodes end to end (node k sits at control coordinate k (nc-1)/(n-1))."""
    W = np.zeros((n, nc))
    for k in range(n):
        u = k * (nc - 1) / (n - 1)
        c0 = min(int(math.floor(u)), nc - 2)
        f = u - c0
        W[k, c0] += 1.0 - f
        W[k, c0 + 1] += f
    return W


def adjoint_grid(seed=1, n=256, nc=32, h=0.2e-3, n_src=32, n_rec=32):
    """256x256 TI grid, orientation bilinear from an nc x nc control grid."""
    ctrl = bilinear_controls(nc, seed)
    Wz = bilinear_weights(n, nc)
    Wx = bilinear_weights(n, nc)
    orient = f32(Wz @ ctrl @ Wx.T)
    step_s = n // n_src
    step_r = n // n_rec
    sources = [(step_s * k + step_s // 2, 0) for k in range(n_src)]
    receivers = [(step_r * k + step_r // 2, n - 1) for k in range(n_rec)]
    m = Medium(n, n, h, [TI_STEEL], np.zeros((n, n), np.uint8), orient, sources, receivers,
               "adjoint%d" % n)
    m.controls = ctrl
    return m


def batch_media(n_media=128, seed=3, lo=256, hi=1024, nc=32, h=0.1e-3, n_src=32, n_rec=32):
    """Uneven batch: square sides uniform in {lo..hi}; orientation as adjoint_grid."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=n_media)
    out = []
    for b, n in enumerate(sides):
        n = int(n)
        ctrl = bilinear_controls(nc, 1000 + b)
        W = bilinear_weights(n, nc)
        orient = f32(W @ ctrl @ W.T)
        sources = [(int(round((k + 0.5) * n / n_src)), 0) for k in range(n_src)]
        receivers = [(int(round((k + 0.5) * n / n_rec)), n - 1) for k in range(n_rec)]
        sources = [(min(s[0], n - 1), s[1]) for s in sources]
        receivers = [(min(r[0], n - 1), r[1]) for r in receivers]
        m = Medium(n, n, h, [TI_STEEL], np.zeros((n, n), np.uint8), orient, sources, receivers,
                   "batch%d" % b)
        m.controls = ctrl
        out.append(m)
    return out


def random_medium(nx, nz, h, seed, n_mats=2, smooth=True):
    """Small random heterogeneous medium for parity tests: a few materials in blocks and
    a smooth or rough orientation field."""
    rng = np.random.default_rng(seed)
    mats = [TI_STEEL, PARENT_STEEL, CUBIC_STEEL][:n_mats]
    bx = max(nx // 4, 1)
    bz = max(nz // 4, 1)
    coarse = rng.integers(0, n_mats, size=((nz + bz - 1) // bz, (nx + bx - 1) // bx))
    mat_id = np.kron(coarse, np.ones((bz, bx), dtype=np.int64))[:nz, :nx].astype(np.uint8)
    if smooth:
        ctrl = rng.uniform(-math.pi / 2, math.pi / 2, size=(6, 6))
        orient = bilinear_weights(nz, 6) @ ctrl @ bilinear_weights(nx, 6).T
    else:
        orient = rng.uniform(-math.pi, math.pi, size=(nz, nx))
    src = (int(rng.integers(0, nx)), int(rng.integers(0, nz)))
    return Medium(nx, nz, h, mats, mat_id, f32(orient), [src], [], "random%d" % seed)
