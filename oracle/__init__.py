"""FP64 CPU oracle for the ALI-FMM travel-time method (arXiv 2302.10988).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU product path never does.  The C sources
here share no code with the HIP kernels.

Every function follows the paper section cited in its docstring.  Inputs are numpy
arrays; orientations are symmetry-axis angles in radians (from +x toward +z), materials
are dicts/tuples (c11, c13, c33, c55, c44, c66, rho) in Pa and kg/m^3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["velocity.c", "fmm.c", "dijkstra.c", "rays.c", "adjoint.c", "nested.c"]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class Material(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("c11", "c13", "c33", "c55", "c44", "c66", "rho")] + \
               [("wave", ctypes.c_int32), ("vtab", ctypes.c_int32), ("grule", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


WAVE_QP, WAVE_SH = 0, 1
GROUP_EXACT, GROUP_PAPER = 0, 1


def as_sh(mats):
    """The same materials for the SH wave (every solver then uses the SH speeds)."""
    return [dict(m, wave=WAVE_SH) for m in mats]


def as_table(mats):
    """The same materials with the paper's velocity table (speeds at whole degrees,
    linearly interpolated) in place of the run-time Christoffel speeds."""
    return [dict(m, vtab=1) for m in mats]


def with_paper_group(mats):
    """The same materials with the group speed of Section 3.2's run-time inversion (the
    phase angle whose polarisation points along the group direction) for every straight
    ray: a second reading of the paper's group speed, used only to test which rule the
    printed errors of Table 3 follow."""
    return [dict(m, grule=GROUP_PAPER) for m in mats]


VAR_MIN_UPDATE, VAR_UNIT_SQUARES_FIRST, VAR_TRIANGLE_LITERAL, VAR_NO_CAUSALITY = 1, 2, 4, 8


def set_reading_variant(v):
    """Switch this thread's oracle calls to alternative readings (VAR_* bits; 0 = the
    oracle's own readings).  Only for measuring which readings reproduce Table 3."""
    _load().or_set_reading_variant(int(v))


def qp_group_speed_paper(mat, phi):
    """Section 3.2's approximate qP group speed along group angle phi (from the c22 axis)."""
    return _load().or_qp_group_speed_paper(_mat_array([mat]), float(phi))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    hdr = os.path.join(_HERE, "ali_oracle.h")
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(p) for p in srcs + [hdr])
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    D, I, I64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
    P = ctypes.c_void_p
    M = ctypes.POINTER(Material)
    lib.or_qp_phase_speed.argtypes = [M, D]
    lib.or_qp_phase_speed.restype = D
    lib.or_qp_group_from_phase.argtypes = [M, D, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.or_qp_group_speed.argtypes = [M, D]
    lib.or_qp_group_speed.restype = D
    lib.or_set_reading_variant.argtypes = [I]
    lib.or_set_reading_variant.restype = None
    lib.or_qp_group_speed_paper.argtypes = [M, D]
    lib.or_qp_group_speed_paper.restype = D
    lib.or_qp_group_speed_support.argtypes = [M, D]
    lib.or_qp_group_speed_support.restype = D
    lib.or_stencil_offsets.argtypes = [I, ctypes.POINTER(I)]
    lib.or_stencil_estimate.argtypes = [M, D, D, ctypes.POINTER(I), D, D, D]
    lib.or_stencil_estimate.restype = D
    lib.or_phi_d.argtypes = [I, I, D, M, P, P, P, P, I, I, ctypes.POINTER(I)]
    lib.or_phi_d.restype = D
    lib.or_source_box.argtypes = [I, I, D, M, P, P, I, I, I, P, P]
    lib.or_solve_fmm.argtypes = [I, I, D, M, I, P, P, I, I, I, P, P, P]
    lib.or_solve_fmm.restype = I64
    lib.or_last_phi_evals.argtypes = []
    lib.or_last_phi_evals.restype = I64
    lib.or_localfmm.argtypes = [I, I, D, M, P, P, P, I, I, ctypes.POINTER(I)]
    lib.or_localfmm.restype = D
    lib.or_sweep_solve.argtypes = [I, I, D, M, I, P, P, I, I, I, I, P]
    lib.or_sweep_solve.restype = I
    lib.or_dijkstra_dense.argtypes = [I, I, D, M, P, P, I, I, D, P]
    lib.or_segment_time.argtypes = [I, I, D, M, P, P, D, D, D, D]
    lib.or_segment_time.restype = D
    lib.or_trace_ray.argtypes = [I, I, D, M, P, P, P, I, I, I, I, I, I, I, P, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.or_trace_ray.restype = I
    lib.or_trace_ray_family.argtypes = [I, I, D, M, P, P, P, I, I, I, I, I, I, I, I, P, ctypes.POINTER(I),
                                        ctypes.POINTER(D)]
    lib.or_trace_ray_family.restype = I
    lib.or_adjoint.argtypes = [I, I, D, M, I, P, P, I, I, I, P, P, P, P]
    lib.or_adjoint.restype = I
    lib.or_qp_phase_speed_deriv.argtypes = [M, D]
    lib.or_qp_phase_speed_deriv.restype = D
    lib.or_qp_group_speed_deriv.argtypes = [M, D]
    lib.or_qp_group_speed_deriv.restype = D
    lib.or_stencil_partials.argtypes = [M, D, D, ctypes.POINTER(I), D, D, D] + [ctypes.POINTER(D)] * 4 + [P]
    lib.or_qp_phase_speed_dA.argtypes = [M, D, ctypes.POINTER(D)]
    for name in ("or_sh_phase_speed", "or_sh_phase_speed_deriv", "or_sh_group_speed", "or_sh_group_speed_deriv",
                 "or_phase_speed", "or_phase_speed_deriv", "or_group_speed", "or_group_speed_deriv",
                 "or_group_speed_support"):
        getattr(lib, name).argtypes = [M, D]
        getattr(lib, name).restype = D
    lib.or_qp_group_speed_dA.argtypes = [M, D, ctypes.POINTER(D)]
    lib.or_field_choices.argtypes = [I, I, D, M, P, P, P, P, P]
    lib.or_fmm_seeded.argtypes = [I, I, D, M, I, P, P, P, P, I, I, I, P, ctypes.POINTER(D)]
    lib.or_fmm_seeded.restype = I64
    lib.or_solve_refined.argtypes = [I, I, D, M, I, P, P, I, I, I, ctypes.POINTER(I), ctypes.POINTER(I), D, P]
    lib.or_solve_refined.restype = I
    lib.or_frozen_field.argtypes = [I, I, D, M, P, P, I, I, I, P, P, ctypes.c_int64, P]
    _lib = lib
    return lib


# ---------------------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------------------
def _mat_array(mats):
    mats = list(mats)
    arr = (Material * len(mats))()
    for k, m in enumerate(mats):
        if isinstance(m, dict):
            vals = [m[n] for n in ("c11", "c13", "c33", "c55", "c44", "c66", "rho")]
            wave = int(m.get("wave", WAVE_QP))
            vtab = int(m.get("vtab", 0))
            grule = int(m.get("grule", GROUP_EXACT))
        else:
            vals = list(m)[:7]
            wave = int(list(m)[7]) if len(list(m)) > 7 else WAVE_QP
            vtab = int(list(m)[8]) if len(list(m)) > 8 else 0
            grule = GROUP_EXACT
        for n, v in zip(("c11", "c13", "c33", "c55", "c44", "c66", "rho"), vals):
            setattr(arr[k], n, float(v))
        arr[k].wave = wave
        arr[k].vtab = vtab
        arr[k].grule = grule
    return arr


def _medium(mat_id, orient):
    mat_id = np.ascontiguousarray(mat_id, dtype=np.uint8)
    orient = np.ascontiguousarray(orient, dtype=np.float64)
    assert mat_id.shape == orient.shape and mat_id.ndim == 2
    return mat_id, orient


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------------------
# Section 3: velocities
# ---------------------------------------------------------------------------------------
def qp_phase_speed(mat, th_p):
    """qP phase speed at phase angle th_p (rad, from the c22 axis); Section 3.2."""
    lib = _load()
    return lib.or_qp_phase_speed(_mat_array([mat]), float(th_p))


def qp_group_from_phase(mat, th_p):
    """(group angle, group speed) for phase angle th_p; Section 3.1 group velocity."""
    lib = _load()
    ga, gs = ctypes.c_double(), ctypes.c_double()
    lib.or_qp_group_from_phase(_mat_array([mat]), float(th_p), ctypes.byref(ga), ctypes.byref(gs))
    return ga.value, gs.value


def qp_group_speed(mat, phi):
    """qP group speed along group angle phi (rad, from the c22 axis); Section 3.2."""
    return _load().or_qp_group_speed(_mat_array([mat]), float(phi))


def phase_speed(mat, th_p):
    """Phase speed of the material's wave (qP, or SH for a material from as_sh)."""
    return _load().or_phase_speed(_mat_array([mat]), float(th_p))


def group_speed(mat, phi):
    """Group speed of the material's wave along group angle phi (from the c22 axis)."""
    return _load().or_group_speed(_mat_array([mat]), float(phi))


def group_speed_support(mat, phi):
    """Group speed of the material's wave by the support-function route."""
    return _load().or_group_speed_support(_mat_array([mat]), float(phi))


def phase_speed_deriv(mat, th_p):
    return _load().or_phase_speed_deriv(_mat_array([mat]), float(th_p))


def group_speed_deriv(mat, phi):
    return _load().or_group_speed_deriv(_mat_array([mat]), float(phi))


def qp_group_speed_support(mat, phi):
    """Group speed by the slowness-curve support function (independent route)."""
    return _load().or_qp_group_speed_support(_mat_array([mat]), float(phi))


# ---------------------------------------------------------------------------------------
# Section 4: stencils and the update
# ---------------------------------------------------------------------------------------
def stencil_offsets(s):
    """(di, dj) of A, B, C for stencil s = 0..31 (Tables 1-2, corrected)."""
    out = (ctypes.c_int * 6)()
    _load().or_stencil_offsets(int(s), out)
    return [(out[0], out[1]), (out[2], out[3]), (out[4], out[5])]


def stencil_estimate(mat, theta_ax, h, offsets, ta, tb, tc):
    """Section 4.2 estimate tau_B + |FD| / v(theta') for one stencil."""
    off = (ctypes.c_int * 6)(*[int(v) for p in offsets for v in p])
    return _load().or_stencil_estimate(_mat_array([mat]), float(theta_ax), float(h), off,
                                       float(ta), float(tb), float(tc))


def phi_d(h, mats, mat_id, orient, T, known, i, j):
    """Section 4.3 choice Phi_D(K); returns (value, choice)."""
    mat_id, orient = _medium(mat_id, orient)
    T = np.ascontiguousarray(T, dtype=np.float64)
    known = np.ascontiguousarray(known, dtype=np.uint8)
    nz, nx = mat_id.shape
    ch = ctypes.c_int()
    v = _load().or_phi_d(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient),
                         _ptr(T), _ptr(known), int(i), int(j), ctypes.byref(ch))
    return v, ch.value


def source_box(h, mats, mat_id, orient, src, R):
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.full((nz, nx), np.inf)
    fixed = np.zeros((nz, nx), np.uint8)
    _load().or_source_box(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient),
                          int(src[0]), int(src[1]), int(R), _ptr(T), _ptr(fixed))
    return T, fixed


def solve_fmm(h, mats, mat_id, orient, src, R=2, return_pops=False):
    """Heap Fast Marching with the ALI update (Section 2, Section 4).  src = (i, j)."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.empty((nz, nx))
    pops = np.empty(nx * nz, np.int64)
    pvals = np.empty(nx * nz)
    n = _load().or_solve_fmm(nx, nz, float(h), _mat_array(mats), len(list(mats)), _ptr(mat_id),
                             _ptr(orient), int(src[0]), int(src[1]), int(R), _ptr(T),
                             _ptr(pops), _ptr(pvals))
    if n < 0:
        raise ValueError("oracle: invalid input")
    if return_pops:
        return T, pops[:n], pvals[:n]
    return T


def solve_fmm_counted(h, mats, mat_id, orient, src, R=2):
    """solve_fmm plus the number of Phi_D evaluations the heap driver made."""
    T = solve_fmm(h, mats, mat_id, orient, src, R)
    return T, int(_load().or_last_phi_evals())


def localfmm(h, mats, mat_id, orient, T, i, j):
    """The local operator at node (i, j) evaluated on field T; returns (value, choice)."""
    mat_id, orient = _medium(mat_id, orient)
    T = np.ascontiguousarray(T, dtype=np.float64)
    nz, nx = mat_id.shape
    ch = ctypes.c_int()
    v = _load().or_localfmm(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient),
                            _ptr(T), int(i), int(j), ctypes.byref(ch))
    return v, ch.value


def sweep_solve(h, mats, mat_id, orient, src, R=2, max_sweeps=1000):
    """Gauss-Seidel sweeps of the local operator to a bitwise fixed point."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.empty((nz, nx))
    n = _load().or_sweep_solve(nx, nz, float(h), _mat_array(mats), len(list(mats)), _ptr(mat_id),
                               _ptr(orient), int(src[0]), int(src[1]), int(R), int(max_sweeps), _ptr(T))
    return T, n


def dijkstra_dense(h, mats, mat_id, orient, src, rad):
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.empty((nz, nx))
    _load().or_dijkstra_dense(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient),
                              int(src[0]), int(src[1]), float(rad), _ptr(T))
    return T


def segment_time(h, mats, mat_id, orient, p0, p1):
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    return _load().or_segment_time(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient),
                                   float(p0[0]), float(p0[1]), float(p1[0]), float(p1[1]))


# ---------------------------------------------------------------------------------------
# Section 5.1: ray tracing
# ---------------------------------------------------------------------------------------
def trace_ray(h, mats, mat_id, orient, T, src, start, window=4, sub=8, max_pts=4096, family=-1):
    """Ray from node `start` to the source `src` of field T; family -1 changes the plane
    family along the ray, 0..3 fixes it (x = k, z = k, x + z = k, x - z = k).  Returns
    (points [n, 2] in grid units (x, z), integrated time, reached flag)."""
    mat_id, orient = _medium(mat_id, orient)
    T = np.ascontiguousarray(T, dtype=np.float64)
    nz, nx = mat_id.shape
    pts = np.zeros((max_pts, 2))
    n = ctypes.c_int()
    t = ctypes.c_double()
    st = _load().or_trace_ray_family(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient), _ptr(T),
                                     int(src[0]), int(src[1]), int(start[0]), int(start[1]), int(family),
                                     int(window), int(sub), int(max_pts), _ptr(pts), ctypes.byref(n),
                                     ctypes.byref(t))
    return pts[: n.value].copy(), t.value, st == 0


def trace_ray_fastest_fixed(h, mats, mat_id, orient, T, src, start, window=4, sub=8, max_pts=4096):
    """The fastest of the four fixed-family rays (the first family wins a tie).  Returns
    (points, time, reached, family)."""
    best = None
    for f in range(4):
        pts, t, ok = trace_ray(h, mats, mat_id, orient, T, src, start, window, sub, max_pts, f)
        if ok and (best is None or t < best[1]):
            best = (pts, t, ok, f)
    return best if best is not None else (np.zeros((0, 2)), float("inf"), False, -1)


# ---------------------------------------------------------------------------------------
# gradient with respect to orientation
# ---------------------------------------------------------------------------------------
def qp_phase_speed_deriv(mat, th_p):
    return _load().or_qp_phase_speed_deriv(_mat_array([mat]), float(th_p))


def qp_group_speed_deriv(mat, phi):
    return _load().or_qp_group_speed_deriv(_mat_array([mat]), float(phi))


def qp_phase_speed_dA(mat, th_p):
    """d v / d (A11, A13, A33, A55) of the qP phase speed, A = C / rho."""
    out = (ctypes.c_double * 4)()
    _load().or_qp_phase_speed_dA(_mat_array([mat]), float(th_p), out)
    return np.array(out[:])


def qp_group_speed_dA(mat, phi):
    """d V / d (A11, A13, A33, A55) of the qP group speed at fixed group angle."""
    out = (ctypes.c_double * 4)()
    _load().or_qp_group_speed_dA(_mat_array([mat]), float(phi), out)
    return np.array(out[:])


def stencil_partials(mat, theta_ax, h, offsets, ta, tb, tc, with_A=False):
    """(dU/dta, dU/dtb, dU/dtc, dU/dtheta), plus dU/dA [4] when with_A."""
    off = (ctypes.c_int * 6)(*[int(v) for p in offsets for v in p])
    out = [ctypes.c_double() for _ in range(4)]
    dA = np.zeros(4)
    _load().or_stencil_partials(_mat_array([mat]), float(theta_ax), float(h), off, float(ta), float(tb),
                                float(tc), *[ctypes.byref(o) for o in out], _ptr(dA))
    res = tuple(o.value for o in out)
    return res + (dA,) if with_A else res


def adjoint(h, mats, mat_id, orient, src, g, R=2, with_A=False):
    """(T, dL/dtheta) for one source given g = dL/dT [nz, nx]; with_A adds dL/dA
    [nz, nx, 4] (A11, A13, A33, A55 of every node, A = C / rho)."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    g = np.ascontiguousarray(g, dtype=np.float64)
    T = np.empty((nz, nx))
    dth = np.empty((nz, nx))
    dA = np.empty((nz, nx, 4)) if with_A else None
    st = _load().or_adjoint(nx, nz, float(h), _mat_array(mats), len(list(mats)), _ptr(mat_id), _ptr(orient),
                            int(src[0]), int(src[1]), int(R), _ptr(g), _ptr(T), _ptr(dth),
                            _ptr(dA) if with_A else None)
    if st != 0:
        raise ValueError("oracle: invalid input")
    return (T, dth, dA) if with_A else (T, dth)


def frozen_setup(h, mats, mat_id, orient, src, R=2):
    """Pop order and choices of the solution (for frozen-choice re-evaluation)."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T, pops, _ = solve_fmm(h, mats, mat_id, orient, src, R, return_pops=True)
    _, fixed = source_box(h, mats, mat_id, orient, src, R)
    choice = np.empty((nz, nx), np.int32)
    _load().or_field_choices(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient), _ptr(T),
                             _ptr(np.ascontiguousarray(fixed)), _ptr(choice))
    return T, np.ascontiguousarray(pops), choice


def frozen_field(h, mats, mat_id, orient, src, choice, pops, R=2):
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.empty((nz, nx))
    _load().or_frozen_field(nx, nz, float(h), _mat_array(mats), _ptr(mat_id), _ptr(orient), int(src[0]),
                            int(src[1]), int(R), _ptr(np.ascontiguousarray(choice, dtype=np.int32)),
                            _ptr(pops), len(pops), _ptr(T))
    return T


# ---------------------------------------------------------------------------------------
# Section 4.4: nested fine grids around the source; whole-grid refinement
# ---------------------------------------------------------------------------------------
PAPER_LEVELS = ((27, 1), (9, 6), (3, 13))


def fmm_seeded(h, mats, mat_id, orient, fixed, T0, centre, stop_r=-1):
    """Heap march from the nodes marked in fixed (times T0).  Returns (T, known, t_stop)."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
    T = np.ascontiguousarray(T0, dtype=np.float64).copy()
    known = np.zeros((nz, nx), np.uint8)
    ts = ctypes.c_double()
    n = _load().or_fmm_seeded(nx, nz, float(h), _mat_array(mats), len(list(mats)), _ptr(mat_id), _ptr(orient),
                              _ptr(fixed), _ptr(T), int(centre[0]), int(centre[1]), int(stop_r), _ptr(known),
                              ctypes.byref(ts))
    if n < 0:
        raise ValueError("oracle: invalid input")
    return T, known.astype(bool), ts.value


def solve_refined(h, mats, mat_id, orient, src, levels=PAPER_LEVELS, vor_half=0.5):
    """Travel times with nested fine grids around the source: levels = ((density, radius),
    ...) from the finest; straight rays within vor_half cells of the source (Section 4.4)."""
    mat_id, orient = _medium(mat_id, orient)
    nz, nx = mat_id.shape
    T = np.empty((nz, nx))
    dens = (ctypes.c_int * max(len(levels), 1))(*[int(d) for d, _ in levels])
    rads = (ctypes.c_int * max(len(levels), 1))(*[int(r) for _, r in levels])
    st = _load().or_solve_refined(nx, nz, float(h), _mat_array(mats), len(list(mats)), _ptr(mat_id), _ptr(orient),
                                  int(src[0]), int(src[1]), len(levels), dens, rads, float(vor_half), _ptr(T))
    if st != 0:
        raise ValueError("oracle: invalid input")
    return T


def refine_medium(mat_id, orient, s):
    """The medium on an s-times finer grid (s odd): every node takes the material and
    orientation of the nearest original node."""
    assert s >= 1 and s % 2 == 1
    nz, nx = np.shape(mat_id)
    jz = (np.arange((nz - 1) * s + 1) + s // 2) // s
    ix = (np.arange((nx - 1) * s + 1) + s // 2) // s
    return (np.ascontiguousarray(np.asarray(mat_id)[np.ix_(jz, ix)]),
            np.ascontiguousarray(np.asarray(orient)[np.ix_(jz, ix)]))
