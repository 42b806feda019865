"""GPU parity: the HIP relaxation (through the C ABI) against the FP64 heap oracle.

Tolerances:
  * f64 entry point: max relative error 1e-12 (same discrete fixed point; the GPU
    evaluates the estimate with a different but algebraically equal formula, so values
    agree to rounding and every stencil decision agrees).
  * float32 entry point, default mixed arithmetic (float64 times and decisions, float32
    wavefront math, float32 output): max relative error 1e-4 over all non-source nodes
    (the contract; observed values are a few 1e-7).
  * float32 entry point, pure float32 arithmetic: 1e-4 on small grids only.  On the
    512x512 weld, float32 rounding of stored times turns near-equal stencil scores into
    exact ties and some fields exceed 1e-4 (measured, reported, not asserted).
"""
import math

import numpy as np
import pytest

import synthmedia as sm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    from paper_2302_10988_amd import Solver
    assert torch.cuda.is_available()
    return Solver(0)


def to_dev(m, precision):
    import torch
    dt = torch.float32 if precision == "f32" else torch.float64
    mid = torch.from_numpy(np.ascontiguousarray(m.mat_id)).cuda()
    ori = torch.from_numpy(np.ascontiguousarray(m.orient)).to(dt).cuda()
    return mid, ori


def gpu_solve(solver, m, sources=None, precision="f32", **kw):
    mid, ori = to_dev(m, precision)
    print("gpu solve:", m.name, m.nx, m.nz, precision, kw, flush=True)
    T, st = solver.solve(m.h, m.mats, mid, ori, sources or m.sources, precision=precision, **kw)
    return T.cpu().numpy().astype(np.float64), st


def rel_err(T, Tref):
    mask = Tref > 0
    assert np.array_equal(np.isfinite(T), np.isfinite(Tref))
    fin = mask & np.isfinite(Tref)
    return np.abs(T - Tref)[fin] / Tref[fin]


def oracle(m, src, R=2):
    import oracle as orc
    return orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient, src, R)


CASES_F64 = [
    ("tiny_ti", lambda: sm.tiny_ti()),
    ("random_37x29", lambda: sm.random_medium(37, 29, 0.2e-3, seed=11)),
    ("random_50_rough", lambda: sm.random_medium(50, 50, 0.2e-3, seed=7, smooth=False)),
    ("weld_96", lambda: sm.weld(96, 0.5e-3)),
]


@pytest.mark.parametrize("name,make", CASES_F64, ids=[c[0] for c in CASES_F64])
def test_f64_logic_parity(solver, name, make):
    m = make()
    T, st = gpu_solve(solver, m, precision="f64")
    Tref = oracle(m, m.sources[0])
    r = rel_err(T[0], Tref)
    print(name, "f64 max rel %.3g" % r.max(), st)
    assert st["converged"] == 1
    assert r.max() <= 1e-12


@pytest.mark.parametrize("arith", ["mixed", "f32", "f64"])
@pytest.mark.parametrize("name,make", CASES_F64[:3], ids=[c[0] for c in CASES_F64[:3]])
def test_f32_small(solver, name, make, arith):
    m = make()
    T, st = gpu_solve(solver, m, arith=arith)
    r = rel_err(T[0], oracle(m, m.sources[0]))
    print(name, arith, "max rel %.3g mean %.3g" % (r.max(), r.mean()))
    assert r.max() <= 1e-4


def test_f32_weld512_single_source(solver):
    # the 512x512 V-weld, one top-surface source, FP32 GPU vs FP64 oracle
    m = sm.weld()
    T, st = gpu_solve(solver, m)
    Tref = oracle(m, m.sources[0])
    r = rel_err(T[0], Tref)
    print("weld512 f32 max rel %.3g mean %.3g p99.99 %.3g" % (r.max(), r.mean(), np.quantile(r, 0.9999)), st)
    assert st["converged"] == 1
    assert r.max() <= 1e-4


def test_f32_weld512_64_sources(solver):
    # 64 top sources solved in one batched call; four fields checked node by node
    # against the oracle, every field checked for structure
    m = sm.weld_multi()
    T, st = gpu_solve(solver, m)
    assert T.shape == (64, 512, 512)
    assert st["converged"] == 1
    for k in (0, 10, 31, 63):
        r = rel_err(T[k], oracle(m, m.sources[k]))
        print("weld512 src %d f32 max rel %.3g" % (k, r.max()))
        assert r.max() <= 1e-4
    for k, (i, j) in enumerate(m.sources):
        assert T[k, j, i] == 0.0
        assert np.all(np.isfinite(T[k]))
        assert np.all(T[k] >= 0)


def test_pure_f32_weld_reported(solver):
    # pure float32: measured and reported; the fixed point is still reached
    m = sm.weld_multi()
    T, st = gpu_solve(solver, m, sources=m.sources[31:32], arith="f32")
    r = rel_err(T[0], oracle(m, m.sources[31]))
    print("weld512 src 31 pure f32 max rel %.3g (above 1e-4 expected: score ties)" % r.max())
    assert st["converged"] == 1 and r.max() < 1e-3


def test_schedule_invariance(solver):
    # the fixed point is unique: the number of sweeps per tile visit cannot change a bit
    m = sm.weld(160, 0.3e-3)
    Ta, sa = gpu_solve(solver, m, inner_sweeps=64)
    Tb, sb = gpu_solve(solver, m, inner_sweeps=1)
    Tc, sc = gpu_solve(solver, m, inner_sweeps=7)
    assert np.array_equal(Ta, Tb) and np.array_equal(Ta, Tc)
    assert sb["outer_iters"] > sa["outer_iters"]


def test_graph_cache_bounded_and_exact(solver):
    # in float32 arithmetic the relaxation works in the output buffer itself, so every
    # output buffer is part of a captured batch's signature; 70 solves into fresh buffers
    # (two graphs each) overflow the handle's cache (128 graphs) and must release and
    # recapture without changing a bit, graph replay or not
    import torch
    m = sm.weld(96, 0.3e-3)
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(m.orient).float().cuda()
    srcs = m.sources
    ref, st = solver.solve(m.h, m.mats, mid, ori, srcs, arith="f32", graph=0)
    assert st["outer_iters"] > 32      # long enough for whole captured batches
    keep = []
    for k in range(70):
        out = torch.full((len(srcs), m.nz, m.nx), -1.0, device="cuda")
        keep.append(out)               # distinct live buffers, distinct signatures
        T, _ = solver.solve(m.h, m.mats, mid, ori, srcs, out=out, arith="f32")
        assert torch.equal(T, ref), k
    print("graph cache: 70 solves' captured signatures, all equal to the one-by-one launches", flush=True)


# Exact ties of the discrete solution are resolved by rounding, so two correct
# implementations may choose different stencils there.  Homogeneous cubic media whose
# axis makes the x and z grid directions mirror images (e.g. 33 deg: 33 and 57 deg from
# the cubic axis) give bitwise-equal straight-ray times in exact arithmetic; the edge
# cases below avoid such symmetric set-ups and use the TI medium instead.
EDGE = [
    ("grid_3x3_corner", lambda: sm.homogeneous(3, 3, 1e-3, sm.TI_STEEL, 20.0, (0, 0))),
    ("ragged_17x33_edge", lambda: sm.homogeneous(17, 33, 1e-3, sm.TI_STEEL, 33.0, (16, 5))),
    ("ragged_45x19_random", lambda: sm.random_medium(45, 19, 0.2e-3, seed=21, n_mats=3)),
    ("one_row_tiles_70x5", lambda: sm.random_medium(70, 5, 0.2e-3, seed=22)),
]


@pytest.mark.parametrize("name,make", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("R", [0, 2, 5])
def test_edge_cases_f64(solver, name, make, R):
    m = make()
    T, st = gpu_solve(solver, m, precision="f64", src_box_radius=R)
    r = rel_err(T[0], oracle(m, m.sources[0], R))
    assert r.size == 0 or r.max() <= 1e-12


def test_errors(solver):
    import torch
    from paper_2302_10988_amd import AliError
    m = sm.tiny_ti()
    mid, ori = to_dev(m, "f32")
    with pytest.raises(AliError) as e:
        solver.solve(m.h, m.mats, mid, ori, [(64, 0)])
    assert e.value.status == -1
    bad = dict(sm.TI_STEEL)
    bad["c13"] = 1e13
    with pytest.raises(AliError):
        solver.solve(m.h, [bad], mid, ori, [(3, 3)])
    with pytest.raises(AliError):
        solver.solve(-1.0, m.mats, mid, ori, [(3, 3)])
    o2 = ori.clone()
    o2[5, 5] = float("nan")
    with pytest.raises(AliError) as e:
        solver.solve(m.h, m.mats, mid, o2, [(3, 3)])
    assert e.value.status == -1
    mid2 = mid.clone()
    mid2[1, 1] = 7
    with pytest.raises(AliError) as e:
        solver.solve(m.h, m.mats, mid2, ori, [(3, 3)])
    assert e.value.status == -1
    with pytest.raises(AliError) as e:
        solver.solve(m.h, m.mats, mid, ori, [(32, 32)], max_sweeps=1)
    assert e.value.status == -4
    # the handle still works after errors
    T, st = solver.solve(m.h, m.mats, mid, ori, [(32, 32)])
    assert st["converged"] == 1
