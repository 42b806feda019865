"""The allocation-free forward entry point (ali_solve_traveltime_noalloc) against the
ordinary one, through the C ABI.

Both run the same kernels on the same inputs, so the fields must be bitwise equal; the
fixed point is unique, and the scratch buffers only change where the kernels keep their
working state.  Two calls in a row, the second on a smaller medium with fewer sources
(the static array keeps the first call's contents, so this checks that every call clears
what must start at zero); the float32 and float64 arithmetic modes; a solve larger than
the static array is refused before any device work.
"""

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


def _case(m, sources):
    import torch
    return m, torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(m.orient).float().cuda(), sources


@pytest.mark.parametrize("arith", ["mixed", "f32", "f64"])
def test_noalloc_equals_solve(solver, arith):
    import torch
    big = sm.random_medium(120, 96, 0.2e-3, seed=11, n_mats=3)
    small = sm.random_medium(40, 33, 0.2e-3, seed=12, n_mats=2)
    cases = [_case(big, [big.sources[0], (0, 0), (119, 95), (60, 2)]),
             _case(small, [(5, 30), small.sources[0]])]
    for m, mid, ori, srcs in cases:
        print("noalloc:", arith, m.nx, "x", m.nz, len(srcs), "sources", flush=True)
        ref, st0 = solver.solve(m.h, m.mats, mid, ori, srcs, arith=arith)
        out = torch.full_like(ref, -1.0)
        got, st1 = solver.solve(m.h, m.mats, mid, ori, srcs, arith=arith, out=out, noalloc=True)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert st0["converged"] == 1 and st1["converged"] == 1
        assert st1["node_updates"] > 0
        assert torch.equal(ref, got)


def test_noalloc_refuses_oversize(solver):
    import torch
    from paper_2302_10988_amd import AliError, _lib
    n = 1024
    mid = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    ori = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    out = torch.zeros((8, n, n), dtype=torch.float32, device="cuda")
    srcs = [(k * 100, 0) for k in range(8)]
    with pytest.raises(AliError) as e:
        solver.solve(1e-4, [sm.TI_STEEL], mid, ori, srcs, out=out, noalloc=True)
    assert e.value.status == -1 and "bytes of device scratch" in str(e.value)
    # nothing was written
    assert int(torch.count_nonzero(out).item()) == 0
    # the handle still works for the ordinary entry point afterwards
    m = sm.random_medium(40, 33, 0.2e-3, seed=12, n_mats=2)
    T, st = solver.solve(m.h, m.mats, torch.from_numpy(m.mat_id).cuda(),
                         torch.from_numpy(m.orient).float().cuda(), [m.sources[0]], noalloc=True)
    assert st["converged"] == 1
    assert _lib.load().ali_solve_traveltime_noalloc is not None
