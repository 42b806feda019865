"""The persistent relaxation (ali_options.persistent: every pass of a forward solve in one
cooperative launch with grid barriers) against the pass-by-pass launches.

The fixed point is unique and both run the same scheduler and tile visits, so the fields
must be bitwise equal: one medium with several sources, a batch of uneven media, the
nested source grids (seeded fields), the velocity table, and the forward inside a misfit
gradient (whose re-derived choices must all reproduce the field).  A barrier wait limit of
zero makes every work-group give up at its first barrier: the call reports a device
error, every kernel exits normally, and the handle keeps working.  Visits of several
tiles at once (ali_options.visit_tiles) give the same fields for every visit size, and the
autotuner keeps its choice per size bucket.
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


def _dev(m):
    import torch
    return torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(m.orient).float().cuda()


@pytest.mark.parametrize("arith", ["mixed", "f64", "f32"])
def test_persistent_single_medium(solver, arith):
    import torch
    m = sm.weld(n=192, h=0.25e-3, seed=1, n_src=6, n_rec=6)
    mid, ori = _dev(m)
    print("persistent: weld 192, 6 sources,", arith, flush=True)
    a, sa = solver.solve(m.h, m.mats, mid, ori, m.sources, arith=arith)
    b, sb = solver.solve(m.h, m.mats, mid, ori, m.sources, arith=arith, persistent=1)
    assert sa["converged"] == 1 and sb["converged"] == 1
    assert sb["outer_iters"] == sa["outer_iters"]
    assert torch.equal(a, b)


def test_persistent_batch_and_modes(solver):
    import torch
    from paper_2302_10988_amd import Batch
    media = sm.batch_media(n_media=12, seed=3, lo=64, hi=200, nc=8, h=0.1e-3, n_src=3, n_rec=3)
    b = Batch(media)
    print("persistent: batch of", b.n_media, "media", flush=True)
    Ta, _ = solver.solve_batch(b)
    Tb, st = solver.solve_batch(b, persistent=1)
    assert st["converged"] == 1 and torch.equal(Ta, Tb)
    m = sm.random_medium(70, 55, 0.2e-3, seed=9, n_mats=3)
    mid, ori = _dev(m)
    srcs = [m.sources[0], (3, 50)]
    print("persistent: nested source grids and velocity table", flush=True)
    a, _ = solver.solve_refined(m.h, m.mats, mid, ori, srcs)
    c, st = solver.solve_refined(m.h, m.mats, mid, ori, srcs, persistent=1)
    assert st["converged"] == 1 and torch.equal(a, c)
    a, _ = solver.solve(m.h, m.mats, mid, ori, srcs, velocity="table")
    c, _ = solver.solve(m.h, m.mats, mid, ori, srcs, velocity="table", persistent=1)
    assert torch.equal(a, c)


def test_persistent_inside_gradient(solver):
    import torch
    m = sm.adjoint_grid(seed=2, n_src=8, n_rec=8)
    mid, ori = _dev(m)
    obs = torch.full((8, 8), 2e-6, device="cuda")
    print("persistent: misfit gradient", flush=True)
    l0, t0, g0, s0 = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs)
    l1, t1, g1, s1 = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs, persistent=1)
    assert s1["forward"]["converged"] == 1 and s1["choice_mismatches"] == 0
    assert torch.equal(t0, t1) and torch.equal(g0, g1)


def test_persistent_barrier_timeout_is_an_error(solver):
    import torch
    from paper_2302_10988_amd import AliError
    m = sm.random_medium(70, 55, 0.2e-3, seed=9, n_mats=3)
    mid, ori = _dev(m)
    print("persistent: zero barrier wait", flush=True)
    solver.set_barrier_timeout(0.0)
    try:
        with pytest.raises(AliError) as e:
            solver.solve(m.h, m.mats, mid, ori, m.sources, persistent=1, max_sweeps=200)
        assert e.value.status == -3 and "barrier" in str(e.value)
    finally:
        solver.set_barrier_timeout(5.0)
    a, _ = solver.solve(m.h, m.mats, mid, ori, m.sources)
    b, st = solver.solve(m.h, m.mats, mid, ori, m.sources, persistent=1)
    assert st["converged"] == 1 and torch.equal(a, b)


def test_visit_sizes_and_tuned_schedule(solver):
    # a batch whose passes list more tiles than there are resident waves, so that visits
    # take several tiles: the fields are the same bit for bit for every visit size, with
    # and without the persistent launch (a race in the shared chunks would show here)
    import torch
    from paper_2302_10988_amd import Batch
    media = sm.batch_media(n_media=48, seed=4, lo=240, hi=280, nc=8, h=0.1e-3, n_src=8, n_rec=4)
    b = Batch(media)
    print("visit sizes: %d fields, %d node-fields" % (b.n_fields, b.field_nodes), flush=True)
    ref, st0 = solver.solve_batch(b, visit_tiles=1)
    assert st0["converged"] == 1
    # more tiles than resident waves in the largest passes
    assert st0["tile_visits"] / st0["outer_iters"] > 4096
    for vt in (2, 3, 4):
        for pers in (0, 1):
            T, st = solver.solve_batch(b, visit_tiles=vt, persistent=pers)
            assert st["converged"] == 1 and st["outer_iters"] == st0["outer_iters"]
            assert torch.equal(ref, T), (vt, pers)
    # the autotuner's choice is kept by the handle for batches of the same size bucket
    import time
    t0 = time.perf_counter()
    c1, ms1, cached1 = solver.autotune_batch(b)
    t1 = time.perf_counter()
    c2, ms2, cached2 = solver.autotune_batch(b)
    t2 = time.perf_counter()
    print("autotune: first %.2f s, second %.4f s, choice %s" % (t1 - t0, t2 - t1, {k: c1[k] for k in
                                                                                  ("band_cells", "inner_sweeps",
                                                                                   "visit_tiles", "persistent")}))
    assert ms1 == ms2 and all(c1[k] == c2[k] for k in ("band_cells", "inner_sweeps", "visit_tiles", "persistent"))
    assert t2 - t1 < 0.1 * (t1 - t0)
