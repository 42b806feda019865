"""Batched forward with nested fine grids around every source (Section 4.4).

Every field of a batch relaxes the same levels as the single-medium call on its own medium
and source (each level's grids take their own medium's materials and orientation), and
the fixed point of every level is unique, so the batch must reproduce
ali_solve_traveltime_refined bit for bit, sources at an edge (clipped level grids)
included; one field per medium is also checked against the FP64 oracle's nested march at
the float32 bar (1e-4 relative).
"""
import ctypes

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


def media():
    out = []
    for k, (nx, nz) in enumerate([(40, 36), (57, 33), (31, 64)]):
        m = sm.random_medium(nx, nz, 0.2e-3, seed=40 + k, n_mats=2 + k % 2)
        rng = np.random.default_rng(100 + k)
        m.sources = [m.sources[0]] + [(int(rng.integers(0, nx)), int(rng.integers(0, nz))) for _ in range(k + 1)]
        if k == 1:
            m.sources.append((0, nz - 1))      # a corner: every level grid is clipped
        out.append(m)
    return out


def _dev(m):
    import torch
    return torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(np.ascontiguousarray(m.orient)).float().cuda()


@pytest.mark.parametrize("levels,half", [(None, 0.5), (((9, 2), (3, 5)), 1.0)])
def test_batch_refined_equals_per_medium(solver, levels, half):
    import torch
    from paper_2302_10988_amd import Batch
    ms = media()
    b = Batch(ms)
    print("batch refined:", len(ms), "media,", b.n_fields, "fields, levels", levels, flush=True)
    T, st = solver.solve_batch_refined(b, levels=levels, start_half_width=half)
    assert st["converged"] == 1 and st["nodes"] == b.field_nodes
    for m, Tb in zip(ms, b.fields(T)):
        mid, ori = _dev(m)
        kw = {} if levels is None else {"levels": levels}
        Tm, _ = solver.solve_refined(m.h, m.mats, mid, ori, m.sources, start_half_width=half, **kw)
        assert torch.equal(Tm, Tb), (m.name, (Tm - Tb).abs().max().item())


def test_batch_refined_vs_oracle(solver, orc):
    from paper_2302_10988_amd import Batch
    ms = media()
    b = Batch(ms)
    T, st = solver.solve_batch_refined(b)
    assert st["converged"] == 1
    for m, Tb in zip(ms, b.fields(T)):
        for k in (0, len(m.sources) - 1):
            ref = orc.solve_refined(m.h, m.mats, m.mat_id, m.orient, m.sources[k])
            got = Tb[k].cpu().numpy().astype(np.float64)
            fin = ref > 0
            rel = np.abs(got - ref)[fin] / ref[fin]
            print("  %s source %s: max rel err %.3g" % (m.name, m.sources[k], rel.max()), flush=True)
            assert np.array_equal(np.isfinite(got), np.isfinite(ref))
            assert got[m.sources[k][1], m.sources[k][0]] == 0.0
            assert rel.max() <= 1e-4


def test_batch_refined_errors(solver):
    import torch
    from paper_2302_10988_amd import Batch, AliError, _lib, _refine, default_options
    ms = media()
    b = Batch(ms)
    out = torch.empty(b.field_nodes, dtype=torch.float32, device="cuda")
    opt = default_options()
    stats = _lib.SolveStats()
    # the s-fold medium is a single-medium option
    ref = _refine(((27, 1), (9, 6), (3, 13)), 0.5, 3)
    st = solver._lib.ali_solve_batch_refined(solver._h, b.media, b.n_media, b.mats, b.n_mats, b.mat_id.data_ptr(),
                                             b.orient.data_ptr(), b.srcs, ctypes.byref(opt), ctypes.byref(ref),
                                             out.data_ptr(), ctypes.byref(stats))
    assert st == _lib.ALI_EUNSUPPORTED
    # densities that do not divide each other are refused before any device work
    with pytest.raises(AliError):
        solver.solve_batch_refined(b, levels=((9, 2), (5, 5)))


def test_batch_refined_node_stiffness(solver):
    # per-node stiffness equal to every node's material: the same fields as the material
    # table (the level grids take the stiffness of their own medium's nearest nodes, and
    # the straight rays that of their source node)
    import torch
    from paper_2302_10988_amd import Batch
    ms = media()
    for m in ms:
        A = np.stack([np.array([x["c11"], x["c13"], x["c33"], x["c55"]]) / x["rho"] for x in m.mats])
        A = A.astype(np.float32)
        # density 1, so the table's C / rho is the float32 value itself
        m.mats = [dict(c11=float(a[0]), c13=float(a[1]), c33=float(a[2]), c55=float(a[3]), c44=float(a[3]),
                       c66=float(a[3]), rho=1.0) for a in A]
        m.nodeA = A[m.mat_id].reshape(-1, 4)
    b = Batch(ms)
    nodeA = torch.from_numpy(np.ascontiguousarray(np.concatenate([m.nodeA for m in ms]))).cuda()
    print("batch refined, per-node stiffness:", len(ms), "media", flush=True)
    Tt, _ = solver.solve_batch_refined(b)
    Tn, st = solver.solve_batch_refined(b, node_A=nodeA)
    assert st["converged"] == 1 and torch.equal(Tt, Tn)


@pytest.mark.parametrize("opt", [{"velocity": "table"}, {"wave": "sh"}])
def test_batch_refined_modes_equal_per_medium(solver, opt):
    # the velocity table (each medium's materials in its own range of the table) and the SH
    # wave reach the level grids of a batch as they reach those of one medium
    import torch
    from paper_2302_10988_amd import Batch
    ms = media()
    b = Batch(ms)
    print("batch refined:", opt, flush=True)
    T, st = solver.solve_batch_refined(b, **opt)
    assert st["converged"] == 1
    for m, Tb in zip(ms, b.fields(T)):
        mid, ori = _dev(m)
        Tm, _ = solver.solve_refined(m.h, m.mats, mid, ori, m.sources, **opt)
        assert torch.equal(Tm, Tb), (m.name, opt, (Tm - Tb).abs().max().item())


def test_batch_refined_f64_equals_per_medium(solver):
    # the float64 entry point through the C ABI: float64 orientation and output
    import torch
    from paper_2302_10988_amd import Batch, _lib, _refine, default_options
    ms = media()
    b = Batch(ms)
    ori64 = b.orient.double().contiguous()
    out = torch.empty(b.field_nodes, dtype=torch.float64, device="cuda")
    opt = default_options()
    stats = _lib.SolveStats()
    ref = _refine(((27, 1), (9, 6), (3, 13)), 0.5, 1)
    print("batch refined f64:", len(ms), "media", flush=True)
    solver._sync_stream()
    st = solver._lib.ali_solve_batch_refined_f64(solver._h, b.media, b.n_media, b.mats, b.n_mats,
                                                 b.mat_id.data_ptr(), ori64.data_ptr(), b.srcs, ctypes.byref(opt),
                                                 ctypes.byref(ref), out.data_ptr(), ctypes.byref(stats))
    torch.cuda.synchronize()
    assert st == 0 and stats.converged == 1
    for m, Tb in zip(ms, b.fields(out)):
        mid, _ = _dev(m)
        ori = torch.from_numpy(np.ascontiguousarray(m.orient)).float().double().cuda()
        Tm, _ = solver.solve_refined(m.h, m.mats, mid, ori, m.sources, precision="f64")
        assert torch.equal(Tm, Tb), (m.name, (Tm - Tb).abs().max().item())
