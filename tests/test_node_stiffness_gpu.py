"""Per-node stiffness (ali_options.d_node_A: A11, A13, A33, A55 of every node in place of
the material table) on the GPU, through the C ABI.

  - the same stiffness given per node and through the table gives the same fields and
    gradients, bit for bit (one medium and a batch);
  - every node its own stiffness (16 x 16, 256 stiffnesses; 48 x 40 drawing from 256):
    float64 fields within 1e-12 of the oracle (which takes one material per stiffness),
    mixed within 1e-4; the orientation and stiffness gradients within 1e-9 of their
    largest entry (all nodes anisotropic, so no mirror ties);
  - the nested source grids and the subgrid take it too (fine nodes take the nearest
    node's): equal to the table path bit for bit, and within 1e-12 of the oracle;
  - ray tracing, SH and the velocity table refuse it; a node that is not positive
    definite, and a tensor of the wrong size, are errors.
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


def _a_of(m):
    return np.array([m["c11"], m["c13"], m["c33"], m["c55"]]) / m["rho"]


def _mat_of(a):
    # density 1, so the table's C / rho is the float32 value itself
    a = [float(v) for v in a]
    return dict(c11=a[0], c13=a[1], c33=a[2], c55=a[3], c44=a[3], c66=a[3], rho=1.0)


def _random_stiffness(rng, n):
    # TI steel with every entry moved by up to 10 %, rounded to float32
    base = _a_of(sm.TI_STEEL)
    return (base[None, :] * rng.uniform(0.9, 1.1, size=(n, 4))).astype(np.float32)


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    fin = np.isfinite(b) & (b > 0)
    return float((np.abs(a - b)[fin] / b[fin]).max())


def test_node_stiffness_equals_the_table(solver):
    import torch
    m = sm.random_medium(96, 80, 0.2e-3, seed=4, n_mats=3)
    A = np.stack([_a_of(x) for x in m.mats]).astype(np.float32)
    mats = [_mat_of(a) for a in A]
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(m.orient).cuda()
    nodeA = torch.from_numpy(np.ascontiguousarray(A[m.mat_id])).cuda()
    sources = [m.sources[0], (0, 0), (95, 79)]
    receivers = [(95, 0), (0, 79), (40, 40)]
    print("per-node stiffness = table: 96 x 80", flush=True)
    for prec, o in (("f64", ori), ("f32", ori.float())):
        Tt, _ = solver.solve(m.h, mats, mid, o, sources, precision=prec)
        Tn, st = solver.solve(m.h, mats, mid, o, sources, precision=prec, node_A=nodeA)
        assert st["converged"] == 1 and torch.equal(Tt, Tn), prec
    g = torch.from_numpy(np.random.default_rng(4).normal(size=(3, 3))).cuda()
    (dt, dAt), _ = solver.adjoint(m.h, mats, mid, ori, sources, receivers, g, precision="f64", stiffness=True)
    (dn, dAn), _ = solver.adjoint(m.h, mats, mid, ori, sources, receivers, g, precision="f64", stiffness=True,
                                  node_A=nodeA)
    assert torch.equal(dt, dn) and torch.equal(dAt, dAn)


@pytest.mark.parametrize("shape,n_stiff,seed", [((16, 16), 256, 1), ((48, 40), 256, 2)])
def test_node_stiffness_vs_oracle(solver, orc, shape, n_stiff, seed):
    import torch
    nx, nz = shape
    rng = np.random.default_rng(seed)
    A = _random_stiffness(rng, n_stiff)
    if nx * nz == n_stiff:
        ids = np.arange(n_stiff, dtype=np.uint8).reshape(nz, nx)
    else:
        ids = rng.integers(0, n_stiff, size=(nz, nx)).astype(np.uint8)
    m = sm.random_medium(nx, nz, 0.2e-3, seed=seed)
    mats_or = [_mat_of(a) for a in A]
    nodeA = torch.from_numpy(np.ascontiguousarray(A[ids])).cuda()
    # the table handed to the library is a single unrelated material: the node values rule
    zeros = torch.zeros((nz, nx), dtype=torch.uint8, device="cuda")
    one = [sm.PARENT_STEEL]
    ori64 = torch.from_numpy(m.orient).cuda()
    sources = [(nx // 2, nz // 2), (0, 0), (nx - 1, 0)]
    receivers = [(nx - 1, nz - 1), (0, nz - 1), (nx // 3, nz - 2)]
    print("per-node stiffness vs oracle: %d x %d, %d stiffnesses" % (nx, nz, n_stiff), flush=True)
    T64, st = solver.solve(m.h, one, zeros, ori64, sources, precision="f64", node_A=nodeA)
    assert st["converged"] == 1
    T32, _ = solver.solve(m.h, one, zeros, ori64.float(), sources, node_A=nodeA)
    for k, src in enumerate(sources):
        ref = orc.solve_fmm(m.h, mats_or, ids, m.orient, src, 2)
        e64, e32 = _rel(T64[k].cpu().numpy(), ref), _rel(T32[k].cpu().numpy(), ref)
        print("  source %s: f64 %.3g, mixed %.3g" % (src, e64, e32), flush=True)
        assert e64 <= 1e-12 and e32 <= 1e-4
    dLdT = rng.normal(size=(len(sources), len(receivers)))
    (dth, dA), st = solver.adjoint(m.h, one, zeros, ori64, sources, receivers, torch.from_numpy(dLdT).cuda(),
                                   precision="f64", stiffness=True, node_A=nodeA)
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    rth, rA = np.zeros((nz, nx)), np.zeros((nz, nx, 4))
    for s, src in enumerate(sources):
        g = np.zeros((nz, nx))
        for r, rec in enumerate(receivers):
            g[rec[1], rec[0]] += dLdT[s, r]
        _, a, b = orc.adjoint(m.h, mats_or, ids, m.orient, src, g, with_A=True)
        rth += a
        rA += b
    eth = np.abs(dth.cpu().numpy() - rth).max() / np.abs(rth).max()
    eA = np.abs(dA.cpu().numpy() - rA).max() / np.abs(rA).max()
    print("  gradients: theta %.3g, A %.3g" % (eth, eA), flush=True)
    assert eth <= 1e-9 and eA <= 1e-9


def test_node_stiffness_batch(solver):
    import torch
    from paper_2302_10988_amd import Batch
    media = [sm.random_medium(30, 26, 0.2e-3, seed=7, n_mats=3), sm.random_medium(41, 33, 0.2e-3, seed=8, n_mats=2)]
    for m in media:
        A = np.stack([_a_of(x) for x in m.mats]).astype(np.float32)
        m.mats = [_mat_of(a) for a in A]
        m.nodeA = A[m.mat_id].reshape(-1, 4)
        m.sources = m.sources + [(0, 0)]
    b = Batch(media)
    nodeA = torch.from_numpy(np.ascontiguousarray(np.concatenate([m.nodeA for m in media]))).cuda()
    print("per-node stiffness: batch of 2", flush=True)
    Tt, _ = solver.solve_batch(b)
    Tn, st = solver.solve_batch(b, node_A=nodeA)
    assert st["converged"] == 1 and torch.equal(Tt, Tn)


def test_node_stiffness_refusals(solver):
    import torch
    from paper_2302_10988_amd import AliError
    m = sm.random_medium(20, 18, 0.2e-3, seed=3)
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(m.orient).float().cuda()
    A = _random_stiffness(np.random.default_rng(0), 20 * 18).reshape(18, 20, 4)
    nodeA = torch.from_numpy(A).cuda()
    T, _ = solver.solve(m.h, m.mats, mid, ori, m.sources, node_A=nodeA)
    for kw in (dict(wave="sh"), dict(velocity="table")):
        with pytest.raises(AliError):
            solver.solve(m.h, m.mats, mid, ori, m.sources, node_A=nodeA, **kw)
    with pytest.raises(AliError):
        solver.trace_rays(m.h, m.mats, mid, ori, T, m.sources, [(19, 17)], node_A=nodeA)
    bad = A.copy()
    bad[5, 7, 3] = -1.0                      # A55 < 0
    with pytest.raises(AliError):
        solver.solve(m.h, m.mats, mid, ori, m.sources, node_A=torch.from_numpy(bad).cuda())
    bad = A.copy()
    bad[2, 3, 1] = 2.0 * np.sqrt(bad[2, 3, 0] * bad[2, 3, 2])   # A13^2 > A11 A33
    with pytest.raises(AliError):
        solver.solve(m.h, m.mats, mid, ori, m.sources, node_A=torch.from_numpy(bad).cuda())
    with pytest.raises(ValueError):
        solver.solve(m.h, m.mats, mid, ori, m.sources, node_A=nodeA[:10])


def test_node_stiffness_nested_grids(solver, orc):
    import torch
    # the same stiffness per node and through the table: equal, with and without a subgrid
    m = sm.random_medium(40, 34, 0.2e-3, seed=6, n_mats=3)
    A = np.stack([_a_of(x) for x in m.mats]).astype(np.float32)
    mats = [_mat_of(a) for a in A]
    mid, ori = torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(m.orient).cuda()
    nodeA = torch.from_numpy(np.ascontiguousarray(A[m.mat_id])).cuda()
    sources = [m.sources[0], (0, 0), (39, 33)]
    print("per-node stiffness: nested grids 40 x 34", flush=True)
    for s in (1, 3):
        Rt, _ = solver.solve_refined(m.h, mats, mid, ori, sources, precision="f64", subgrid=s)
        Rn, st = solver.solve_refined(m.h, mats, mid, ori, sources, precision="f64", subgrid=s, node_A=nodeA)
        assert st["converged"] == 1 and torch.equal(Rt, Rn), s
    # every node its own stiffness: the oracle's nested grids with one material per node
    rng = np.random.default_rng(5)
    A = _random_stiffness(rng, 256)
    ids = np.arange(256, dtype=np.uint8).reshape(16, 16)
    mm = sm.random_medium(16, 16, 0.2e-3, seed=5)
    mats_or = [_mat_of(a) for a in A]
    nodeA = torch.from_numpy(np.ascontiguousarray(A[ids])).cuda()
    zeros = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    src = [(8, 8), (0, 3)]
    R64, st = solver.solve_refined(mm.h, [sm.PARENT_STEEL], zeros, torch.from_numpy(mm.orient).cuda(), src,
                                   precision="f64", node_A=nodeA)
    assert st["converged"] == 1
    for k, sn in enumerate(src):
        ref = orc.solve_refined(mm.h, mats_or, ids, mm.orient, sn)
        e = _rel(R64[k].cpu().numpy(), ref)
        print("  source %s: f64 %.3g" % (sn, e), flush=True)
        assert e <= 1e-12


def test_stiffness_inversion_step_lowers_the_misfit(solver, orc):
    # the use the per-node input is for: observations from the oracle on a true model with
    # 256 stiffnesses scattered over the nodes, a uniform starting model, one step along
    # -dL/dA (largest change 0.3 % of the stiffness) through per-node values; the misfit
    # falls by the first-order prediction step |dL/dA|^2 within 10 % (the oracle's own
    # gradient and fields give 0.980 of it on this case)
    import torch
    n, h = 16, 0.3e-3
    rng = np.random.default_rng(9)
    A_true = _random_stiffness(rng, 256)
    ids = rng.integers(0, 256, size=(n, n)).astype(np.uint8)
    orient = sm.f32(np.full((n, n), 0.4))
    sources = [(2, 0), (8, 0), (13, 0)]
    receivers = [(1, n - 1), (6, n - 1), (10, n - 1), (14, n - 1), (n - 1, 8), (0, 8)]
    mats_true = [_mat_of(a) for a in A_true]
    obs = np.array([[orc.solve_fmm(h, mats_true, ids, orient, s, 2)[r[1], r[0]] for r in receivers]
                    for s in sources])
    zeros = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    ori = torch.from_numpy(orient).cuda()
    A0 = np.tile(_a_of(sm.TI_STEEL).astype(np.float32), (n, n, 1))
    dobs = torch.from_numpy(obs).cuda()

    def misfit(A, grad=False):
        out = solver.misfit_gradient(h, [sm.PARENT_STEEL], zeros, ori, sources, receivers, dobs, precision="f64",
                                     stiffness=grad, node_A=torch.from_numpy(np.ascontiguousarray(A)).cuda())
        return float(out[0].item()), out[2]

    print("inversion step: 16 x 16, 256 true stiffnesses", flush=True)
    L0, (_, dA) = misfit(A0, grad=True)
    g = dA.cpu().numpy()
    step = 0.003 * np.abs(A0).max() / np.abs(g).max()
    A1 = (A0 - step * g).astype(np.float32)
    L1, _ = misfit(A1)
    pred = -step * float((g * g).sum())
    print("  loss %.4e -> %.4e (predicted change %.3e, got %.3e)" % (L0, L1, pred, L1 - L0), flush=True)
    assert L1 < L0
    assert abs((L1 - L0) - pred) <= 0.1 * abs(pred)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autograd_stiffness(solver, prec):
    # receiver_times with node_A as a differentiable input: for a loss linear in the
    # receiver times, dL/dT is the weight tensor itself, so the autograd gradients must be
    # bitwise those of the adjoint entry point called with the same weights; a quadratic
    # misfit must match the fused misfit call to the rounding of the residuals.
    import torch
    from paper_2302_10988_amd import receiver_times
    m = sm.random_medium(64, 48, 0.2e-3, seed=6, n_mats=3)
    rng = np.random.default_rng(6)
    A = _random_stiffness(rng, m.nx * m.nz).reshape(m.nz, m.nx, 4)
    mats = [_mat_of(a) for a in _random_stiffness(rng, 3)]
    dt = torch.float64 if prec == "f64" else torch.float32
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(m.orient).to(dt).cuda().requires_grad_(True)
    nodeA = torch.from_numpy(A).cuda().requires_grad_(True)
    sources = [m.sources[0], (2, 1), (60, 3)]
    receivers = [(63, 47), (0, 47), (30, 47), (10, 20)]
    W = torch.from_numpy(rng.normal(size=(3, 4))).to(dt).cuda()
    print("autograd stiffness:", prec, flush=True)
    Tr = receiver_times(solver, m.h, mats, mid, ori, sources, receivers, node_A=nodeA)
    assert Tr.dtype == dt
    (Tr * W).sum().backward()
    (dth, dA), _ = solver.adjoint(m.h, mats, mid, ori.detach(), sources, receivers, W.contiguous(),
                                  precision=prec, stiffness=True, node_A=nodeA.detach())
    assert torch.equal(ori.grad, dth)
    assert nodeA.grad.dtype == torch.float32 and nodeA.grad.shape == nodeA.shape
    assert torch.equal(nodeA.grad, dA.to(torch.float32))
    # quadratic misfit against the fused forward + adjoint call
    ori.grad = None
    nodeA.grad = None
    obs = torch.full((3, 4), 3e-6, dtype=dt, device="cuda")
    Tr = receiver_times(solver, m.h, mats, mid, ori, sources, receivers, node_A=nodeA)
    (0.5 * ((Tr.double() - obs.double()) ** 2).sum()).backward()
    _, _, (dth2, dA2), _ = solver.misfit_gradient(m.h, mats, mid, ori.detach(), sources, receivers, obs,
                                                   precision=prec, stiffness=True, node_A=nodeA.detach())
    tol = 1e-5 if prec == "f32" else 1e-12
    gd = (ori.grad - dth2).abs().max().item() / dth2.abs().max().item()
    ga = (nodeA.grad.double() - dA2.double()).abs().max().item() / dA2.abs().max().item()
    print("  vs fused misfit: dtheta %.3g, dA %.3g" % (gd, ga), flush=True)
    assert gd <= tol and ga <= max(tol, 1e-6)
