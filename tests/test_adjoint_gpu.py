"""GPU orientation gradient (through the C ABI) against the oracle's reverse sweep.

Bars:
  - float64 mode: the GPU field equals the oracle's to ~1e-15, so both sides freeze the
    same choices; the gradient then agrees to 1e-9 of its largest entry (the two sides
    use different but exact derivative formulas: the oracle differentiates the paper's
    geometric construction, the GPU its rsqrt form; the oracle's group-speed derivative
    is a Richardson difference good to ~1e-10).
  - mixed mode (float32 wavefront math): travel times differ from float64 by < 1e-6
    relative, which moves the partial derivatives by about as much; a stencil choice can
    only differ where two candidates tie within that rounding.  Bar: cosine similarity
    >= 0.99999 and every entry within 1e-4 of the largest.
  - the tomography misfit over a 32 x 32 bilinear control grid (256 x 256 nodes, 32
    sources, 32 receivers): control gradient against the oracle, and against central
    differences of the GPU forward solve: step 1e-6 rad on 48 controls (tight), step
    1e-3 rad on all 1024 (the controls whose step crosses a stencil switch, found by a
    second difference at half the step, are held only through the median over all; the
    cosine bar applies to the others);
  - the GPU gradient against the ray-path gradient along the GPU's own rays (a different
    discretisation of the same derivative): projected onto 6 x 6 smooth controls, cosine
    at least 0.95 on a 128 x 128 medium, and the same as the oracle's pair within 1e-3.
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


def _dev(m, dtype):
    import torch
    return torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(np.ascontiguousarray(m.orient)).to(dtype).cuda()


def oracle_grad(orc, m, sources, receivers, dLdT):
    """Sum over sources of the oracle gradient for g = dL/dT at the receivers."""
    tot = np.zeros((m.nz, m.nx))
    for s, src in enumerate(sources):
        g = np.zeros((m.nz, m.nx))
        for r, rec in enumerate(receivers):
            g[rec[1], rec[0]] += dLdT[s, r]
        tot += orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g)[1]
    return tot


def _cos(a, b):
    return float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("seed", [5, 8])
def test_adjoint_f64_vs_oracle(solver, orc, seed):
    import torch
    m = sm.random_medium(53, 41, 0.2e-3, seed=seed, n_mats=3)
    rng = np.random.default_rng(seed)
    sources = [m.sources[0], (3, 2), (50, 38)]
    receivers = [(52, 40), (0, 40), (26, 0), (10, 20), (45, 5)]
    dLdT = rng.normal(size=(len(sources), len(receivers)))
    mid, ori = _dev(m, torch.float64)
    print("adjoint f64 vs oracle: seed", seed, flush=True)
    dth, T, st = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers,
                                torch.from_numpy(dLdT).cuda(), precision="f64", return_T=True)
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    ref = oracle_grad(orc, m, sources, receivers, dLdT)
    got = dth.cpu().numpy()
    scale = np.abs(ref).max()
    print("max |diff| / max |ref| = %.3g, lambda updates %d, passes %d"
          % (np.abs(got - ref).max() / scale, st["lambda_updates"], st["outer_iters"]))
    assert np.abs(got - ref).max() <= 1e-9 * scale
    for s, src in enumerate(sources):
        Tref = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient, src, 2)
        assert np.allclose(T[s].cpu().numpy(), Tref, rtol=1e-12, atol=0)


def test_adjoint_mixed_vs_oracle(solver, orc):
    import torch
    m = sm.weld(n=128, h=0.4e-3, seed=0)
    sources = [(20, 0), (64, 0), (110, 0)]
    receivers = [(8 * k + 4, 127) for k in range(16)]
    rng = np.random.default_rng(1)
    dLdT = rng.normal(size=(len(sources), len(receivers)))
    mid, ori = _dev(m, torch.float32)
    print("adjoint mixed vs oracle: weld 128", flush=True)
    dth, st = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers,
                             torch.from_numpy(dLdT).float().cuda())
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    ref = oracle_grad(orc, m, sources, receivers, dLdT)
    got = dth.cpu().numpy().astype(np.float64)
    scale = np.abs(ref).max()
    c = _cos(got, ref)
    print("mixed: cos %.9f, max |diff|/max %.3g" % (c, np.abs(got - ref).max() / scale))
    assert c >= 0.99999
    assert np.abs(got - ref).max() <= 1e-4 * scale


def test_adjoint_deterministic_and_schedule_invariant(solver):
    import torch
    m = sm.random_medium(70, 66, 0.2e-3, seed=3, n_mats=2)
    sources = [m.sources[0], (0, 0)]
    receivers = [(69, 65), (0, 65), (35, 30)]
    dLdT = torch.ones((2, 3), dtype=torch.float64, device="cuda")
    mid, ori = _dev(m, torch.float64)
    a, _ = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers, dLdT, precision="f64")
    b, _ = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers, dLdT, precision="f64")
    c, st = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers, dLdT, precision="f64", inner_sweeps=3)
    assert torch.equal(a, b)
    assert torch.equal(a, c), (a - c).abs().max().item()


def test_misfit_gradient_tomography(solver, orc):
    # 256 x 256 TI grid, orientation from 32 x 32 controls (evaluation model seed 2),
    # observations from the true model (seed 1) by the oracle, 32 sources x 32 receivers
    import torch
    true = sm.adjoint_grid(seed=1)
    m = sm.adjoint_grid(seed=2)
    nc = m.controls.shape[0]
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(8)     # the oracle's C calls release the GIL
    print("misfit gradient: oracle observations", flush=True)

    def observe(s):
        Tt = orc.solve_fmm(true.h, true.mats, true.mat_id, true.orient, s, 2)
        return [Tt[r[1], r[0]] for r in true.receivers]
    obs = np.array(list(pool.map(observe, true.sources)))
    mid, _ = _dev(m, torch.float32)
    ctrl = torch.from_numpy(m.controls).float().cuda()
    ori = solver.bilinear(ctrl, m.nz, m.nx)
    # the device interpolation reproduces the generator's float32 orientation
    assert np.allclose(ori.cpu().numpy(), m.orient, rtol=0, atol=2e-7)
    print("misfit gradient: GPU", flush=True)
    loss, trec, dth, st = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers,
                                                 torch.from_numpy(obs).float().cuda())
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    gc = solver.bilinear_transpose(dth, nc, nc).cpu().numpy().astype(np.float64)
    # oracle: same loss through the float32 orientation
    print("misfit gradient: oracle", flush=True)
    W = sm.bilinear_weights(m.nz, nc)
    obs32 = obs.astype(np.float32).astype(np.float64)

    def one_source(s):
        src = m.sources[s]
        T = orc.solve_fmm(m.h, m.mats, m.mat_id, m.orient, src, 2)
        g = np.zeros_like(T)
        ls = 0.0
        for r, rec in enumerate(m.receivers):
            d = T[rec[1], rec[0]] - obs32[s, r]
            g[rec[1], rec[0]] += d
            ls += 0.5 * d * d
        print("  oracle source", s, flush=True)
        return ls, orc.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g)[1]
    parts = list(pool.map(one_source, range(len(m.sources))))
    ref_loss = sum(p[0] for p in parts)
    dref = sum(p[1] for p in parts)
    gref = W.T @ dref @ W
    c = _cos(gc, gref)
    print("tomography: loss gpu %.6e oracle %.6e, control-gradient cos %.9f, max diff / max %.3g"
          % (loss.item(), ref_loss, c, np.abs(gc - gref).max() / np.abs(gref).max()))
    assert abs(loss.item() - ref_loss) <= 1e-3 * ref_loss
    assert c >= 0.9999
    assert np.abs(gc - gref).max() <= 1e-3 * np.abs(gref).max()
    # central differences of the GPU forward (float64): a sample of controls at 1e-6 rad, all at 1e-3
    rng = np.random.default_rng(0)
    sample = rng.choice(nc * nc, 48, replace=False)
    mid64 = torch.from_numpy(m.mat_id).cuda()
    obs_d = torch.from_numpy(obs32).cuda()
    rows = torch.tensor([r[1] for r in m.receivers], device="cuda")
    cols = torch.tensor([r[0] for r in m.receivers], device="cuda")

    def loss_at(cv):
        th = solver.bilinear(torch.from_numpy(cv).cuda(), m.nz, m.nx)
        T, _ = solver.solve(m.h, m.mats, mid64, th, m.sources, precision="f64")
        return 0.5 * float(((T[:, rows, cols] - obs_d) ** 2).sum().item())

    base = m.controls.astype(np.float32).astype(np.float64)

    def central(qs, e):
        out = []
        for q in qs:
            cp, cm = base.copy(), base.copy()
            cp.flat[q] += e
            cm.flat[q] -= e
            out.append((loss_at(cp) - loss_at(cm)) / (2 * e))
        return np.array(out)

    # step 1e-6 rad on the sample: no stencil switch within the step, so the discrete map
    # is differentiated exactly
    ga = gc.flat[sample]
    fd = central(sample, 1e-6)
    rel = np.abs(ga - fd) / np.abs(fd).max()
    print("central differences, step 1e-6 (48 controls): cos %.6f, median rel %.3g, max rel %.3g"
          % (_cos(ga, fd), np.median(rel), rel.max()), flush=True)
    assert _cos(ga, fd) >= 0.99999
    assert rel.max() <= 1e-3
    # step 1e-3 rad (the configuration's) on all 1024 controls.  The choice by score makes
    # T piecewise smooth with small jumps; a step across a jump gives a difference that
    # grows like 1/step, and with 256 x 256 nodes under every control about half of the
    # steps cross one.  Such controls are found by a second difference at half the step
    # (a smooth entry agrees to O(step^2)); the cosine bar holds on the others, the median
    # bar over all, both scaled by the largest gradient entry.
    qs = np.arange(nc * nc)
    ga = gc.flat[qs]
    f1, f2 = central(qs, 1e-3), central(qs, 5e-4)
    scale = np.abs(ga).max()
    smooth = np.abs(f1 - f2) <= 0.05 * np.abs(f1) + 1e-3 * scale
    rel = np.abs(ga - f1) / scale
    cs = _cos(ga[smooth], f1[smooth])
    print("central differences, step 1e-3 (1024 controls): %d cross a stencil switch; on the others cos %.6f, "
          "median rel %.3g, max rel %.3g; median rel over all %.3g"
          % ((~smooth).sum(), cs, np.median(rel[smooth]), rel[smooth].max(), np.median(rel)), flush=True)
    # measured: 457 of 1024 steps cross a switch; cosine 0.99907 on the others, median
    # 1.1e-3 there and 4.8e-3 over all
    assert smooth.sum() >= 0.4 * len(qs)
    assert cs >= 0.98
    assert np.median(rel) <= 1e-2


def test_bilinear_against_matrices(solver):
    import torch
    rng = np.random.default_rng(4)
    for nz, nx, ncz, ncx in ((256, 256, 32, 32), (37, 53, 5, 9), (20, 20, 2, 2)):
        ctrl = rng.normal(size=(ncz, ncx))
        Wz, Wx = sm.bilinear_weights(nz, ncz), sm.bilinear_weights(nx, ncx)
        th = solver.bilinear(torch.from_numpy(ctrl).cuda(), nz, nx).cpu().numpy()
        assert np.allclose(th, Wz @ ctrl @ Wx.T, rtol=0, atol=1e-14)
        g = rng.normal(size=(nz, nx))
        gt = solver.bilinear_transpose(torch.from_numpy(g).cuda(), ncz, ncx).cpu().numpy()
        assert np.allclose(gt, Wz.T @ g @ Wx, rtol=1e-12, atol=1e-12)


def test_adjoint_errors(solver):
    import torch
    from paper_2302_10988_amd import AliError
    m = sm.tiny_ti()
    mid, ori = _dev(m, torch.float32)
    g = torch.ones((1, 1), device="cuda")
    with pytest.raises(AliError):
        solver.adjoint(m.h, m.mats, mid, ori, m.sources, [(64, 3)], g)
    with pytest.raises(AliError) as e:
        solver.adjoint(m.h, m.mats, mid, ori, m.sources, [(3, 3)], g, arith="f32")
    assert e.value.status == -5
    with pytest.raises(AliError):
        solver.bilinear(torch.ones((1, 4), device="cuda"), 10, 10)


@pytest.mark.parametrize("band,inner", [(1, 2), (1, 64), (2, 2), (2, 64), (3, 4), (0, 4)])
def test_forward_is_exact_fixed_point_under_every_schedule(solver, band, inner):
    # the adjoint re-derives every node's candidate with the same update on the final
    # field; any node whose stored value the update does not reproduce is counted.  A
    # schedule that misses a re-evaluation (a lost mark, a stale comparison) shows here.
    # band 0 is the unbanded schedule: every marked tile is due at once, and the pass
    # cap turns a schedule that never goes idle into an error instead of a long run.
    import torch
    for m in (sm.adjoint_grid(seed=2, n_src=8, n_rec=8), sm.weld(n=192, h=0.25e-3, seed=1, n_src=6, n_rec=6)):
        mid = torch.from_numpy(m.mat_id).cuda()
        for arith, dt in (("mixed", torch.float32), ("f64", torch.float32)):
            ori = torch.from_numpy(m.orient).to(dt).cuda()
            g = torch.ones((len(m.sources), len(m.receivers)), device="cuda")
            print("fixed point:", m.name, "band", band, "inner", inner, arith, flush=True)
            _, st = solver.adjoint(m.h, m.mats, mid, ori, m.sources, m.receivers, g, arith=arith,
                                   band_cells=band, inner_sweeps=inner, max_sweeps=20000)
            assert st["forward"]["converged"] == 1 and st["converged"] == 1
            assert st["choice_mismatches"] == 0


def test_autograd_matches_misfit_gradient(solver):
    # loss built with torch ops on the differentiable receiver times and control grid:
    # its gradient must equal the fused misfit entry point's (same kernels, same sums)
    import torch
    from paper_2302_10988_amd import bilinear_orientation, receiver_times
    m = sm.adjoint_grid(seed=2, n_src=8, n_rec=8)
    mid = torch.from_numpy(m.mat_id).cuda()
    ctrl = torch.from_numpy(m.controls).float().cuda().requires_grad_(True)
    obs = torch.full((8, 8), 2e-6, device="cuda")
    ori = bilinear_orientation(solver, ctrl, m.nz, m.nx)
    Tr = receiver_times(solver, m.h, m.mats, mid, ori, m.sources, m.receivers)
    loss = 0.5 * ((Tr.double() - obs.double()) ** 2).sum()
    loss.backward()
    with torch.no_grad():
        ori2 = solver.bilinear(ctrl.detach(), m.nz, m.nx)
        l2, tr2, dth, _ = solver.misfit_gradient(m.h, m.mats, mid, ori2, m.sources, m.receivers, obs)
        g2 = solver.bilinear_transpose(dth, 32, 32)
    gd = (ctrl.grad - g2).abs().max().item() / g2.abs().max().item()
    print("autograd: loss %.9e fused %.9e, control gradient max diff / max %.3g"
          % (loss.item(), l2.item(), gd))
    assert torch.equal(Tr.detach(), tr2)
    # the fused call forms the residuals from float64 times, the autograd graph from the
    # float32 receiver times: the losses differ by the rounding of T (~1e-7 relative)
    assert abs(loss.item() - l2.item()) <= 1e-5 * abs(l2.item())
    assert gd <= 1e-5


def test_gradient_vs_ray_path_gradient(solver, orc):
    # the oracle's version of this comparison gives cosine 0.963 at this size (128 x 128,
    # 6 x 6 controls, one source, six weighted receivers)
    import torch
    from raypath_grad import cosine, ray_path_gradient
    rng = np.random.default_rng(3)
    n, nc, h = 128, 6, 0.25e-3
    ctrl = rng.uniform(-0.8, 0.8, size=(nc, nc))
    w = rng.normal(size=6)
    W = sm.bilinear_weights(n, nc)
    th = sm.f32(W @ ctrl @ W.T)          # float32 values: the rays take float32 orientations
    mats, mid = [sm.TI_STEEL], np.zeros((n, n), np.uint8)

    def at(p):
        return (int(round(p[0] * (n - 1) / 63)), int(round(p[1] * (n - 1) / 63)))

    src = at((20, 0))
    recs = [at(r) for r in [(5, 63), (30, 63), (50, 63), (63, 40), (63, 20), (40, 63)]]
    did, dth = torch.from_numpy(mid).cuda(), torch.from_numpy(th).cuda()
    print("ray-path gradient: 128 x 128, 6 receivers", flush=True)
    grad, T, st = solver.adjoint(h, mats, did, dth, [src], recs, torch.from_numpy(w[None, :]).cuda(),
                                 precision="f64", return_T=True)
    assert st["converged"] == 1
    paths, npts, _ = [x.cpu().numpy() for x in solver.trace_rays(h, mats, did, dth.float(), T, [src], recs)]
    ray = np.zeros((n, n))
    for b in range(len(recs)):
        assert npts[0, b] > 1
        ray += w[b] * ray_path_gradient(orc, h, mats, mid, th, paths[0, b, : npts[0, b]].astype(np.float64))
    ga, gr = W.T @ grad.cpu().numpy() @ W, W.T @ ray @ W
    c = cosine(ga, gr)
    # the same comparison on the oracle's own field, gradient and rays
    Tref = orc.solve_fmm(h, mats, mid, th, src, 2)
    g = np.zeros((n, n))
    rref = np.zeros((n, n))
    for b, r in enumerate(recs):
        g[r[1], r[0]] += w[b]
        pts, _, ok = orc.trace_ray(h, mats, mid, th, Tref, src, r)
        rref += w[b] * ray_path_gradient(orc, h, mats, mid, th, pts)
    cref = cosine(W.T @ orc.adjoint(h, mats, mid, th, src, g)[1] @ W, W.T @ rref @ W)
    print("  control-space cosine: GPU %.4f, oracle %.4f" % (c, cref), flush=True)
    assert c >= 0.95 and abs(c - cref) <= 1e-3
