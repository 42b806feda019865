"""SH wave mode on the GPU (through the C ABI) against the oracle's SH mode.

The GPU runs its qP kernels on the record whose qP speeds are the SH speeds (c11 = c66,
c33 = c44, c55 = min(c44, c66), c13 = -c55); the oracle computes SH from its own
Christoffel entry and the closed-form elliptical wave surface.  Bars as for qP:
  - float64: fields within 1e-12, the nested source grids too; orientation gradient within
    1e-9 of its largest entry;
  - mixed arithmetic: fields within 1e-4; rays: time within 1e-4 relative and path within
    0.05 cells of the oracle's;
  - the stiffness gradient refuses SH (ALI_EUNSUPPORTED), and an SH material needs c44,
    c66 > 0 only.
"""

import numpy as np
import pytest

import synthmedia as sm

pytestmark = pytest.mark.gpu

SH_MATS = [sm.TI_STEEL, dict(sm.CUBIC_STEEL, c66=60e9), dict(sm.PARENT_STEEL, c66=40e9)]


@pytest.fixture(scope="module")
def solver():
    import torch
    from paper_2302_10988_amd import Solver
    assert torch.cuda.is_available()
    return Solver(0)


def _medium(seed, nx=45, nz=39):
    m = sm.random_medium(nx, nz, 0.2e-3, seed=seed, n_mats=3)
    m.mats = list(SH_MATS)
    return m


def _dev(m, dtype):
    import torch
    return torch.from_numpy(m.mat_id).cuda(), torch.from_numpy(np.ascontiguousarray(m.orient)).to(dtype).cuda()


def _poly_dist(points, poly):
    """Distance of each point to a polyline."""
    a, b = poly[:-1], poly[1:]
    ab = b - a
    L2 = np.maximum((ab ** 2).sum(1), 1e-30)
    out = []
    for p in points:
        t = np.clip(((p - a) * ab).sum(1) / L2, 0, 1)
        q = a + t[:, None] * ab
        out.append(np.sqrt(((q - p) ** 2).sum(1)).min())
    return np.array(out)


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    fin = np.isfinite(b) & (b > 0)
    return float((np.abs(a - b)[fin] / b[fin]).max())


@pytest.mark.parametrize("seed", [3, 8])
def test_sh_forward_vs_oracle(solver, orc, seed):
    import torch
    m = _medium(seed)
    sources = [m.sources[0], (0, 0), (44, 38)]
    sh = orc.as_sh(m.mats)
    mid, ori64 = _dev(m, torch.float64)
    print("SH forward: seed", seed, flush=True)
    T64, st = solver.solve(m.h, m.mats, mid, ori64, sources, precision="f64", wave="sh")
    assert st["converged"] == 1
    T32, _ = solver.solve(m.h, m.mats, mid, ori64.float(), sources, wave="sh")
    R64, _ = solver.solve_refined(m.h, m.mats, mid, ori64, sources, precision="f64", wave="sh")
    for k, src in enumerate(sources):
        ref = orc.solve_fmm(m.h, sh, m.mat_id, m.orient, src, 2)
        e64, e32 = _rel(T64[k].cpu().numpy(), ref), _rel(T32[k].cpu().numpy(), ref)
        refr = orc.solve_refined(m.h, sh, m.mat_id, m.orient, src)
        er = _rel(R64[k].cpu().numpy(), refr)
        print("  source %s: f64 %.3g, mixed %.3g, refined f64 %.3g" % (src, e64, e32, er), flush=True)
        assert e64 <= 1e-12 and e32 <= 1e-4 and er <= 1e-12
    # the qP fields differ: the wave option is honoured
    Tq, _ = solver.solve(m.h, m.mats, mid, ori64, sources, precision="f64")
    assert (Tq - T64).abs().max().item() > 1e-3 * T64[torch.isfinite(T64)].max().item()


def test_sh_adjoint_vs_oracle(solver, orc):
    import torch
    m = _medium(5)
    sh = orc.as_sh(m.mats)
    sources = [m.sources[0], (3, 2)]
    receivers = [(44, 38), (0, 38), (22, 0), (40, 4)]
    dLdT = np.random.default_rng(5).normal(size=(len(sources), len(receivers)))
    mid, ori = _dev(m, torch.float64)
    print("SH adjoint f64", flush=True)
    dth, st = solver.adjoint(m.h, m.mats, mid, ori, sources, receivers, torch.from_numpy(dLdT).cuda(),
                             precision="f64", wave="sh")
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    ref = np.zeros((m.nz, m.nx))
    for s, src in enumerate(sources):
        g = np.zeros((m.nz, m.nx))
        for r, rec in enumerate(receivers):
            g[rec[1], rec[0]] += dLdT[s, r]
        ref += orc.adjoint(m.h, sh, m.mat_id, m.orient, src, g)[1]
    err = np.abs(dth.cpu().numpy() - ref).max() / np.abs(ref).max()
    print("  max |diff| / max |ref| = %.3g" % err, flush=True)
    assert err <= 1e-9
    from paper_2302_10988_amd import AliError
    with pytest.raises(AliError):
        solver.adjoint(m.h, m.mats, mid, ori, sources, receivers, torch.from_numpy(dLdT).cuda(),
                       precision="f64", wave="sh", stiffness=True)


def test_sh_rays_vs_oracle(solver, orc):
    import torch
    m = _medium(11, 64, 48)
    sh = orc.as_sh(m.mats)
    sources = [(5, 0), (40, 0)]
    receivers = [(60, 47), (10, 47), (33, 30)]
    mid, ori = _dev(m, torch.float32)
    print("SH rays", flush=True)
    T, _ = solver.solve(m.h, m.mats, mid, ori, sources, wave="sh")
    paths, npts, tray = solver.trace_rays(m.h, m.mats, mid, ori, T, sources, receivers, wave="sh")
    paths, npts, tray = paths.cpu().numpy(), npts.cpu().numpy(), tray.cpu().numpy()
    assert np.all(npts > 0)
    for a, s in enumerate(sources):
        Tref = orc.solve_fmm(m.h, sh, m.mat_id, m.orient, s, 2)
        for b, r in enumerate(receivers):
            pts, t, ok = orc.trace_ray(m.h, sh, m.mat_id, m.orient, Tref, s, r)
            assert ok
            gp = paths[a, b, : npts[a, b]].astype(np.float64)
            d = _poly_dist(gp, np.asarray(pts, np.float64)).max()
            print("  %s -> %s: time %.3g, path %.3g" % (r, s, abs(tray[a, b] - t) / t, d), flush=True)
            assert abs(tray[a, b] - t) / t <= 1e-4 and d <= 0.05


def test_sh_material_checks(solver):
    import torch
    from paper_2302_10988_amd import AliError
    m = _medium(1, 20, 20)
    mid, ori = _dev(m, torch.float32)
    # an SH record needs c44, c66 > 0 only (the qP entries may be anything finite)
    shear_only = [dict(c11=0.0, c13=0.0, c33=0.0, c55=0.0, c44=80e9, c66=50e9, rho=7800.0)]
    T, st = solver.solve(m.h, shear_only, torch.zeros_like(mid), ori, m.sources, wave="sh")
    assert st["converged"] == 1 and torch.isfinite(T).all()
    with pytest.raises(AliError):
        solver.solve(m.h, shear_only, torch.zeros_like(mid), ori, m.sources)
    with pytest.raises(AliError):
        solver.solve(m.h, [dict(sm.TI_STEEL, c44=0.0)], torch.zeros_like(mid), ori, m.sources, wave="sh")
