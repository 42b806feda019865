"""The misfit gradient on the s-fold refined medium (Section 4.5's subgrid size) through the
C-ABI (ali_misfit_gradient_subgrid): against the oracle composition of tests/subgrid_grad.py
(fine-grid adjoint carried back through the nearest-node refinement), at the float64 bar of
the plain adjoint (1e-9 of the largest entry) and, in mixed arithmetic, at the cosine and
1e-4 bars of the plain mixed adjoint; the loss, the modelled times and the fields at the nodes
with them."""
import numpy as np
import pytest

import synthmedia as sm
from subgrid_grad import misfit_gradient as ref_grad

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    from paper_2302_10988_amd import Solver
    assert torch.cuda.is_available()
    return Solver(0)


def _cos(a, b):
    return float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))


def _obs(orc, m, sources, receivers, s, seed):
    _, t0, _ = ref_grad(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers,
                        np.zeros((len(sources), len(receivers))), s)
    return t0 * (1.0 + 0.01 * np.random.default_rng(seed).normal(size=t0.shape))


@pytest.mark.parametrize("s", [3, 5])
def test_subgrid_gradient_f64_vs_oracle(solver, orc, s):
    import torch
    m = sm.random_medium(31, 26, 0.2e-3, seed=6, n_mats=3)
    sources = [(15, 0), (2, 3)]
    receivers = [(0, 25), (30, 25), (15, 25), (28, 10)]
    obs = _obs(orc, m, sources, receivers, s, 1)
    print("subgrid gradient f64 vs oracle: s", s, flush=True)
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(np.ascontiguousarray(m.orient)).double().cuda()
    T = torch.empty((len(sources), m.nz, m.nx), dtype=torch.float64, device="cuda")
    loss, trec, dth, st = solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers,
                                                 torch.from_numpy(obs).cuda(), precision="f64", T_out=T,
                                                 subgrid=s)
    L, tref, G = ref_grad(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers, obs, s)
    got = dth.cpu().numpy()
    scale = np.abs(G).max()
    print("max |diff| / max |ref| = %.3g, loss %.6e vs %.6e" % (np.abs(got - G).max() / scale, loss.item(), L))
    assert st["converged"] == 1 and st["choice_mismatches"] == 0
    assert np.abs(got - G).max() <= 1e-9 * scale
    assert abs(loss.item() - L) <= 1e-12 * L
    assert np.allclose(trec.cpu().numpy(), tref, rtol=1e-12, atol=0)
    mid_f, ori_f = orc.refine_medium(m.mat_id, m.orient, s)
    for k, (si, sj) in enumerate(sources):
        Tf = orc.solve_fmm(m.h / s, m.mats, mid_f, ori_f, (si * s, sj * s), 2)
        assert np.allclose(T[k].cpu().numpy(), Tf[::s, ::s], rtol=1e-12, atol=0)


def test_subgrid_gradient_mixed_vs_oracle(solver, orc):
    import torch
    m = sm.weld(n=96, h=0.4e-3, seed=0)
    s = 3
    sources = [(16, 0), (48, 0), (80, 0)]
    receivers = [(12 * k + 6, 95) for k in range(8)]
    obs = _obs(orc, m, sources, receivers, s, 2)
    print("subgrid gradient mixed vs oracle: weld 96, s 3", flush=True)
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(np.ascontiguousarray(m.orient)).float().cuda()
    loss, trec, dth, st = solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers,
                                                 torch.from_numpy(obs).float().cuda(), subgrid=s)
    L, tref, G = ref_grad(orc, m.h, m.mats, m.mat_id, m.orient, sources, receivers, obs, s)
    got = dth.cpu().numpy().astype(np.float64)
    scale = np.abs(G).max()
    c = _cos(got, G)
    print("mixed: cos %.9f, max |diff|/max %.3g" % (c, np.abs(got - G).max() / scale))
    assert st["converged"] == 1
    assert c >= 0.99999
    assert np.abs(got - G).max() <= 1e-4 * scale
    assert np.allclose(trec.cpu().numpy(), tref, rtol=1e-4, atol=0)


def test_subgrid_one_equals_plain_and_errors(solver):
    import torch
    m = sm.random_medium(24, 20, 0.2e-3, seed=3, n_mats=2)
    sources = [(12, 0)]
    receivers = [(0, 19), (23, 19)]
    mid = torch.from_numpy(m.mat_id).cuda()
    ori = torch.from_numpy(np.ascontiguousarray(m.orient)).float().cuda()
    obs = torch.zeros((1, 2), device="cuda")
    a = solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers, obs)
    b = solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers, obs, subgrid=1)
    assert torch.equal(a[2], b[2]) and torch.equal(a[1], b[1])
    for bad in (2, 17, -3):
        with pytest.raises(RuntimeError):
            solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers, obs, subgrid=bad)
    with pytest.raises(ValueError):
        solver.misfit_gradient(m.h, m.mats, mid, ori, sources, receivers, obs, subgrid=3, stiffness=True)
