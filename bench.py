"""Benchmark: batched anisotropic travel-time fields, their misfit gradient and ray paths
on one MI355X.

One step = one pass of the hot path over one batch: the 512x512 synthetic V-weld with 64
top-surface sources, solved in one batched relaxation (the paper's forward modeller,
Sections 2-4) inside one forward + adjoint call for the misfit of the 64 x 64 bottom
receiver times (orientation gradient at every node), then the 64 x 64 ray paths from the
receivers to every source through those fields (Section 5.1); float32 output, inputs
resident in HBM.

Prints one JSON line.  `value` is node updates per second of step time (one update = one
evaluation of the local ALI update at one node).  Alongside: forward+adjoint field solves
per second, rays per second, solved nodes/s, redundancy, the relaxation kernel's position
against its roof (HIP events around each launch), the accuracy of the last step against
the FP64 oracle, the plain single-field solve on the same GPU, and the oracle itself timed
on a bounded sample on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic arithmetic of the relaxation kernel (counted from the update's formulas):
# per node update: ordering tests of the 16 stencil pairs (96 compares), 8 straight-ray
# candidates (40 ops), acceptance test (2); per single-stencil estimate: 47 ops
# (interpolation weight, wavefront normal, phase speed with one sqrt, rsqrt, causality,
# score and ranking).  FMA counts as 2.
OPS_PER_UPDATE = 138
OPS_PER_ESTIMATE = 47
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published fp32 vector peak

# HBM traffic of the relaxation kernel from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE; each scaled by the same counter on a 256 MiB device copy in the same program),
# per launch, for the kernel sources with this hash.  Reported as null once the sources
# differ (profiles/k_relax_weld512x64.md holds the command and the raw figures).
TRAFFIC = {"sources_sha256_16": "2b281753796594bc", "fetch_bytes_per_launch": 32.863e6,
           "write_bytes_per_launch": 2.029e6}


def kernel_sources_hash():
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2302_10988_amd", "csrc")
    data = b"".join(open(p, "rb").read() for p in sorted(glob.glob(os.path.join(csrc, "*.hip"))) +
                    sorted(glob.glob(os.path.join(csrc, "*.hpp"))))
    return hashlib.sha256(data).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="weld512x64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (known bytes, to scale HBM counters)")
    return ap.parse_args()


def workload(name):
    import synthmedia as sm
    if name == "weld512x64":
        return sm.weld_multi()
    if name == "weld512":
        return sm.weld()
    raise SystemExit("unknown workload %s" % name)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the solver has no multi-GPU path; "
              "fields shard across GPUs without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2302_10988_amd import Solver

    m = workload(args.workload)
    dev = torch.device("cuda:0")
    mid = torch.from_numpy(m.mat_id).to(dev)
    ori = torch.from_numpy(m.orient).to(torch.float32).to(dev)
    out = torch.empty((len(m.sources), m.nz, m.nx), dtype=torch.float32, device=dev)
    rays = len(m.receivers) > 0
    solver = Solver(0)
    print("bench: workload %s, %d fields of %dx%d, warmup %d, steps %d"
          % (args.workload, len(m.sources), m.nx, m.nz, args.warmup, args.steps), file=sys.stderr, flush=True)

    if args.calib_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("bench: calibration copy of %d bytes done" % (a.numel() * 4), file=sys.stderr, flush=True)
        del a, b

    # observed times: straight rays at the parent steel's speed (a plain synthetic
    # target; the misfit's value does not change the work)
    src_xy = np.array(m.sources, dtype=np.float64)
    rec_xy = np.array(m.receivers, dtype=np.float64)
    dist = np.hypot(*(src_xy[:, None, :] - rec_xy[None, :, :]).transpose(2, 0, 1)) * m.h
    obs = torch.from_numpy(dist / 5900.0).to(torch.float32).to(dev)

    def step():
        t0 = time.perf_counter()
        loss, _, _, st = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs, T_out=out)
        t1 = time.perf_counter()
        solver.trace_rays(m.h, m.mats, mid, ori, out, m.sources, m.receivers)
        t2 = time.perf_counter()
        return st, t1 - t0, t2 - t1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    tot = dict(node_updates=0, stencil_evals=0, outer_iters=0, relax_ms=0.0, nodes=0, tile_visits=0)
    adj = dict(lambda_updates=0, outer_iters=0, relax_ms=0.0, ms=0.0, fwd_ms=0.0)
    wall_fa = wall_rays = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st, tfa, tr = step()
        f = st["forward"]
        for key in tot:
            tot[key] += f[key]
        for key in ("lambda_updates", "outer_iters", "relax_ms", "ms"):
            adj[key] += st[key]
        adj["fwd_ms"] += f["ms"]
        wall_fa += tfa
        wall_rays += tr
        print("bench: step %d done, %d + %d passes, forward %.2f ms, forward+adjoint %.2f ms, rays %.2f ms"
              % (k, f["outer_iters"], st["outer_iters"], f["ms"], st["ms"], tr * 1e3), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    # the plain single-field solver on the same GPU (one top source of the same weld)
    single = torch.empty((1, m.nz, m.nx), dtype=torch.float32, device=dev)
    solver.solve(m.h, m.mats, mid, ori, [m.sources[len(m.sources) // 2]], out=single)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, sst = solver.solve(m.h, m.mats, mid, ori, [m.sources[len(m.sources) // 2]], out=single)
    single_ms = (time.perf_counter() - ts) * 1e3

    n_fields = len(m.sources) * args.steps
    value = tot["node_updates"] / el
    ops = OPS_PER_UPDATE * tot["node_updates"] + OPS_PER_ESTIMATE * tot["stencil_evals"]
    achieved = ops / (tot["relax_ms"] * 1e-3) / 1e12
    line = {
        "metric": "node-updates/s & batched forward+adjoint field solves/s at ≤1e-4 rel err",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 wavefront math, f64 travel times and derivatives",
        "data": "synthetic",
        "config": {"workload": "V-weld %dx%d, h=%.1f mm, %d top sources x %d bottom receivers: batched forward + "
                               "adjoint (misfit gradient) + %d x %d ray paths"
                               % (m.nx, m.nz, m.h * 1e3, len(m.sources), len(m.receivers), len(m.sources),
                                  len(m.receivers)),
                   "grid": [m.nz, m.nx], "fields_per_step": len(m.sources), "src_box_radius": 2},
        "fwd_adj_field_solves_per_s": n_fields / el,
        "rays_per_s": len(m.sources) * len(m.receivers) * args.steps / el,
        "solved_nodes_per_s": tot["nodes"] / el,
        "redundancy_updates_per_node": tot["node_updates"] / max(tot["nodes"], 1),
        "stencil_estimates_per_update": tot["stencil_evals"] / max(tot["node_updates"], 1),
        "forward_ms_per_step": adj["fwd_ms"] / args.steps,
        "adjoint_ms_per_step": (adj["ms"] - adj["fwd_ms"]) / args.steps,
        "rays_ms_per_step": wall_rays * 1e3 / args.steps,
        "relax_launches_per_step": tot["outer_iters"] / args.steps,
        "relax_kernel_ms_per_step": tot["relax_ms"] / args.steps,
        "adjoint_lambda_updates_per_node": adj["lambda_updates"] / max(tot["nodes"], 1),
        "adjoint_launches_per_step": adj["outer_iters"] / args.steps,
        "adjoint_relax_kernel_ms_per_step": adj["relax_ms"] / args.steps,
        "single_field_solve": {"ms": single_ms, "fields_per_s": 1e3 / single_ms, "passes": sst["outer_iters"]},
        "roofline": {"kernel": "k_relax<double,float>", "bound": "alu", "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": (TRAFFIC["fetch_bytes_per_launch"] + TRAFFIC["write_bytes_per_launch"]
                                 if kernel_sources_hash() == TRAFFIC["sources_sha256_16"] else None),
                     "traffic_unit": "bytes per launch",
                     "avg_launch_ms": tot["relax_ms"] / max(tot["outer_iters"], 1)},
    }

    if not args.no_check:
        import oracle
        k = 0
        Tg = out[k].cpu().numpy().astype(np.float64)
        Tref = oracle.solve_fmm(m.h, m.mats, m.mat_id, m.orient, m.sources[k], 2)
        mask = Tref > 0
        rel = np.abs(Tg - Tref)[mask] / Tref[mask]
        line["max_rel_err_vs_oracle"] = float(rel.max())
        line["checked_fields"] = [k]

    if not args.no_cpu_baseline:
        import oracle
        # bounded sample of the same step on the host: one field (forward with its
        # update count, then the oracle's adjoint, which solves the field again) and 8 of
        # its 64 rays; the per-field time scales the rays up to all receivers
        k = len(m.sources) // 2
        src = m.sources[k]
        t0 = time.perf_counter()
        T, n_upd = oracle.solve_fmm_counted(m.h, m.mats, m.mat_id, m.orient, src, 2)
        g = np.zeros_like(T)
        for r, rec in enumerate(m.receivers):
            g[rec[1], rec[0]] += T[rec[1], rec[0]] - float(obs[k, r])
        oracle.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g)
        t_fa = time.perf_counter() - t0
        ray_sample = m.receivers[::8]
        t0 = time.perf_counter()
        for rec in ray_sample:
            oracle.trace_ray(m.h, m.mats, m.mat_id, m.orient, T, src, rec)
        t_rays = (time.perf_counter() - t0) * len(m.receivers) / len(ray_sample)
        per_field = t_fa + t_rays
        line["cpu_baseline"] = {"value": n_upd / per_field, "unit": "node-updates/s", "cores": 1,
                                "kind": "oracle", "fwd_adj_field_solves_per_s": 1.0 / per_field,
                                "forward_adjoint_s": t_fa, "rays_s_extrapolated": t_rays,
                                "sample": "field %d of %d: FP64 heap FMM forward + adjoint (re-solving the "
                                          "field) + %d of its %d rays, scaled to all %d; single thread"
                                          % (k, len(m.sources), len(ray_sample), len(m.receivers),
                                             len(m.receivers))}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
