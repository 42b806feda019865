"""Benchmark: batched anisotropic travel-time fields, their misfit gradient and ray paths
on one MI355X.

Workloads (one step each, inputs resident in HBM, float32 output):
  weld512x64 (default): the 512x512 synthetic V-weld with 64 top-surface sources, solved
      in one batched relaxation (the paper's forward modeller, Sections 2-4) inside one
      forward + adjoint call for the misfit of the 64 x 64 bottom-receiver times
      (orientation gradient at every node), then the 64 x 64 ray paths from the receivers
      to every source through those fields (Section 5.1).
  batch128: 128 media of uneven sizes (sides 256..1024), 32 top sources and 32 bottom
      receivers each (4096 fields), forward + adjoint of the per-medium misfit in one call
      with the autotuned schedule.

Prints one JSON line.  `value` is node updates per second of step time (one update = one
evaluation of the local ALI update at one node).  Alongside: forward+adjoint field solves
per second, rays per second, solved nodes/s, redundancy, the relaxation kernel against its
roofs (HIP events around each launch of one extra, untimed solve launched pass by pass),
the accuracy of the last step against the FP64 oracle, the plain single-field solve on the
same GPU, and the oracle itself timed on a bounded sample on the host (cpu_baseline).
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

# Algorithmic work of the relaxation kernel per node update (mixed arithmetic):
#  bytes: travel time read and written (float64, 16 B), orientation (float32, 4 B),
#  material id (1 B) = 21 B;
#  operations: ordering tests of the 16 stencil pairs (96 compares), 8 straight-ray
#  candidates (40 ops), acceptance test (2) = 138, plus 47 per admissible single-stencil
#  estimate (interpolation weight, wavefront normal, phase speed with one sqrt, rsqrt,
#  causality, score and ranking); FMA counts as 2.
BYTES_PER_UPDATE = 21
OPS_PER_UPDATE = 138
OPS_PER_ESTIMATE = 47
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector

# HBM traffic of the relaxation kernel from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE; each scaled by the same counter on a 256 MiB device copy in the same
# program), per launch of the 64-field weld forward (grid 8192 x 64; the counters are split
# by grid size), for the kernel sources with this hash, and the wave-level VALU instructions
# of the same launches (rocprofv3 --pmc SQ_INSTS_VALU).  Reported as null once the sources
# differ.
TRAFFIC = {"sources_sha256_16": "d4e0470f7521208c", "fetch_bytes_per_launch": 22.88e6,
           "write_bytes_per_launch": 1.559e6, "valu_wave_insts_per_launch": 5.822e6}


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
    ap.add_argument("--workload", default="weld512x64", choices=["weld512x64", "batch128"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-call timings of the other modes (nested source grids, SH, velocity "
                         "table, stiffness gradient, fixed ray plane families)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (known bytes, to scale HBM counters)")
    return ap.parse_args()


def straight_ray_obs(sources, receivers, h, v=5900.0):
    """Observed times of a plain synthetic target: straight rays at the parent steel's
    speed (the misfit's value does not change the work)."""
    import numpy as np
    s = np.array(sources, dtype=np.float64)
    r = np.array(receivers, dtype=np.float64)
    return np.hypot(*(s[:, None, :] - r[None, :, :]).transpose(2, 0, 1)) * h / v


def relax_roofline(solver, call):
    """Run `call(graph=0)` once (passes launched one by one, HIP events around each relax
    launch on the solver's stream) and return the relaxation kernel's position against
    the HBM and ALU roofs."""
    st = call()
    f = st["forward"] if "forward" in st else st
    launches = max(f["outer_iters"], 1)
    sec = f["relax_ms"] * 1e-3
    gbs = BYTES_PER_UPDATE * f["node_updates"] / sec / 1e9
    tflops = (OPS_PER_UPDATE * f["node_updates"] + OPS_PER_ESTIMATE * f["stencil_evals"]) / sec / 1e12
    traffic = valu = None
    if TRAFFIC["sources_sha256_16"] == kernel_sources_hash():
        traffic = TRAFFIC["fetch_bytes_per_launch"] + TRAFFIC["write_bytes_per_launch"]
        # per node update, in wave instructions (each covers 64 lanes)
        valu = TRAFFIC["valu_wave_insts_per_launch"] / (f["node_updates"] / launches)
    return {"kernel": "k_relax<double,float>", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "bytes_per_update": BYTES_PER_UPDATE, "avg_launch_ms": f["relax_ms"] / launches,
            "updates_per_launch": f["node_updates"] / launches,
            "alu": {"achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / FP32_VECTOR_PEAK_TFLOPS},
            "valu_wave_insts_per_update": valu}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path (independent fields "
              "would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synthmedia as sm
    from paper_2302_10988_amd import Batch, Solver

    dev = torch.device("cuda:0")
    solver = Solver(0)
    if args.calib_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("bench: calibration copy of %d bytes done" % (a.numel() * 4), file=sys.stderr, flush=True)
        del a, b

    line = {"metric": "node-updates/s & batched forward+adjoint field solves/s at ≤1e-4 rel err",
            "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 wavefront math and adjoint pull weights; f64 travel times, lambda and gradient sums", "data": "synthetic"}

    if args.workload == "weld512x64":
        m = sm.weld_multi()
        mid = torch.from_numpy(m.mat_id).to(dev)
        ori = torch.from_numpy(m.orient).to(torch.float32).to(dev)
        out = torch.empty((len(m.sources), m.nz, m.nx), dtype=torch.float32, device=dev)
        obs_np = straight_ray_obs(m.sources, m.receivers, m.h)
        obs = torch.from_numpy(obs_np).to(torch.float32).to(dev)
        n_fields, n_rays = len(m.sources), len(m.sources) * len(m.receivers)
        line["config"] = {"workload": "V-weld %dx%d, h=%.1f mm, %d top sources x %d bottom receivers: batched "
                                      "forward + adjoint (misfit gradient) + %d x %d ray paths"
                                      % (m.nx, m.nz, m.h * 1e3, len(m.sources), len(m.receivers),
                                         len(m.sources), len(m.receivers)),
                          "grid": [m.nz, m.nx], "fields_per_step": n_fields, "src_box_radius": 2}

        def step():
            t0 = time.perf_counter()
            _, _, _, st = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs, T_out=out)
            t1 = time.perf_counter()
            solver.trace_rays(m.h, m.mats, mid, ori, out, m.sources, m.receivers)
            return st, t1 - t0, time.perf_counter() - t1

        roof_call = lambda: solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs,
                                                   T_out=out, graph=0)[3]
    else:
        media = sm.batch_media()
        batch = Batch(media, device=dev)
        n_fields, n_rays = batch.n_fields, 0
        obs_np = np.concatenate([straight_ray_obs(md.sources, md.receivers, md.h).ravel() for md in media])
        obs = torch.from_numpy(obs_np).to(torch.float32).to(dev)
        print("bench: autotuning the schedule (untimed)", file=sys.stderr, flush=True)
        tuned, tune_ms = solver.autotune_batch(batch)
        sched = {"band_cells": tuned["band_cells"], "inner_sweeps": tuned["inner_sweeps"]}
        sides = [md.nx for md in media]
        line["config"] = {"workload": "%d media, sides %d..%d (seed 3), h=0.1 mm, 32 top sources x 32 bottom "
                                      "receivers each: batched forward + adjoint of the per-medium misfit"
                                      % (len(media), min(sides), max(sides)),
                          "fields_per_step": n_fields, "node_fields": batch.field_nodes, "src_box_radius": 2,
                          "schedule": sched,
                          "autotune_ms": {"band%d_inner%d" % k: v for k, v in tune_ms.items()}}

        def step():
            t0 = time.perf_counter()
            _, _, _, st = solver.misfit_gradient_batch(batch, obs, **sched)
            return st, time.perf_counter() - t0, 0.0

        roof_call = lambda: solver.misfit_gradient_batch(batch, obs, graph=0, **sched)[3]

    print("bench: workload %s, %d fields, warmup %d, steps %d" % (args.workload, n_fields, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    tot = dict(node_updates=0, stencil_evals=0, outer_iters=0, nodes=0)
    adj = dict(lambda_updates=0, outer_iters=0, ms=0.0, fwd_ms=0.0)
    wall_rays = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st, tfa, tr = step()
        f = st["forward"]
        for key in tot:
            tot[key] += f[key]
        for key in ("lambda_updates", "outer_iters", "ms"):
            adj[key] += st[key]
        adj["fwd_ms"] += f["ms"]
        wall_rays += tr
        print("bench: step %d done, %d + %d passes, forward %.2f ms, forward+adjoint %.2f ms, rays %.2f ms"
              % (k, f["outer_iters"], st["outer_iters"], f["ms"], st["ms"], tr * 1e3), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    line.update({
        "value": tot["node_updates"] / el,
        "ms_per_step": el * 1e3 / args.steps,
        "fwd_adj_field_solves_per_s": n_fields * args.steps / el,
        "rays_per_s": n_rays * args.steps / el if n_rays else None,
        "solved_nodes_per_s": tot["nodes"] / el,
        "redundancy_updates_per_node": tot["node_updates"] / max(tot["nodes"], 1),
        "stencil_estimates_per_update": tot["stencil_evals"] / max(tot["node_updates"], 1),
        "forward_ms_per_step": adj["fwd_ms"] / args.steps,
        "adjoint_ms_per_step": (adj["ms"] - adj["fwd_ms"]) / args.steps,
        "rays_ms_per_step": wall_rays * 1e3 / args.steps,
        "relax_passes_per_step": tot["outer_iters"] / args.steps,
        "adjoint_lambda_updates_per_node": adj["lambda_updates"] / max(tot["nodes"], 1),
        "adjoint_passes_per_step": adj["outer_iters"] / args.steps,
    })

    # the relaxation kernel against its roofs: one more (untimed) call, passes launched one
    # by one with HIP events around each relax launch
    line["roofline"] = relax_roofline(solver, roof_call)

    if args.workload == "weld512x64":
        # the plain single-field solver on the same GPU (one top source of the same weld)
        single = torch.empty((1, m.nz, m.nx), dtype=torch.float32, device=dev)
        src1 = [m.sources[len(m.sources) // 2]]
        solver.solve(m.h, m.mats, mid, ori, src1, out=single)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, sst = solver.solve(m.h, m.mats, mid, ori, src1, out=single)
        single_ms = (time.perf_counter() - ts) * 1e3
        line["single_field_solve"] = {"ms": single_ms, "fields_per_s": 1e3 / single_ms, "passes": sst["outer_iters"]}

        if not args.no_extras:
            # the other modes on the same weld and sources: a warm-up call, then the faster of
            # two timed calls (a mode's first calls can include one-off host work)
            def timed(fn):
                fn()
                best = float("inf")
                for _ in range(2):
                    torch.cuda.synchronize()
                    ts = time.perf_counter()
                    fn()
                    torch.cuda.synchronize()
                    best = min(best, (time.perf_counter() - ts) * 1e3)
                return best

            srcs, recs = m.sources, m.receivers
            xo = torch.empty_like(out)      # the step's fields in `out` stay for the check below
            line["extras"] = {
                "forward_box_ms": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo)),
                "forward_nested_source_grids_ms": timed(lambda: solver.solve_refined(m.h, m.mats, mid, ori, srcs,
                                                                                     out=xo)),
                "forward_subgrid3_ms": timed(lambda: solver.solve_refined(m.h, m.mats, mid, ori, srcs, out=xo,
                                                                          subgrid=3)),
                "forward_sh_ms": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo, wave="sh")),
                "forward_velocity_table_ms": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo,
                                                                        velocity="table")),
                "misfit_gradient_ms": timed(lambda: solver.misfit_gradient(m.h, m.mats, mid, ori, srcs, recs, obs)),
                "misfit_gradient_with_stiffness_ms": timed(lambda: solver.misfit_gradient(
                    m.h, m.mats, mid, ori, srcs, recs, obs, stiffness=True)),
                "rays_changing_family_ms": timed(lambda: solver.trace_rays(m.h, m.mats, mid, ori, out, srcs, recs)),
                "rays_fastest_fixed_family_ms": timed(lambda: solver.trace_rays(m.h, m.mats, mid, ori, out, srcs,
                                                                                recs, planes="fastest")),
            }

    if not args.no_check:
        import oracle
        if args.workload == "weld512x64":
            k, mm, Tg = 0, m, out[0]
        else:
            # the median-size medium, first source: rerun its forward alone (same fixed point)
            order = np.argsort([md.nx for md in media])
            kk = int(order[len(order) // 2])
            mm = media[kk]
            Tk, _ = solver.solve(mm.h, mm.mats, torch.from_numpy(mm.mat_id).to(dev),
                                 torch.from_numpy(mm.orient).float().to(dev), [mm.sources[0]])
            k, Tg = 0, Tk[0]
        Tref = oracle.solve_fmm(mm.h, mm.mats, mm.mat_id, mm.orient, mm.sources[k], 2)
        mask = Tref > 0
        rel = np.abs(Tg.cpu().numpy().astype(np.float64) - Tref)[mask] / Tref[mask]
        line["max_rel_err_vs_oracle"] = float(rel.max())
        line["checked"] = "%s source %d" % (getattr(mm, "name", "medium"), k)

    if not args.no_cpu_baseline:
        import oracle
        # bounded sample of the same step on the host: one field (forward with its update
        # count, then the oracle's adjoint, which solves the field again) and, for the weld,
        # 8 of its 64 rays scaled up to all receivers
        if args.workload == "weld512x64":
            mm, k, o = m, len(m.sources) // 2, obs_np
        else:
            order = np.argsort([md.nx for md in media])
            kk = int(order[len(order) // 2])
            mm, k = media[kk], 0
            o = straight_ray_obs(mm.sources, mm.receivers, mm.h)
        src = mm.sources[k]
        t0 = time.perf_counter()
        T, n_upd = oracle.solve_fmm_counted(mm.h, mm.mats, mm.mat_id, mm.orient, src, 2)
        g = np.zeros_like(T)
        for r, rec in enumerate(mm.receivers):
            g[rec[1], rec[0]] += T[rec[1], rec[0]] - float(np.float32(o[k, r]))
        oracle.adjoint(mm.h, mm.mats, mm.mat_id, mm.orient, src, g)
        t_fa = time.perf_counter() - t0
        t_rays = 0.0
        ray_sample = []
        if args.workload == "weld512x64":
            ray_sample = mm.receivers[::8]
            t0 = time.perf_counter()
            for rec in ray_sample:
                oracle.trace_ray(mm.h, mm.mats, mm.mat_id, mm.orient, T, src, rec)
            t_rays = (time.perf_counter() - t0) * len(mm.receivers) / len(ray_sample)
        per_field = t_fa + t_rays
        line["cpu_baseline"] = {"value": n_upd / per_field, "unit": "node-updates/s", "cores": 1,
                                "kind": "oracle", "fwd_adj_field_solves_per_s": 1.0 / per_field,
                                "forward_adjoint_s": t_fa, "rays_s_extrapolated": t_rays,
                                "sample": "one %dx%d field: FP64 heap FMM forward + adjoint (re-solving the field)%s; "
                                          "single thread" % (mm.nx, mm.nz,
                                                             (" + %d of its %d rays, scaled to all"
                                                              % (len(ray_sample), len(mm.receivers)))
                                                             if ray_sample else "")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
