"""Benchmark: batched anisotropic travel-time fields and their misfit gradients on one
MI355X.

Workloads (one step each, inputs resident in HBM, float32 output):
  batch128 (default): 128 media of uneven sizes (square sides 256..1024, seed 3), 32 top
      sources and 32 bottom receivers each (4096 fields, 1.84e9 node-fields): forward +
      adjoint of the per-medium receiver misfit in one call (the batched tomography step),
      with the schedule picked by the autotuner (tuned once, untimed; the choice is kept
      by the handle and in a JSON cache next to the library).
  weld512x64: the 512x512 synthetic V-weld with 64 top-surface sources, solved in one
      batched relaxation (the paper's forward modeller, Sections 2-4) inside one forward +
      adjoint call for the misfit of the 64 x 64 bottom-receiver times, then the 64 x 64
      ray paths from the receivers to every source through those fields (Section 5.1).
      With the default workload its figures are reported under `extras`.

Prints one JSON line.  `value` is node updates per second of step time (one update = one
evaluation of the local ALI update at one node).  Alongside: forward+adjoint field solves
per second, solved nodes/s, redundancy, the relaxation kernel against its roofs (HIP
events around each launch of one extra, untimed solve launched pass by pass), the
accuracy of the measured batch against the FP64 oracle, and the oracle itself timed on a
bounded sample on all host cores (cpu_baseline).
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

# Algorithmic work of the relaxation kernel per node update:
#  bytes: travel time read and written (float32, 8 B), orientation (float32, 4 B),
#  material id (1 B) = 13 B.  (The mixed-arithmetic kernel keeps its working travel times
#  in float64, 21 B on the same count; the algorithm needs float32 values.)
#  operations: ordering tests of the 16 stencil pairs (96 compares), 8 straight-ray
#  candidates (40 ops), acceptance test (2) = 138, plus 47 per admissible single-stencil
#  estimate (interpolation weight, wavefront normal, phase speed with one sqrt, rsqrt,
#  causality, score and ranking); FMA counts as 2.
BYTES_PER_UPDATE = 13
OPS_PER_UPDATE = 138
OPS_PER_ESTIMATE = 47
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
# Vector ALU peak without packed FP32 (the build forbids v_pk_*_f32): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops per FMA x 2.4 GHz = 78.6 TFLOP/s, the same as FP64.
VECTOR_PEAK_TFLOPS = 78.6

# HBM traffic of the relaxation kernel from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE; each scaled by the same counter on a 256 MiB device copy in the same
# program), per launch of the batch128 forward (all launches of one forward, averaged),
# for the kernel sources with this hash, and the wave-level VALU instructions of the same
# launches (rocprofv3 --pmc SQ_INSTS_VALU).  Reported as null once the sources differ.
TRAFFIC = {"sources_sha256_16": "5d08ad48be618a41", "fetch_bytes_per_launch": 859807831,
           "write_bytes_per_launch": 84428288, "valu_wave_insts_per_launch": 1.912e8}

TUNE_CACHE = os.path.join(ROOT, "paper_2302_10988_amd", "tuned_schedules.json")


def kernel_sources_hash():
    """Hash of the sources the relaxation and scheduler kernels (forward and adjoint) are
    built from: ali_solve.hip, ali_adjoint.hip and every header of csrc."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2302_10988_amd", "csrc")
    files = [os.path.join(csrc, "ali_solve.hip"), os.path.join(csrc, "ali_adjoint.hip")]
    data = b"".join(open(p, "rb").read() for p in files + sorted(glob.glob(os.path.join(csrc, "*.hpp"))))
    return hashlib.sha256(data).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch128", choices=["batch128", "weld512x64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the weld figures and the single-call timings of the other modes (nested "
                         "source grids, SH, velocity table, stiffness gradient, fixed ray plane families)")
    ap.add_argument("--retune", action="store_true", help="ignore the tuned-schedule cache")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (known bytes, to scale HBM counters)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def straight_ray_obs(sources, receivers, h, v=5900.0):
    """Observed times of a plain synthetic target: straight rays at the parent steel's
    speed (the misfit's value does not change the work)."""
    import numpy as np
    s = np.array(sources, dtype=np.float64)
    r = np.array(receivers, dtype=np.float64)
    return np.hypot(*(s[:, None, :] - r[None, :, :]).transpose(2, 0, 1)) * h / v


def host_cores():
    """Worker threads for the oracle: this process's CPUs, at most 16 (a one-GPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def relax_roofline(call):
    """Run `call()` once (passes launched one by one, HIP events around each relax launch
    on the solver's stream) and return the relaxation kernel's position against the HBM
    and vector-ALU roofs."""
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
            "launches": launches, "updates_per_launch": f["node_updates"] / launches,
            "alu": {"achieved": tflops, "peak": VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / VECTOR_PEAK_TFLOPS},
            "valu_wave_insts_per_update": valu}


def oracle_pool(tasks, cores):
    """Run oracle tasks (callables) on `cores` threads (the oracle's C calls release the GIL);
    returns (results, wall seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(lambda f: f(), tasks))
    return res, time.perf_counter() - t0


def weld_step_figures(solver, dev, steps, warmup, extras, check):
    """The 64-source weld step (forward + adjoint + rays); returns its figures."""
    import numpy as np
    import torch

    import synthmedia as sm
    m = sm.weld_multi()
    mid = torch.from_numpy(m.mat_id).to(dev)
    ori = torch.from_numpy(m.orient).to(torch.float32).to(dev)
    out = torch.empty((len(m.sources), m.nz, m.nx), dtype=torch.float32, device=dev)
    obs_np = straight_ray_obs(m.sources, m.receivers, m.h)
    obs = torch.from_numpy(obs_np).to(torch.float32).to(dev)
    n_fields, n_rays = len(m.sources), len(m.sources) * len(m.receivers)

    def step():
        t0 = time.perf_counter()
        _, _, _, st = solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources, m.receivers, obs, T_out=out)
        t1 = time.perf_counter()
        solver.trace_rays(m.h, m.mats, mid, ori, out, m.sources, m.receivers)
        torch.cuda.synchronize()
        return st, t1 - t0, time.perf_counter() - t1

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tot_upd = tot_nodes = fwd = adj = rays = 0.0
    passes = apasses = 0
    t0 = time.perf_counter()
    for k in range(steps):
        st, tfa, tr = step()
        tot_upd += st["forward"]["node_updates"]
        tot_nodes += st["forward"]["nodes"]
        fwd += st["forward"]["ms"]
        adj += st["ms"] - st["forward"]["ms"]
        rays += tr * 1e3
        passes, apasses = st["forward"]["outer_iters"], st["outer_iters"]
    el = time.perf_counter() - t0
    res = {"workload": "V-weld %dx%d, h=%.1f mm, %d top sources x %d bottom receivers: forward + adjoint "
                       "(misfit gradient) + %d x %d ray paths" % (m.nx, m.nz, m.h * 1e3, len(m.sources),
                                                                 len(m.receivers), len(m.sources), len(m.receivers)),
           "steps": steps, "ms_per_step": el * 1e3 / steps, "node_updates_per_s": tot_upd / el,
           "fwd_adj_field_solves_per_s": n_fields * steps / el, "rays_per_s": n_rays * steps / el,
           "redundancy_updates_per_node": tot_upd / max(tot_nodes, 1),
           "forward_ms": fwd / steps, "adjoint_ms": adj / steps, "rays_ms": rays / steps,
           "forward_passes": passes, "adjoint_passes": apasses}

    # the plain single-field solver on the same GPU (one top source of the same weld)
    single = torch.empty((1, m.nz, m.nx), dtype=torch.float32, device=dev)
    src1 = [m.sources[len(m.sources) // 2]]
    solver.solve(m.h, m.mats, mid, ori, src1, out=single)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, sst = solver.solve(m.h, m.mats, mid, ori, src1, out=single)
    single_ms = (time.perf_counter() - ts) * 1e3
    res["single_field_solve"] = {"ms": single_ms, "fields_per_s": 1e3 / single_ms, "passes": sst["outer_iters"]}

    if extras:
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
        res["modes_ms"] = {
            "forward_box": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo)),
            "forward_nested_source_grids": timed(lambda: solver.solve_refined(m.h, m.mats, mid, ori, srcs, out=xo)),
            "forward_subgrid3": timed(lambda: solver.solve_refined(m.h, m.mats, mid, ori, srcs, out=xo, subgrid=3)),
            "forward_sh": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo, wave="sh")),
            "forward_velocity_table": timed(lambda: solver.solve(m.h, m.mats, mid, ori, srcs, out=xo,
                                                                 velocity="table")),
            "misfit_gradient": timed(lambda: solver.misfit_gradient(m.h, m.mats, mid, ori, srcs, recs, obs)),
            "misfit_gradient_with_stiffness": timed(lambda: solver.misfit_gradient(m.h, m.mats, mid, ori, srcs,
                                                                                   recs, obs, stiffness=True)),
            "rays_changing_family": timed(lambda: solver.trace_rays(m.h, m.mats, mid, ori, out, srcs, recs)),
            "rays_fastest_fixed_family": timed(lambda: solver.trace_rays(m.h, m.mats, mid, ori, out, srcs, recs,
                                                                         planes="fastest")),
        }
    if check:
        import oracle
        Tref = oracle.solve_fmm(m.h, m.mats, m.mat_id, m.orient, m.sources[0], 2)
        mask = Tref > 0
        rel = np.abs(out[0].cpu().numpy().astype(np.float64) - Tref)[mask] / Tref[mask]
        res["max_rel_err_vs_oracle"] = float(rel.max())
        res["checked"] = "weld source 0"
    return res, (m, mid, ori, out, obs_np, obs)


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
        log("calibration copy of %d bytes done" % (a.numel() * 4))
        del a, b

    line = {"metric": "node-updates/s & batched forward+adjoint field solves/s at ≤1e-4 rel err",
            "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 travel times, scores and decisions; f32 wavefront math and adjoint pull weights; "
                     "f64 lambda and gradient sums",
            "data": "synthetic"}

    if args.workload == "weld512x64":
        res, (m, mid, ori, out, obs_np, obs) = weld_step_figures(solver, dev, args.steps, args.warmup,
                                                                 not args.no_extras, not args.no_check)
        line["config"] = {"workload": res["workload"], "grid": [m.nz, m.nx], "fields_per_step": len(m.sources),
                          "src_box_radius": 2}
        line.update({"value": res["node_updates_per_s"], "ms_per_step": res["ms_per_step"]})
        line.update({k: v for k, v in res.items() if k not in ("workload", "steps", "node_updates_per_s",
                                                                 "ms_per_step")})
        if not args.no_roofline:
            line["roofline"] = relax_roofline(lambda: solver.misfit_gradient(m.h, m.mats, mid, ori, m.sources,
                                                                             m.receivers, obs, T_out=out,
                                                                             graph=0)[3])
        if not args.no_cpu_baseline:
            import oracle
            cores = host_cores()
            srcs = [m.sources[(k * len(m.sources)) // cores] for k in range(cores)]

            def task(src):
                def run():
                    T, n_upd = oracle.solve_fmm_counted(m.h, m.mats, m.mat_id, m.orient, src, 2)
                    k = m.sources.index(src)
                    g = np.zeros_like(T)
                    for r, rec in enumerate(m.receivers):
                        g[rec[1], rec[0]] += T[rec[1], rec[0]] - float(np.float32(obs_np[k, r]))
                    oracle.adjoint(m.h, m.mats, m.mat_id, m.orient, src, g)
                    return n_upd
                return run

            res_c, wall = oracle_pool([task(s) for s in srcs], cores)
            line["cpu_baseline"] = {"value": sum(res_c) / wall, "unit": "node-updates/s", "cores": cores,
                                    "kind": "oracle", "fwd_adj_field_solves_per_s": len(srcs) / wall,
                                    "wall_s": wall, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                                    "sample": "%d of the 64 weld fields (one per thread): FP64 heap FMM forward + "
                                              "adjoint (re-solving the field); rays not included" % len(srcs)}
        print(json.dumps(line), flush=True)
        return

    # ---- batch128 --------------------------------------------------------------------
    media = sm.batch_media()
    batch = Batch(media, device=dev)
    n_fields = batch.n_fields
    obs_np = [straight_ray_obs(md.sources, md.receivers, md.h) for md in media]
    obs = torch.from_numpy(np.concatenate([o.ravel() for o in obs_np])).to(torch.float32).to(dev)
    log("autotuning the schedule (untimed; cached per size bucket)")
    t_tune = time.perf_counter()
    tuned, tune_ms, cached = solver.autotune_batch(batch, cache_file=None if args.retune else TUNE_CACHE)
    t_tune = time.perf_counter() - t_tune
    from paper_2302_10988_amd import _lib
    sched = {k: tuned[k] for k in _lib.TUNE_KNOBS}
    sides = [md.nx for md in media]
    line["config"] = {"workload": "%d media, square sides %d..%d (seed 3), h=0.1 mm, 32 top sources x 32 bottom "
                                  "receivers each: batched forward + adjoint of the per-medium misfit"
                                  % (len(media), min(sides), max(sides)),
                      "fields_per_step": n_fields, "node_fields": batch.field_nodes, "src_box_radius": 2,
                      "schedule": sched, "schedule_from_cache": cached, "autotune_s": t_tune,
                      "autotune_ms": {"band%d_inner%d_visit%d_persistent%d" % k: v for k, v in tune_ms.items()}}

    def step():
        t0 = time.perf_counter()
        r = solver.misfit_gradient_batch(batch, obs, **sched)
        return r, time.perf_counter() - t0

    log("workload batch128, %d fields, warmup %d, steps %d" % (n_fields, args.warmup, args.steps))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    tot = dict(node_updates=0, stencil_evals=0, outer_iters=0, nodes=0, tile_visits=0)
    adj = dict(lambda_updates=0, outer_iters=0, ms=0.0, fwd_ms=0.0, tile_visits=0)
    t0 = time.perf_counter()
    for k in range(args.steps):
        (loss, trec, dth, st), tfa = step()
        f = st["forward"]
        for key in tot:
            tot[key] += f[key]
        for key in ("lambda_updates", "outer_iters", "ms", "tile_visits"):
            adj[key] += st[key]
        adj["fwd_ms"] += f["ms"]
        log("step %d done, %d + %d passes, forward %.1f ms, forward+adjoint %.1f ms"
            % (k, f["outer_iters"], st["outer_iters"], f["ms"], st["ms"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    line.update({
        "value": tot["node_updates"] / el,
        "ms_per_step": el * 1e3 / args.steps,
        "fwd_adj_field_solves_per_s": n_fields * args.steps / el,
        "solved_nodes_per_s": tot["nodes"] / el,
        "redundancy_updates_per_node": tot["node_updates"] / max(tot["nodes"], 1),
        "stencil_estimates_per_update": tot["stencil_evals"] / max(tot["node_updates"], 1),
        "forward_ms_per_step": adj["fwd_ms"] / args.steps,
        "adjoint_ms_per_step": (adj["ms"] - adj["fwd_ms"]) / args.steps,
        "relax_passes_per_step": tot["outer_iters"] / args.steps,
        "adjoint_lambda_updates_per_node": adj["lambda_updates"] / max(tot["nodes"], 1),
        "adjoint_passes_per_step": adj["outer_iters"] / args.steps,
        "tile_visits_per_pass": tot["tile_visits"] / max(tot["outer_iters"], 1),
        "updates_per_tile_visit": tot["node_updates"] / max(tot["tile_visits"], 1),
        "adjoint_tile_visits_per_pass": adj["tile_visits"] / max(adj["outer_iters"], 1),
        "adjoint_updates_per_tile_visit": adj["lambda_updates"] / max(adj["tile_visits"], 1),
    })
    trec_np = trec.cpu().numpy().astype(np.float64)

    if not args.no_roofline:
        # the relaxation kernel against its roofs: one more (untimed) call, passes launched
        # one by one with HIP events around each relax launch
        line["roofline"] = relax_roofline(lambda: solver.misfit_gradient_batch(batch, obs, graph=0, **sched)[3])

    # the plain single-field solver on the same GPU: one field of the median medium
    order = np.argsort(sides)
    kmed = int(order[len(order) // 2])
    mm = media[kmed]
    mid1 = torch.from_numpy(mm.mat_id).to(dev)
    ori1 = torch.from_numpy(mm.orient).float().to(dev)
    solver.solve(mm.h, mm.mats, mid1, ori1, [mm.sources[0]])
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, sst = solver.solve(mm.h, mm.mats, mid1, ori1, [mm.sources[0]])
    single_ms = (time.perf_counter() - ts) * 1e3
    line["single_field_solve"] = {"medium": "%dx%d" % (mm.nx, mm.nz), "ms": single_ms,
                                  "fields_per_s": 1e3 / single_ms, "passes": sst["outer_iters"]}

    if not args.no_extras:
        log("batch forward modes (extras)")
        bo = torch.empty(batch.field_nodes, dtype=torch.float32, device=dev)

        def once(fn):
            fn()            # the first call captures the pass graphs of new shapes
            torch.cuda.synchronize()
            ts = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - ts) * 1e3

        batch_modes = {"forward_box": once(lambda: solver.solve_batch(batch, out=bo, **sched)),
                       "forward_nested_source_grids": once(lambda: solver.solve_batch_refined(batch, out=bo,
                                                                                             **sched))}
        del bo
        log("weld figures (extras)")
        res, _ = weld_step_figures(solver, dev, 3, 1, True, not args.no_check)
        line["extras"] = {"weld512x64": res, "batch_forward_modes_ms": batch_modes}

    if not args.no_check:
        import oracle
        # the measured launch's receiver times, and the fields of one batched forward of the
        # same batch, against the oracle: smallest, median and largest medium, source 0
        picks = [int(order[0]), kmed, int(order[-1])]
        Tb, _ = solver.solve_batch(batch, **sched)
        views = batch.fields(Tb)
        fields_gpu = {kk: views[kk][0].cpu().numpy().astype(np.float64) for kk in picks}
        obs_off = np.cumsum([0] + [len(md.sources) * len(md.receivers) for md in media])

        def ref(kk):
            md = media[kk]
            return lambda: oracle.solve_fmm(md.h, md.mats, md.mat_id, md.orient, md.sources[0], 2)

        refs, _ = oracle_pool([ref(kk) for kk in picks], len(picks))
        errs, rerrs = [], []
        for kk, Tref in zip(picks, refs):
            md = media[kk]
            mask = Tref > 0
            errs.append(float((np.abs(fields_gpu[kk] - Tref)[mask] / Tref[mask]).max()))
            rec = np.array(md.receivers)
            tr = trec_np[obs_off[kk]: obs_off[kk] + len(md.receivers)]
            rr = Tref[rec[:, 1], rec[:, 0]]
            rerrs.append(float((np.abs(tr - rr) / rr).max()))
        line["max_rel_err_vs_oracle"] = max(errs + rerrs)
        line["checked"] = ("source 0 of media %s (sides %s): whole fields of a batched forward, and the receiver "
                           "times of the last measured step; field errors %s, receiver errors %s"
                           % (picks, [media[k].nx for k in picks], ["%.2g" % e for e in errs],
                              ["%.2g" % e for e in rerrs]))

    if not args.no_cpu_baseline:
        import oracle
        # bounded sample of the same step on the host: one field per thread (forward with
        # its update count, then the oracle's adjoint, which solves the field again), the
        # media nearest the median size
        cores = host_cores()
        near = list(order[max(0, len(order) // 2 - cores // 2):][:cores])

        def task(kk):
            md = media[kk]

            def run():
                T, n_upd = oracle.solve_fmm_counted(md.h, md.mats, md.mat_id, md.orient, md.sources[0], 2)
                g = np.zeros_like(T)
                for r, rec in enumerate(md.receivers):
                    g[rec[1], rec[0]] += T[rec[1], rec[0]] - float(np.float32(obs_np[kk][0, r]))
                oracle.adjoint(md.h, md.mats, md.mat_id, md.orient, md.sources[0], g)
                return n_upd, md.nx * md.nz
            return run

        res_c, wall = oracle_pool([task(int(kk)) for kk in near], cores)
        n_upd = sum(r[0] for r in res_c)
        nodes = sum(r[1] for r in res_c)
        line["cpu_baseline"] = {"value": n_upd / wall, "unit": "node-updates/s", "cores": cores, "kind": "oracle",
                                "fwd_adj_field_solves_per_s": len(near) / wall,
                                "step_s_extrapolated": wall * batch.field_nodes / nodes,
                                "wall_s": wall, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                                "sample": "%d fields (source 0 of the %d media nearest the median side, one per "
                                          "thread): FP64 heap FMM forward + adjoint (re-solving the field); the "
                                          "whole step extrapolated by node-fields" % (len(near), len(near))}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
