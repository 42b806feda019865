"""Benchmark: batched anisotropic travel-time fields on one MI355X.

One step = one pass of the hot path over one batch: the 512x512 synthetic V-weld with 64
top-surface sources solved in one batched relaxation (the paper's forward modeller,
Sections 2-4), then the 64 x 64 ray paths from 64 bottom receivers to every source
through those fields (Section 5.1); float32 output, inputs resident in HBM.

Prints one JSON line.  `value` is node updates per second (one update = one evaluation
of the local ALI update at one node).  Alongside: fields/s, solved nodes/s, redundancy,
the relaxation kernel's position against its roof (HIP events around each launch), the
accuracy of the last step against the FP64 oracle, and the oracle itself timed on a
bounded sample on the host (cpu_baseline).
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

    def step():
        _, st = solver.solve(m.h, m.mats, mid, ori, m.sources, out=out)
        tr = None
        if rays:
            tr = solver.trace_rays(m.h, m.mats, mid, ori, out, m.sources, m.receivers)
        return st, tr

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    tot = dict(node_updates=0, stencil_evals=0, outer_iters=0, relax_ms=0.0, nodes=0, tile_visits=0)
    t0 = time.perf_counter()
    for k in range(args.steps):
        st, tr = step()
        for key in tot:
            tot[key] += st[key]
        print("bench: step %d done, %d passes, %.2f ms" % (k, st["outer_iters"], st["ms"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

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
        "dtype": "f32 wavefront math, f64 travel times",
        "data": "synthetic",
        "config": {"workload": "V-weld %dx%d, h=%.1f mm, %d top sources: batched forward solve + %d x %d ray paths"
                               % (m.nx, m.nz, m.h * 1e3, len(m.sources), len(m.sources), len(m.receivers)),
                   "grid": [m.nz, m.nx], "fields_per_step": len(m.sources), "src_box_radius": 2},
        "fields_per_s": n_fields / el,
        "rays_per_s": (len(m.sources) * len(m.receivers) * args.steps / el) if rays else None,
        "solved_nodes_per_s": tot["nodes"] / el,
        "redundancy_updates_per_node": tot["node_updates"] / max(tot["nodes"], 1),
        "stencil_estimates_per_update": tot["stencil_evals"] / max(tot["node_updates"], 1),
        "relax_launches_per_step": tot["outer_iters"] / args.steps,
        "relax_kernel_ms_per_step": tot["relax_ms"] / args.steps,
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
        # bounded sample: the FP64 heap oracle on a few of the step's fields, one thread
        sample = [0, len(m.sources) // 2, len(m.sources) - 1][: max(1, min(3, len(m.sources)))]
        t0 = time.perf_counter()
        upd = 0
        for k in sample:
            _, n_upd = oracle.solve_fmm_counted(m.h, m.mats, m.mat_id, m.orient, m.sources[k], 2)
            upd += n_upd
        ct = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": upd / ct, "unit": "node-updates/s", "cores": 1,
                                "kind": "oracle", "fields_per_s": len(sample) / ct,
                                "sample": "%d of the %d fields (sources %s), FP64 heap FMM, single thread"
                                          % (len(sample), len(m.sources), sample)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
