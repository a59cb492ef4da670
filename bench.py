"""Benchmark: layered-media FMM matvecs per second on one MI355X.

Workload (default): three-layer medium d = (0, -1), eps = (1, 5, 2), N = 1,048,576
charges uniform in the three layer boxes, p = 10, one charge vector; inputs are
resident in HBM before the timed region.  A step is one fmm_layered_eval (free
space + all 16 reaction components).  Prints one JSON line.
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

METRIC = "FMM matvecs/sec at N=1M 3-layer p=10 vs plain FP64 GPU FMM at <=1e-5 rel error"
PEAK_FP64 = 78.6e12  # MI355X vector FP64, FLOP/s


def stage_flops(stats, p, stage):
    """Algorithmic floating-point work of one launch of a stage (see the design notes)."""
    nc = (p + 1) * (p + 2) // 2
    full = (p + 1) ** 2
    if stage == "m2l":
        return 8.0 * nc * full * (stats["m2l_free_pairs"] + stats["m2l_reaction_pairs"])
    if stage == "p2p_free":
        return 11.0 * stats["p2p_free_pairs"]
    if stage == "p2p_reaction":
        return 2.0 * stats["p2p_reaction_pairs"]
    if stage in ("p2m", "l2p"):
        return 10.0 * full * stats["n_tree_points"]
    if stage in ("m2m", "l2l"):
        return 2.0 * (p + 1) ** 4 * stats["n_boxes"]
    return 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--leaf-cap", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=8, help="oracle targets for the CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a "
              "design note, not a build target", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1908_10863_amd import fmmlm, workloads

    w = workloads.config(args.workload)
    p = args.p or w["p"]
    cap = args.leaf_cap or 64
    dev = torch.device("cuda:0")
    print(f"[bench] workload {w['name']} N={len(w['x'])} p={p} leaf_cap={cap}", file=sys.stderr,
          flush=True)
    plan = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=p, leaf_cap=cap)
    st = plan.stats()
    print(f"[bench] plan {st['plan_seconds']:.2f}s boxes={st['n_boxes']} m2l={st['m2l_free_pairs']}"
          f"+{st['m2l_reaction_pairs']} p2p={st['p2p_free_pairs']}", file=sys.stderr, flush=True)
    q = torch.tensor(w["q"][0], dtype=torch.float64, device=dev)
    out = torch.empty_like(q)
    for _ in range(args.warmup):
        plan.eval(q, out=out)
    torch.cuda.synchronize()
    plan.profile_begin(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.eval(q, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, nrec = plan.profile_end()
    phi = out.cpu().numpy()
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    avg = {k: v / max(nrec, 1) for k, v in stage_ms.items()}
    dom = max((k for k in avg if stage_flops(st, p, k) > 0), key=lambda k: avg[k])
    flops = stage_flops(st, p, dom)
    achieved = flops / (avg[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64 / 1e12), "traffic": None,
                "flops_per_launch": flops, "avg_ms": avg[dom]}
    print(f"[bench] {value:.2f} matvec/s, stages(ms) " +
          ", ".join(f"{k}={v:.3f}" for k, v in avg.items()), file=sys.stderr, flush=True)

    # CPU baseline: the oracle on a bounded sample of targets of the same workload
    import oracle
    rng = np.random.default_rng(0)
    tgt = np.sort(rng.choice(len(w["x"]), args.cpu_sample, replace=False))
    c0 = time.perf_counter()
    ref = oracle.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0],
                           targets=tgt)
    ct = time.perf_counter() - c0
    n = len(w["x"])
    cpu = {"value": (len(tgt) / n) / ct, "unit": "matvec/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{len(tgt)} targets x {n} sources, direct sum (image-series reaction "
                     f"kernels), {ct:.1f} s"}
    err = float(np.linalg.norm(phi[tgt] - ref) / np.linalg.norm(ref))

    rec = {
        "metric": METRIC, "value": value, "unit": "matvec/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["name"], "n": n, "p": p, "layers": 3, "leaf_cap": cap,
                   "precision": "fp64", "rhs": 1},
        "roofline": roofline, "cpu_baseline": cpu,
        "rel_error_vs_oracle": err,
        "stage_ms": avg, "plan_seconds": st["plan_seconds"],
        "counts": {k: st[k] for k in ("n_boxes", "n_leaves", "m2l_free_pairs", "m2l_reaction_pairs",
                                      "p2p_free_pairs", "p2p_reaction_pairs", "max_level")},
    }
    plan.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
