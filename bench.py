"""Benchmark: TDVP site updates/s of the FP64 TTNS one-site TDVP step on one
MI355X, with the roofline of the dominant kernel and the CPU oracle beside it.

A step is one second-order TDVP step of the whole tree (pre-order sweep with
h = dt/2 and its adjoint post-order sweep: every node evolved, every bond
evolved backward, the QR / environment / absorb work of every centre move,
and the observables of the step), i.e. 2 * n_nodes site updates.

Default workload: the five-level vibronic tree (4 chains x 40 sites, local
dimension 20, bond dimension 20, dt = 0.5 fs), synthetic seeded parameters.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 (vector and matrix): 256 CU x 128 flop/clk x 2.4 GHz

WORKLOADS = {
    "vibronic": (W.vibronic_reference,
                 "five-level vibronic tree: 4 Ohmic chains x 40 sites, d=20, D=20, wc=0.2 eV, "
                 "dt=0.5 fs, seed 2"),
    "spin_boson": (W.spin_boson_reference,
                   "spin-boson: 1 Ohmic chain x 10 sites, d=10, D=8, alpha=0.1, dt=0.05"),
    "large_er": (W.large_tree,
                 "five-level root, ER tree of 6 nodes, 8 chains x 100 sites, d=30, D=48, seed 4"),
}


def cpu_baseline(model, seconds=20.0):
    """The oracle, timed on the host cores on a bounded sample of the same
    workload: whole TDVP steps until ~``seconds`` of CPU work."""
    from threadpoolctl import threadpool_info
    from oracle.model import build_tree
    from oracle.ttns import TTNS
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    tt = TTNS(build_tree(model), krylov=model.get("krylov", 12))
    steps = 0
    t0 = time.perf_counter()
    while True:
        tt.step(model["dt"])
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    upd = 2 * tt.n * steps
    return {"value": upd / el, "unit": "site updates/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d full TDVP step(s) of the same workload (%d site updates) in %.1f s"
                      % (steps, upd, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="vibronic", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the TDVP sweep of one tree is sequential and this "
              "library does not shard it across GPUs (pass --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_01362_amd import ttns as T

    make, desc = WORKLOADS[args.workload]
    model = make()
    n_nodes = W.node_count(model)
    upd_per_step = 2 * n_nodes
    total = args.warmup + args.steps + args.profile_steps + 1
    ctx = T.Context([model], opts=T.default_opts(record_capacity=total + 1))
    dt = model["dt"]

    ctx.ttns_tdvp_step(dt, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ttns_tdvp_step(dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0

    # dominant kernel (the H_eff contraction inside Lanczos): HIP events
    # around each of its launches over extra steps of the same run
    ctx.profile(True)
    ctx.ttns_tdvp_step(dt, args.profile_steps)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    torch.cuda.synchronize()
    h = ctx.history()
    drift = {"norm": float(np.abs(h["norm"] - 1).max()),
             "energy": float(np.abs(h["energy"] - h["energy"][0]).max())}
    ctx.close()

    achieved = prof["flops_per_launch"] / (prof["avg_ms"] * 1e-3) / 1e12 if prof["avg_ms"] > 0 else 0.0
    out = {
        "metric": "TDVP site updates/s + % MFMA peak vs FP64 plain at ≤1e-6 population error",
        "value": upd_per_step * args.steps / el,
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "nodes": n_nodes, "site_updates_per_step": upd_per_step,
                   "krylov": model["krylov"], "executor": "wide kernels in one HIP graph per step"},
        "roofline": {"bound": "alu", "kernel": "k_op<OP_APPLY_LZ> (H_eff apply in Lanczos)",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "avg_launch_ms": prof["avg_ms"], "launches": prof["launches"],
                     "flops_per_launch": prof["flops_per_launch"]},
        "drift": drift,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
