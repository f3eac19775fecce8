"""Benchmark: TDVP site updates/s of the TTNS one-site TDVP step on one
MI355X, with the roofline of the dominant kernel and the CPU oracle beside it.

A step is one second-order TDVP step of the whole tree (pre-order sweep with
h = dt/2 and its adjoint post-order sweep: every node evolved, every bond
evolved backward, the QR / environment / absorb work of every centre move,
and the observables of the step), i.e. 2 * n_nodes site updates per tree.

Default workload: the five-level vibronic tree (4 chains x 40 sites, local
dimension 20, bond dimension 20, dt = 0.5 fs), synthetic seeded parameters,
FP64.  The cost of a step grows along a trajectory (the Lanczos processes of
chain sites still in their vacuum stop after one iteration early on), so the
benchmark runs the workload's whole job from t = 0 and times K of its steps
spread evenly over it (step floor(i * job / K) for i < K), each bracketed by
device synchronisations, with the inputs resident in HBM: their mean is the
job's mean step time.  W warm-up steps run first on a separate context.  The
per-kernel figures come from a few profiled steps spread over the job (one
launch at a time, HIP events around each launch on the library's stream);
the trajectory is compared with the oracle's stored one where it exists.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision fp64|fp32|bf16x3] [--job STEPS]
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

# MI355X published peaks
PEAK = {"fp64": 78.6, "fp32_mfma": 157.3, "bf16_mfma": 2500.0, "hbm_gbs": 8000.0}

WORKLOADS = {
    "vibronic": (lambda: [W.vibronic_reference()],
                 "five-level vibronic tree: 4 Ohmic chains x 40 sites, d=20, D=20, wc=0.2 eV, "
                 "dt=0.5 fs, seed 2"),
    "spin_boson": (lambda: [W.spin_boson_reference()],
                   "spin-boson: 1 Ohmic chain x 10 sites, d=10, D=8, alpha=0.1, dt=0.05"),
    "large_er": (lambda: [W.large_tree()],
                 "five-level root, ER tree of 6 nodes, 8 chains x 100 sites, d=30, D=48, seed 4"),
    "ensemble": (lambda: W.ensemble(),
                 "256 uneven spin-boson trees (L 20..120, d 8/16/24, D 8/16/32), one persistent "
                 "launch per step, seed 3"),
}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
# length of each workload's job (steps from t = 0)
JOB = {"vibronic": 400, "spin_boson": 200, "large_er": 200, "ensemble": 100}
# the oracle's stored trajectory of a workload (tests/golden)
GOLDEN = {"vibronic": "five_level_tree_fp64_400.npz"}


def cpu_baseline(models, seconds=20.0):
    """The oracle, timed on the host cores on a bounded sample of the same
    workload: whole TDVP steps (of the first tree) until ~``seconds``."""
    from threadpoolctl import threadpool_info
    from oracle.model import build_tree
    from oracle.ttns import TTNS
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    model = models[0]
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
            "sample": "%d full TDVP step(s) of tree 0 of the same workload (%d site updates) in %.1f s"
                      % (steps, upd, el)}


def roofline_of(kid, k, prec):
    """Bound, achieved and peak of one kernel from its live totals."""
    secs = k["ms"] * 1e-3
    fl, by = k["flops"], k["bytes"]
    if kid in (16, 17, 18):  # matrix-core groups
        if kid == 16:
            peak, unit, achieved = PEAK["fp64"], "TFLOP/s", fl / secs / 1e12
        elif kid == 17:
            peak, unit, achieved = PEAK["fp32_mfma"], "TFLOP/s", fl / secs / 1e12
        else:  # three bf16 products per real product
            peak, unit, achieved = PEAK["bf16_mfma"], "TFLOP/s", 3 * fl / secs / 1e12
        bound = "mfma"
    else:
        intensity = fl / by if by else 0.0
        if intensity >= PEAK["fp64"] * 1e12 / (PEAK["hbm_gbs"] * 1e9):
            bound, peak, unit, achieved = "alu", PEAK["fp64"], "TFLOP/s", fl / secs / 1e12
        else:
            bound, peak, unit, achieved = "hbm", PEAK["hbm_gbs"], "GB/s", by / secs / 1e9
    return {"bound": bound, "kernel": k["name"], "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "avg_launch_ms": k["ms"] / k["launches"],
            "launches": k["launches"], "flops_per_launch": fl / k["launches"],
            "bytes_per_launch": by / k["launches"], "share_of_step_time": None}


def sample_positions(job, k):
    """Job step (0-based) of each of the k timed steps: spread evenly over
    the job; beyond one job's length, whole further jobs from t = 0."""
    if k <= job:
        return [(i * job) // k for i in range(k)]
    return [i % job for i in range(k)]


def pop_error(hist, golden_path, n):
    """Largest |P_j(t_k) - P_j^oracle(t_k)| over the first n records."""
    g = np.load(golden_path, allow_pickle=False)
    pg = np.einsum("kjj->kj", hist["rdm"][:n]).real
    po = np.einsum("kjj->kj", g["rdm"][:n]).real
    return float(np.abs(pg - po).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps, spread over the job")
    ap.add_argument("--warmup", type=int, default=2, help="untimed steps on a separate context first")
    ap.add_argument("--workload", default="vibronic", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC))
    ap.add_argument("--job", type=int, default=None, help="job length in steps (default: the workload's)")
    ap.add_argument("--profile-steps", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--executor", default="auto", choices=["auto", "wide", "persistent"])
    ap.add_argument("--autotune", action="store_true",
                    help="time the H_eff and QR variants at build and plan the fastest")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the TDVP sweep of one tree is sequential and this "
              "library does not shard it across GPUs (pass --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_01362_amd import ttns as T

    make, desc = WORKLOADS[args.workload]
    job = args.job if args.job is not None else JOB[args.workload]
    models = make()
    upd_per_step = sum(2 * W.node_count(m) for m in models)
    flags = T.TTNS_FLAG_AUTOTUNE if args.autotune else 0
    ex = {"auto": T.TTNS_EXEC_AUTO, "wide": T.TTNS_EXEC_WIDE, "persistent": T.TTNS_EXEC_PERSISTENT}[args.executor]
    persistent = args.executor == "persistent" or (args.executor == "auto" and len(models) > 1)
    dt = models[0]["dt"]
    opts = dict(record_capacity=job + 1, executor=ex, precision=PREC[args.precision], flags=flags)

    if args.warmup > 0:  # code loading, graph instantiation, caches
        wctx = T.Context(models, opts=T.default_opts(**opts))
        for i in range(args.warmup):
            wctx.ttns_tdvp_step(dt, 1)
            torch.cuda.synchronize()
        wctx.close()
        print("warm-up: %d steps" % args.warmup, file=sys.stderr, flush=True)

    timed = sample_positions(job, args.steps)
    n_jobs = (args.steps + job - 1) // job
    n_prof = 0 if persistent else min(args.profile_steps, job)
    # profiled steps sit between the timed ones (first job only)
    prof_at = sorted(set(((2 * i + 1) * job) // (2 * n_prof) for i in range(n_prof)) - set(timed))
    el = 0.0
    t_build = 0.0
    kern = None
    hist = None
    step_flops = 0.0
    for jn in range(n_jobs):
        tb = time.perf_counter()
        ctx = T.Context(models, opts=T.default_opts(**opts))
        torch.cuda.synchronize()
        t_build = time.perf_counter() - tb
        step_flops = sum(ctx.step_flops(i)[0] for i in range(len(models)))
        mine = [p for i, p in enumerate(timed) if i // job == jn] if args.steps > job else timed
        last = job - 1 if jn == 0 else max(mine)  # the first job runs to its end
        for pos in range(last + 1):
            if pos in mine:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.ttns_tdvp_step(dt, 1)
                torch.cuda.synchronize()
                el += time.perf_counter() - t0
            elif jn == 0 and pos in prof_at:
                ctx.profile(True)
                ctx.ttns_tdvp_step(dt, 1)
                ctx.profile(False)
            else:
                ctx.ttns_tdvp_step(dt, 1)
            if (pos + 1) % 50 == 0:
                torch.cuda.synchronize()
                print("job %d: step %d/%d" % (jn, pos + 1, last + 1), file=sys.stderr, flush=True)
        if jn == 0:
            if n_prof:
                kern = ctx.profile_kernels()
            hist = [ctx.history(i) for i in range(len(models))]
        ctx.close()

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
        "dtype": {"fp64": "f64", "fp32": "f32 contractions (f64 elsewhere)",
                  "bf16x3": "split-bf16 contractions (f64 elsewhere)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "trees": len(models), "site_updates_per_step": upd_per_step,
                   "krylov": models[0]["krylov"],
                   "executor": "one persistent workgroup per tree" if persistent
                   else "one kernel per operation, replayed as HIP graphs",
                   "autotuned": bool(args.autotune), "build_s": round(t_build, 2),
                   "window": "%d steps spread evenly over the %d-step job from t = 0 (steps %s)"
                             % (args.steps, job, ",".join(str(p) for p in timed[:8])
                                + (",..." if len(timed) > 8 else ""))},
        "step_tflops": step_flops / (el / args.steps) / 1e12,
    }
    if persistent:
        # one kernel per step: its own duration is the step time
        out["roofline"] = {"bound": "alu", "kernel": "ttns::k_persistent (whole step)",
                           "achieved": out["step_tflops"], "peak": PEAK["fp64"], "unit": "TFLOP/s",
                           "frac": out["step_tflops"] / PEAK["fp64"], "traffic": None,
                           "avg_launch_ms": out["ms_per_step"], "flops_per_launch": step_flops}
    elif kern:
        tot = sum(k["ms"] for k in kern.values())
        dom = max(kern, key=lambda k: kern[k]["ms"])
        out["roofline"] = roofline_of(dom, kern[dom], args.precision)
        out["roofline"]["share_of_step_time"] = kern[dom]["ms"] / tot
        out["roofline"]["profiled_steps"] = prof_at
        heff = [kid for kid in (1, 16, 17, 18) if kid in kern]
        out["heff_rooflines"] = []
        for kid in heff:
            r = roofline_of(kid, kern[kid], args.precision)
            r["share_of_step_time"] = kern[kid]["ms"] / tot
            out["heff_rooflines"].append(r)
        out["kernel_time_share"] = {kern[k]["name"]: round(kern[k]["ms"] / tot, 4)
                                    for k in sorted(kern, key=lambda k: -kern[k]["ms"])}
    h = hist[0]
    out["drift"] = {"norm": float(np.abs(h["norm"] - 1).max()),
                    "energy": float(np.abs(h["energy"] - h["energy"][0]).max()),
                    "records": int(len(h["norm"]))}
    gname = GOLDEN.get(args.workload)
    gpath = os.path.join(ROOT, "tests", "golden", gname) if gname else None
    if gpath and os.path.exists(gpath):
        n = len(h["norm"])
        out["pop_error_vs_oracle"] = {"value": pop_error(h, gpath, n), "records": n,
                                      "reference": "tests/golden/" + gname}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(models, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
