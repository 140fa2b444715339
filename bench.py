#!/usr/bin/env python3
"""Benchmark: batched SUR GLS solves/s, mixed precision vs plain FP64 PCG-Aug.

Workload: 512 independent SUR instances (G ~ U{4..32}, M ~ U{500..5000},
n_i ~ U{3..20}, K = 16 right-hand sides each; X_i intercept + N(0,1),
Omega = A A^T + 0.1 I), seeded synthetic data drawn on the host and resident
in HBM before timing.  One step = factor (batched Householder QR) + solve of
all 8,192 (instance, rhs) pairs.  `value` is the mixed-precision throughput;
the FP64 path is timed on the same inputs and both are checked against the
CPU oracle on a sample of instances at <= 1e-10 relative error.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SUR GLS solves/s: batched mixed-prec vs plain FP64 PCG at ≤1e-10 rel err"
HBM_PEAK_GBS = 8000.0
# HBM traffic of the projection passes measured with rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE, calibrated against a plain copy kernel); valid only
# for the kernel sources it was taken from
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_proj_sur_batch512_k16.json")
KERNEL_SOURCES = ["paper_2510_14471_amd/csrc/proj.hip", "paper_2510_14471_amd/csrc/api.hip",
                  "paper_2510_14471_amd/csrc/glm_internal.h", "paper_2510_14471_amd/csrc/reduce.hip",
                  "paper_2510_14471_amd/csrc/qr_panel.h"]
PASS_NAMES = {0: "k_proj_a<float> (pass A: u <- g + mu u, B = U Omega, d = u.B, T += Q^T B)",
              1: "k_proj_b<float> (pass B: g -= (lambda/alpha)(B - Q T), w -= lambda u, c = g.g)",
              2: "k_red_gemm_tn (model reduction: reduced responses Y_red = Q1^T Y, "
                 "Q1 = first n + 1 columns of the Q of W = [X_1 ... X_G])"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel(a, b):
    import numpy as np
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--check", type=int, default=12, help="instances checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-unreduced", action="store_true",
                    help="skip the runs without the model reduction")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the batched solver has no multi-GPU path in "
              "this build (instances would shard across GPUs without communication); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_14471_amd as glm
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    batch = synth.config2(B=args.instances)
    insts = list(batch)
    log(f"generated {len(insts)} instances in {time.time() - t0:.1f}s")
    lay, d = glm.pack_instances(insts)
    torch.cuda.synchronize()
    n_solves = lay.n_rhs
    log(f"packed: X {d['X'].numel() * 8 / 1e9:.2f} GB, y {d['y'].numel() * 8 / 1e9:.2f} GB")

    def timed(solver, steps, profile=False):
        if profile:
            solver.profile(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        iters = 0
        outer = 0
        for _ in range(steps):
            solver.factor(d["X"])
            beta, u, _, info, _ = solver.solve(d["Omega"], d["y"], tol=args.tol)
            st = solver.stats()
            iters += st["pcg_iterations"]
            outer += st["outer_steps"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        prof = None
        if profile:
            prof = {k: solver.profile_read(k) for k in PASS_NAMES}
            solver.profile(False)
        return dt, iters, outer, beta, u, info, prof

    # the product path (model reduction: one QR of W, the iteration on n + 1
    # rotated rows) and the iteration on all M rows, each in mixed precision
    # and in plain FP64
    runs = [("mixed", True), ("fp64", True)]
    if not args.no_unreduced:
        runs += [("mixed", False), ("fp64", False)]
    if args.no_fp64:
        runs = [r for r in runs if r[0] == "mixed"]
    results = {}
    for prec, red in runs:
        key = prec + ("" if red else "_unreduced")
        s = glm.SURSolver(lay, prec, reduce=red)
        log(f"{key}: workspace {s.workspace_bytes / 1e9:.2f} GB")
        for _ in range(args.warmup):
            timed(s, 1)
        dt, iters, outer, beta, u, info, prof = timed(s, args.steps, profile=(prec == "mixed"))
        infos = info.cpu().numpy()
        results[key] = dict(dt=dt, iters=iters, outer=outer, beta=beta, u=u,
                            ok=int(np.sum((infos == 0) | (infos == 1))), prof=prof)
        log(f"{key}: {args.steps} steps in {dt:.3f}s -> {n_solves * args.steps / dt:.1f} solves/s,"
            f" {iters / args.steps:.0f} PCG iterations/step, outer {outer / args.steps:.1f},"
            f" ok {results[key]['ok']}/{n_solves}")
        s.close()
        del s
        torch.cuda.empty_cache()

    # accuracy against the oracle on a sample of instances
    from oracle import gls as ogls
    errs = {}
    sample = list(range(0, len(insts), max(1, len(insts) // max(1, args.check))))[: args.check]
    ref = {b: ogls.sur_gls(insts[b]) for b in sample}
    for prec, r in results.items():
        betas = glm.unpack(lay, r["beta"], "beta")
        us = glm.unpack(lay, r["u"], "u")
        eb = eu = 0.0
        for b in sample:
            beta_o, U_o = ref[b]
            for k in range(insts[b].K):
                eb = max(eb, rel(betas[b][:, k], beta_o[:, k]))
                eu = max(eu, rel(us[b][:, :, k], U_o[:, :, k]))
        errs[prec] = (eb, eu)
        log(f"{prec}: max rel err on {len(sample)} instances: beta {eb:.2e}, u {eu:.2e}")

    mixed = results["mixed"]
    value = n_solves * args.steps / mixed["dt"]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * mixed["dt"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"sur_batch{len(insts)}_K16: G~U{{4..32}}, M~U{{500..5000}}, "
                               "n_i~U{3..20}, Omega=AA^T+0.1I; step = model reduction (QR of "
                               "W = [X_1..X_G], rotation of Y) + per-block QR + solve of all "
                               "(instance, rhs), u of the full model",
                   "instances": len(insts), "solves_per_step": n_solves, "tol": args.tol},
        "pcg_iterations_per_s": round(mixed["iters"] / mixed["dt"], 1),
        "outer_steps": round(mixed["outer"] / args.steps, 2),
        "max_rel_err": {p: {"beta": e[0], "u": e[1]} for p, e in errs.items()},
        "converged": {p: f"{r['ok']}/{n_solves}" for p, r in results.items()},
    }
    if "fp64" in results:
        f64 = results["fp64"]
        v64 = n_solves * args.steps / f64["dt"]
        out["fp64_solves_per_s"] = round(v64, 2)
        out["speedup_mixed_vs_fp64"] = round(value / v64, 3)
        out["fp64_pcg_iterations_per_s"] = round(f64["iters"] / f64["dt"], 1)
    if "mixed_unreduced" in results:
        un = {"mixed_solves_per_s": round(n_solves * args.steps / results["mixed_unreduced"]["dt"], 2),
              "pcg_iterations_per_s": round(results["mixed_unreduced"]["iters"] /
                                            results["mixed_unreduced"]["dt"], 1)}
        if "fp64_unreduced" in results:
            un["fp64_solves_per_s"] = round(n_solves * args.steps / results["fp64_unreduced"]["dt"], 2)
            un["speedup_mixed_vs_fp64"] = round(un["mixed_solves_per_s"] / un["fp64_solves_per_s"], 3)
        rl = roofline(results["mixed_unreduced"]["prof"], reduced=False)
        if rl:
            un["roofline"] = rl[0]
        out["without_model_reduction"] = un
    rl = roofline(mixed["prof"], reduced=True)
    if rl:
        out["roofline"], others = rl
        if others:
            out["roofline_other"] = others
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel_path in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel_path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(pass_id, reduced):
    """HBM bytes per launch of the timed kernel from the committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != kernel_sources_sha256():
        return None
    k = t.get("passes", {}).get(("r" if reduced else "") + str(pass_id))
    return None if k is None else k.get("hbm_bytes_per_launch")


def roofline(prof, reduced):
    """(roofline of the kernel with the most timed milliseconds, the others)."""
    if not prof:
        return None
    timed_ids = [k for k in PASS_NAMES if prof.get(k) and prof[k][0] and prof[k][1] > 0]
    if not timed_ids:
        return None
    kid = max(timed_ids, key=lambda k: prof[k][1])
    n_l, ms, by = prof[kid]
    ach = (by / n_l) / (ms / n_l * 1e-3) / 1e9
    main_rl = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kid, reduced),
               "kernel": PASS_NAMES[kid], "launches": n_l, "avg_us": round(1000 * ms / n_l, 2),
               "alg_bytes_per_launch": round(by / n_l)}
    others = []
    for k in timed_ids:
        if k != kid:
            n2, ms2, by2 = prof[k]
            others.append({"kernel": PASS_NAMES[k], "launches": n2,
                           "avg_us": round(1000 * ms2 / n2, 2),
                           "achieved": round((by2 / n2) / (ms2 / n2 * 1e-3) / 1e9, 1),
                           "share_of_timed_ms": round(ms2 / sum(prof[j][1] for j in timed_ids), 3)})
    main_rl["share_of_timed_ms"] = round(ms / sum(prof[j][1] for j in timed_ids), 3)
    return main_rl, others


def cpu_baseline(insts, budget_s):
    """The oracle (textbook SUR GLS by Cholesky, NumPy/LAPACK) on the host cores,
    on the first instances of the same workload until ~budget_s of work."""
    import numpy as np
    from oracle import gls as ogls
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    t = time.perf_counter()
    solves = 0
    done = 0
    for inst in insts:
        ogls.sur_gls(inst)
        solves += inst.K
        done += 1
        if time.perf_counter() - t > budget_s:
            break
    dt = time.perf_counter() - t
    return {"value": round(solves / dt, 2), "unit": "solves/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"first {done} of {len(insts)} instances ({solves} solves), {dt:.1f}s"}


if __name__ == "__main__":
    main()
