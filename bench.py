#!/usr/bin/env python3
"""Benchmark: batched SUR GLS solves/s, mixed precision vs plain FP64 PCG-Aug.

Headline workload: 512 independent SUR instances (G ~ U{4..32},
M ~ U{500..5000}, n_i ~ U{3..20}, K = 16 right-hand sides each; X_i intercept
+ N(0,1), Omega = A A^T + 0.1 I), seeded synthetic data drawn on the host and
resident in HBM before timing.  One step = the model reduction (QR of
W = [X_1 ... X_G], Q1^T Y) + the per-block QR of the reduced problem + the
solve of all 8,192 (instance, rhs) pairs + u of the full model, with the
preconditioner's D = diag(omega_ii) (x) I_M (the paper's D_2; --precond
scalar selects D = alpha I).  `value` is the mixed-precision throughput;
the FP64 path is timed on the same inputs and with the same D,
both without the reduction too, and every run is checked against the CPU
oracle on a sample of instances at <= 1e-10 relative error.

The timed steps run with kernel profiling off; one more step with profiling
on (outside the timed region) gives the HIP-event durations and algorithmic
bytes of the projection passes for the roofline.  The single large SUR
(G = 50, M = 1e4), the differentiation workload (G = 20, M = 2e4) and the
singular, restricted workload (G = 100, M = 5e4, rank G - 2, 10 restrictions)
are measured the same way through the model reduction (`configs`).  The
comparator PCG-NE (CG on the normal equations) is timed on the headline
workload (`pcg_ne`), and the Monte Carlo comparison of the two estimators
runs at 4096 replications (`montecarlo`).  The restricted VAR workload
(multivariate models with exclusions, common regressors) is timed through
its own reduction (`mvrglm`).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
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
# the pass kernels' source and the descriptor structs they read (the text of
# glm_internal.h from `struct InstDesc` to the pass constants); launcher
# declarations elsewhere in that header do not change the kernels
KERNEL_SOURCES = [("paper_2510_14471_amd/csrc/proj.hip", None, None),
                  ("paper_2510_14471_amd/csrc/glm_internal.h", "struct InstDesc",
                   "constexpr int PROJ_NT")]
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


class Runner:
    """Times factor + solve of one packed workload on one solver."""

    def __init__(self, glm, torch, lay, d, tol, precond="scalar"):
        self.glm, self.torch, self.lay, self.d, self.tol = glm, torch, lay, d, tol
        self.precond = precond

    def step(self, s):
        s.factor(self.d["X"], self.d["Rc"])
        beta, u, _, info, _ = s.solve(self.d["Omega"], self.d["y"], self.d["r"], tol=self.tol)
        return beta, u, info, s.stats()

    def run(self, prec, reduce, steps, warmup, profile):
        torch = self.torch
        s = self.glm.SURSolver(self.lay, prec, reduce=reduce, precond=self.precond)
        for _ in range(warmup):
            self.step(s)
        torch.cuda.synchronize()
        t = time.perf_counter()
        iters = outer = 0
        for _ in range(steps):
            beta, u, info, st = self.step(s)
            iters += st["pcg_iterations"]
            outer += st["outer_steps"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        prof = None
        if profile:
            # one more step with the kernel timers on, outside the timed region
            s.profile(True)
            self.step(s)
            torch.cuda.synchronize()
            prof = {k: s.profile_read(k) for k in PASS_NAMES}
            s.profile(False)
        ws = s.workspace_bytes
        s.close()
        del s
        torch.cuda.empty_cache()
        return dict(dt=dt, iters=iters, outer=outer, beta=beta, u=u, info=info, prof=prof,
                    ws=ws, steps=steps)


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
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single large, differentiation and singular workloads")
    ap.add_argument("--precond", choices=("scalar", "equation"), default="equation",
                    help="the preconditioner's D: diag(omega_ii) (x) I (equation, the paper's "
                         "D_2; 7 %% fewer PCG iterations on the batched workload) or alpha I, "
                         "alpha = max omega_ii (scalar, D_1)")
    ap.add_argument("--no-ne", action="store_true",
                    help="skip the PCG-NE comparator and the Monte Carlo study")
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
    insts = list(synth.config2(B=args.instances))
    log(f"generated {len(insts)} instances in {time.time() - t0:.1f}s")
    lay, d = glm.pack_instances(insts)
    torch.cuda.synchronize()
    n_solves = lay.n_rhs
    log(f"packed: X {d['X'].numel() * 8 / 1e9:.2f} GB, y {d['y'].numel() * 8 / 1e9:.2f} GB")
    runner = Runner(glm, torch, lay, d, args.tol, args.precond)

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
        r = runner.run(prec, red, args.steps, args.warmup, profile=(prec == "mixed"))
        infos = r["info"].cpu().numpy()
        r["ok"] = int(np.sum((infos == 0) | (infos == 1)))
        results[key] = r
        log(f"{key}: workspace {r['ws'] / 1e9:.2f} GB; {args.steps} steps in {r['dt']:.3f}s -> "
            f"{n_solves * args.steps / r['dt']:.1f} solves/s, {r['iters'] / args.steps:.0f} PCG "
            f"iterations/step, outer {r['outer'] / args.steps:.1f}, ok {r['ok']}/{n_solves}")

    # accuracy against the oracle on a sample of instances
    from oracle import gls as ogls
    errs = {}
    sample = list(range(0, len(insts), max(1, len(insts) // max(1, args.check))))[: args.check]
    ref = {b: ogls.sur_gls(insts[b]) for b in sample}
    for key, r in results.items():
        betas = glm.unpack(lay, r["beta"], "beta")
        us = glm.unpack(lay, r["u"], "u")
        eb = eu = 0.0
        for b in sample:
            beta_o, U_o = ref[b]
            for k in range(insts[b].K):
                eb = max(eb, rel(betas[b][:, k], beta_o[:, k]))
                eu = max(eu, rel(us[b][:, :, k], U_o[:, :, k]))
        errs[key] = (eb, eu)
        log(f"{key}: max rel err on {len(sample)} instances: beta {eb:.2e}, u {eu:.2e}")

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
                               "W = [X_1..X_G], Q1^T Y) + per-block QR + solve of all "
                               "(instance, rhs), u of the full model",
                   "instances": len(insts), "solves_per_step": n_solves, "tol": args.tol,
                   "preconditioner": ("D = alpha I, alpha = max omega_ii" if args.precond == "scalar"
                                      else "D = diag(omega_ii) (x) I_M")},
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
        mu = results["mixed_unreduced"]
        un = {"mixed_solves_per_s": round(n_solves * args.steps / mu["dt"], 2),
              "pcg_iterations_per_s": round(mu["iters"] / mu["dt"], 1)}
        if "fp64_unreduced" in results:
            un["fp64_solves_per_s"] = round(n_solves * args.steps / results["fp64_unreduced"]["dt"], 2)
            un["speedup_mixed_vs_fp64"] = round(un["mixed_solves_per_s"] / un["fp64_solves_per_s"], 3)
        rl = roofline(mu["prof"], traffic_key="")
        if rl:
            un["roofline"] = rl[0]
        out["without_model_reduction"] = un
    rl = roofline(mixed["prof"], traffic_key="r")
    if rl:
        out["roofline"], others = rl
        if others:
            out["roofline_other"] = others
    del runner, d
    torch.cuda.empty_cache()
    ceil = stream_ceiling(glm, torch, insts)
    if "roofline" in out:
        rl = out["roofline"]
        rl["same_mix_ceiling"] = ceil
        if rl.get("traffic"):
            touched = rl["traffic"] / (rl["avg_us"] * 1e-6) / 1e9
            rl["touched_gbs"] = round(touched, 1)
            rl["touched_frac_of_same_mix_ceiling"] = round(touched / ceil["pass_b"]["gbs"], 3)
    if not args.no_configs:
        out["configs"] = other_configs(glm, torch, synth, args)
    if not args.no_configs:
        out["mvrglm"] = mvrglm_config(glm, torch, synth, args)
    if not args.no_ne:
        out["pcg_ne"] = ne_comparator(glm, torch, synth, args)
        out["montecarlo"] = montecarlo(glm, torch, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def other_configs(glm, torch, synth, args):
    """The single large SUR, the differentiation and the singular, restricted
    workloads through the model reduction, mixed and FP64: solves/s (factor +
    solve per step), PCG iterations/s, the dominant pass's roofline and the
    error against the oracle."""
    import numpy as np
    from oracle import gls as ogls
    out = {}
    specs = [("sur_large_G50_M10000", synth.config1),
             ("sur_grad_G20_M20000", synth.config3),
             ("sur_singular_restricted_G100_M50000_k10", synth.config4)]
    for name, make in specs:
        inst = list(make())[0]
        lay, d = glm.pack_instances([inst])
        t = time.perf_counter()
        beta_o, U_o, SU_o = ogls.sur_solution(inst)
        t_oracle = time.perf_counter() - t
        runner = Runner(glm, torch, lay, d, args.tol, args.precond)
        entry = {"oracle_s": round(t_oracle, 2)}
        for prec in ("mixed", "fp64"):
            r = runner.run(prec, True, 1, 1, profile=True)
            beta = glm.unpack(lay, r["beta"], "beta")[0]
            u = glm.unpack(lay, r["u"], "u")[0]
            if U_o is not None:
                eu = rel(u, U_o)
            else:
                eu = rel(np.einsum("tjk,ji->tik", u, inst.Omega), SU_o)
            info = int(r["info"].cpu().numpy()[0])
            e = {"solves_per_s": round(1.0 / r["dt"], 3), "ms_per_step": round(1000 * r["dt"], 2),
                 "pcg_iterations": int(r["iters"]),
                 "pcg_iterations_per_s": round(r["iters"] / r["dt"], 1),
                 "outer_steps": int(r["outer"]), "info": info,
                 "max_rel_err": {"beta": rel(beta, beta_o),
                                 ("u" if U_o is not None else "Sigma_u"): eu}}
            rl = roofline(r["prof"], traffic_key=None, names={
                0: f"k_proj_a<{'float' if prec == 'mixed' else 'double'}>",
                1: f"k_proj_b<{'float' if prec == 'mixed' else 'double'}>",
                2: PASS_NAMES[2]})
            if rl:
                e["roofline"] = rl[0]
            entry[prec] = e
            log(f"{name} {prec}: {1000 * r['dt']:.1f} ms/step, {r['iters']} PCG iterations, "
                f"beta err {e['max_rel_err']['beta']:.2e}")
        entry["speedup_mixed_vs_fp64"] = round(entry["mixed"]["solves_per_s"] /
                                               entry["fp64"]["solves_per_s"], 3)
        out[name] = entry
        del runner, d
        torch.cuda.empty_cache()
    return out


MVR_MODELS = [(0.9, 0.26, 4.48), (1.05, 0.26, 4.48), (0.9, 0.26, 448.0), (1.05, 0.26, 448.0),
              (0.9, 0.80, 448.0), (1.05, 0.80, 448.0)]


def mvrglm_config(glm, torch, synth, args, per_model=40, K=16):
    """The restricted VAR workload: 240 multivariate models with exclusions
    (the six kinds of the paper's VAR experiments, 40 of each: G = 12,
    M = 300, N = 60, K = 16 right-hand sides), one step = factor + solve.
    Through the common-regressor reduction (one QR of Z0, N + 1 rows) and,
    for comparison, through the SUR reduction of X = [Z0[:, sel_i]]; PCG
    iterations with D = alpha I and with D = diag(omega_ii) (x) I; the error
    against the oracle on one instance of each kind."""
    import numpy as np
    from oracle import mvrglm as omvr
    insts = []
    for q, (lam, sp, oc) in enumerate(MVR_MODELS):
        insts += synth.mvrglm_var(seed=700 + q, B=per_model, K=K, lam_max=lam, sparsity=sp,
                                  omega_cond=oc)
    lay, d = glm.pack_mvr(insts)
    n_solves = lay.n_rhs
    out = {"workload": f"mvrglm_var4_batch{len(insts)}_K{K}: G=12, M=300, N=60, sparsity "
                       "26%/80%, largest root 0.90/1.05, cond(Omega) 4.48/448",
           "instances": len(insts), "solves_per_step": n_solves}

    def timed(make, factor_args, solve_args, steps):
        s = make()
        res = None
        for it in range(steps + 1):
            if it == 1:
                torch.cuda.synchronize()
                t = time.perf_counter()
            s.factor(*factor_args)
            res = s.solve(*solve_args)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        st = s.stats()
        s.close()
        return dt, res, st

    sample = [q * per_model for q in range(len(MVR_MODELS))]
    for prec in ("mixed", "fp64"):
        for precond in ("scalar", "equation"):
            dt, res, st = timed(lambda: glm.MVRSolver(lay, d["N"], d["sel"], prec,
                                                      precond=precond),
                                (d["Z0"],), (d["Omega"], d["y"], None, 1e-12), args.steps)
            e = {"solves_per_s": round(n_solves / dt, 1), "ms_per_step": round(1000 * dt, 2),
                 "pcg_iterations": int(st["pcg_iterations"]),
                 "max_iterations": int(st["max_iterations"])}
            if precond == "scalar":
                betas = glm.unpack(lay, res[0], "beta")
                errs = []
                for b in sample:
                    inst = insts[b]
                    ref = (omvr.mvrglm_gls(inst)[0] if np.linalg.cond(inst.Z0) < 1e3
                           else omvr.mvrglm_gls_whitened(inst)[0])
                    errs.append(rel(betas[b], ref))
                e["max_rel_err_beta"] = {f"lam{m[0]}_sp{m[1]}_om{m[2]}": v
                                         for m, v in zip(MVR_MODELS, errs)}
            out[f"{prec}_{'D1' if precond == 'scalar' else 'D2'}"] = e
            log(f"mvrglm {prec} {precond}: {e['ms_per_step']} ms/step, "
                f"{e['pcg_iterations']} PCG iterations")
    surs = [i.to_sur() for i in insts]
    lay2, d2 = glm.pack_instances(surs)
    dt, _, st = timed(lambda: glm.SURSolver(lay2, "mixed", reduce=True), (d2["X"], d2["Rc"]),
                      (d2["Omega"], d2["y"], d2["r"], 1e-12), args.steps)
    out["mixed_via_sur_reduction"] = {"solves_per_s": round(n_solves / dt, 1),
                                      "ms_per_step": round(1000 * dt, 2),
                                      "pcg_iterations": int(st["pcg_iterations"])}
    log(f"mvrglm via the SUR reduction: {1000 * dt:.1f} ms/step")
    del d, d2
    torch.cuda.empty_cache()
    return out


def ne_comparator(glm, torch, synth, args):
    """PCG-NE (CG on the normal equations, block-Jacobi preconditioner, FP64)
    on the headline workload through the same model reduction: one step =
    reduction QR + per-block QR + the normal-equation solves, stopped at
    ||r|| <= 1e-13 ||b||."""
    import numpy as np
    from oracle import gls as ogls
    insts = list(synth.config2(B=args.instances))
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, "fp64", reduce=True)

    def step():
        s.factor(d["X"], d["Rc"])
        return s.solve_ne(d["Omega"], d["y"], tol=1e-13, max_iter=0)

    step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = 0
    for _ in range(args.steps):
        beta, info, iters = step()
        its += s.stats()["pcg_iterations"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    infos = info.cpu().numpy()
    betas = glm.unpack(lay, beta, "beta")
    sample = list(range(0, len(insts), max(1, len(insts) // max(1, args.check))))[: args.check]
    eb = max(rel(betas[b][:, k], ogls.sur_gls(insts[b])[0][:, k])
             for b in sample for k in range(insts[b].K))
    out = {"solves_per_s": round(lay.n_rhs * args.steps / dt, 2),
           "ms_per_step": round(1000 * dt / args.steps, 2),
           "iterations_per_s": round(its / dt, 1),
           "mean_iterations": round(its / args.steps / lay.n_rhs, 1),
           "converged": f"{int(np.sum(infos == 0))}/{lay.n_rhs}",
           "max_rel_err_beta": eb}
    log(f"pcg-ne: {out}")
    s.close()
    del s, d
    torch.cuda.empty_cache()
    return out


def montecarlo(glm, torch, synth, iters=(1, 2, 3, 4, 6, 8, 12, 16, 20)):
    """The Monte Carlo comparison of the PCG-Aug and PCG-NE estimators
    (section on the statistical properties of the PCG-Aug estimator) at
    4096 replications of its SUR counterpart (m = 80, n = 20, Sigma with
    eigenvalues 0.01, 0.1, 10, 50): for each iteration count, the largest
    |mean error| / standard error over the coefficients, the RMSE of beta,
    and the mean and 2.5/97.5 % quantiles of the error of beta_2."""
    import numpy as np
    insts = list(synth.mc_sur(seed=21, B=256, K=16))
    lay, d = glm.pack_instances(insts)
    truth = np.array([inst.beta_true[:, k] for inst in insts for k in range(inst.K)])
    res = {"workload": "mc_sur_m80_n20: G=4, M=20, n_i=5, Omega eigenvalues "
                       "(0.01, 0.1, 10, 50); X, Omega, beta fixed, y redrawn",
           "replications": int(truth.shape[0]), "iterations": list(iters)}
    t = time.perf_counter()
    for name in ("pcg_aug", "pcg_ne"):
        s = glm.SURSolver(lay, "fp64")
        s.factor(d["X"], d["Rc"])
        rows = {"max_abs_z": [], "rmse": [], "beta2_mean_err": [], "beta2_q025": [],
                "beta2_q975": []}
        for i in iters:
            if name == "pcg_aug":
                beta = s.solve(d["Omega"], d["y"], d["r"], tol=0.0, max_iter=i)[0]
            else:
                beta = s.solve_ne(d["Omega"], d["y"], tol=0.0, max_iter=i)[0]
            bs = glm.unpack(lay, beta, "beta")
            est = np.array([bs[b][:, k] for b, inst in enumerate(insts) for k in range(inst.K)])
            e = est - truth
            z = np.abs(e.mean(0)) / (e.std(0, ddof=1) / np.sqrt(e.shape[0]))
            rows["max_abs_z"].append(round(float(z.max()), 2))
            rows["rmse"].append(float(np.sqrt(np.mean(np.sum(e * e, axis=1)))))
            rows["beta2_mean_err"].append(float(e[:, 1].mean()))
            rows["beta2_q025"].append(float(np.quantile(e[:, 1], 0.025)))
            rows["beta2_q975"].append(float(np.quantile(e[:, 1], 0.975)))
        res[name] = rows
        s.close()
    res["seconds"] = round(time.perf_counter() - t, 2)
    log(f"montecarlo: PCG-Aug max|z| {res['pcg_aug']['max_abs_z']}, "
        f"PCG-NE max|z| {res['pcg_ne']['max_abs_z']}")
    del d
    torch.cuda.empty_cache()
    return res


def stream_ceiling(glm, torch, insts, reps=20):
    """Rate of a plain streaming kernel (glm_stream_mix) moving the bytes of
    the reduced solve's projection passes in their pattern, at the full
    sizes of the batched workload (every rhs active): FP32 vectors of
    sum Mr G K elements and Q of sum Mr n (Mr = min(M, n + 1)).  Pass B reads
    u, g, w and Q and writes g and w in place; pass A (without its partial
    sums) reads u, g and Q and writes u in place; a copy moves one vector."""
    V = sum(min(i.M, i.n + 1) * i.G * i.K for i in insts)
    nq = sum(min(i.M, i.n + 1) * i.n for i in insts)
    V, nq = (V + 3) // 4 * 4, (nq + 3) // 4 * 4
    dev = torch.device("cuda")
    u, g, w = (torch.randn(V, device=dev) for _ in range(3))
    Q = torch.randn(nq, device=dev)
    mixes = {"pass_b": ([u, Q], [g, w], [], 5 * V + nq, "read u, g, w, Q; write g, w in place"),
             "pass_a": ([g, Q], [u], [], 3 * V + nq, "read u, g, Q; write u in place"),
             "copy": ([u], [], [g], 2 * V, "read one vector, write another")}
    res = {}
    for name, (ro, rw, wo, elems, what) in mixes.items():
        for _ in range(3):
            glm.glm_stream_mix(ro, rw, wo)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            glm.glm_stream_mix(ro, rw, wo)
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        res[name] = {"mix": what, "bytes": 4 * elems, "avg_us": round(us, 2),
                     "gbs": round(4 * elems / (us * 1e-6) / 1e9, 1)}
    log("same-mix streaming ceiling: " + ", ".join(f"{k} {v['gbs']} GB/s" for k, v in res.items()))
    del u, g, w, Q
    torch.cuda.empty_cache()
    return res


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel_path, start, end in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel_path), "rb") as f:
            text = f.read()
        if start is not None:
            i = text.index(start.encode())
            text = text[i:text.index(end.encode(), i)]
        h.update(text)
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of the timed kernel from the committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    if key is None:
        return None
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != kernel_sources_sha256():
        return None
    k = t.get("passes", {}).get(key)
    return None if k is None else k.get("hbm_bytes_per_launch")


def roofline(prof, traffic_key, names=None):
    """(roofline of the kernel with the most timed milliseconds, the others)."""
    names = names or PASS_NAMES
    if not prof:
        return None
    timed_ids = [k for k in names if prof.get(k) and prof[k][0] and prof[k][1] > 0]
    if not timed_ids:
        return None
    kid = max(timed_ids, key=lambda k: prof[k][1])
    n_l, ms, by = prof[kid]
    ach = (by / n_l) / (ms / n_l * 1e-3) / 1e9
    main_rl = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4),
               "traffic": measured_traffic(None if traffic_key is None
                                           else traffic_key + str(kid)),
               "kernel": names[kid], "launches": n_l, "avg_us": round(1000 * ms / n_l, 2),
               "alg_bytes_per_launch": round(by / n_l)}
    others = []
    for k in timed_ids:
        if k != kid:
            n2, ms2, by2 = prof[k]
            others.append({"kernel": names[k], "launches": n2,
                           "avg_us": round(1000 * ms2 / n2, 2),
                           "achieved": round((by2 / n2) / (ms2 / n2 * 1e-3) / 1e9, 1),
                           "share_of_timed_ms": round(ms2 / sum(prof[j][1] for j in timed_ids), 3)})
    main_rl["share_of_timed_ms"] = round(ms / sum(prof[j][1] for j in timed_ids), 3)
    return main_rl, others


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def _oracle_rate(insts, budget_s):
    from oracle import gls as ogls
    t = time.perf_counter()
    solves = done = 0
    for inst in insts:
        ogls.sur_gls(inst)
        solves += inst.K
        done += 1
        if time.perf_counter() - t > budget_s:
            break
    return solves, done, time.perf_counter() - t


def cpu_baseline(insts, budget_s):
    """The oracle (textbook SUR GLS by Cholesky, NumPy/LAPACK) on the host
    cores, on the first instances of the same workload until ~budget_s of
    work, with every BLAS thread, then with one."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    solves, done, dt = _oracle_rate(insts, budget_s)
    out = {"value": round(solves / dt, 2), "unit": "solves/s", "cores": int(cores),
           "kind": "oracle", "cpu": cpu_model(), "logical_cpus": os.cpu_count(),
           "sample": f"first {done} of {len(insts)} instances ({solves} solves), {dt:.1f}s, "
                     f"{cores} BLAS threads"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            s1, d1, t1 = _oracle_rate(insts, budget_s / 2)
        out["single_thread"] = {"value": round(s1 / t1, 2), "unit": "solves/s",
                                "sample": f"first {d1} instances ({s1} solves), {t1:.1f}s"}
    return out


if __name__ == "__main__":
    main()
