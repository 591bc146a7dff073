#!/usr/bin/env python3
"""Adaptive-Multilevel BDDC on one MI355X: set-up + solve benchmark.

One step = the whole hot path on the workload: numeric set-up (element
matrices, batched interior factorisations and Schur complements, BDDC
structures, batched LOBPCG over every face pair with the adaptive selection,
enriched BDDC, next levels, coarsest factorisation) followed by PCG with the
multilevel BDDC preconditioner to relative residual 1e-10.  Coefficients and
right-hand sides are resident on the GPU before the timed region; the mesh
analysis (integer structure, done once per mesh) is reported separately.

Prints one JSON line (rank 0 only; this build runs on one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve time to rel. residual 1e-10 & pair eigenproblems/s, FP32+batched vs FP64"

# MI355X peaks (published): FP64 vector and FP64 MFMA 78.6 TFLOP/s, HBM3E 8 TB/s.
PEAK_F64 = 78.6e12
PEAK_HBM = 8.0e12
# Kernel classes timed with HIP events inside the library during the timed
# steps.  The roofline is reported for the single-kernel class with the most
# time; the others are listed for context.
TIMED = ["pair_rr", "pair_apply", "pair_gram", "schur", "bddc_apply"]
SINGLE_KERNEL = {
    # class: (kernel, bound, peak, unit)
    "pair_rr": ("k_rr (batched pair Rayleigh-Ritz)", "alu", PEAK_F64, "TFLOP/s"),
    "pair_apply": ("k_gemm, grouped S^s products of the pair LOBPCG", "mfma", PEAK_F64, "TFLOP/s"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1],
                    help="mode of the timed headline steps: 0 = FP64 throughout, 1 = the PCG "
                         "preconditioner's dense subdomain operators stored in FP32")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the steps in the other precision mode")
    ap.add_argument("--cpu-pairs", type=int, default=0,
                    help="pair eigenproblems the oracle solves for a sampled CPU baseline "
                         "(0 = run the whole method in the oracle)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the steps, copy a device buffer of this size once (a plain "
                         "copy kernel of known traffic, for calibrating HBM counters)")
    return ap.parse_args()


def traffic_for(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, calibrated by a plain copy), if the kernel sources are
    unchanged since the measurement; else None."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    try:
        for rel in rec["sources"]:
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"]


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return 1


def cpu_baseline(prob, npairs_sample, rtol):
    """The FP64 oracle on the host cores, on the same workload.

    npairs_sample <= 0: the whole method (hierarchy set-up with every dense
    pair eigenproblem, then PCG to rtol), timed as it runs.  Otherwise only
    that many pair eigenproblems are solved and their time is scaled to all
    pairs; the PCG then runs with the partially enriched preconditioner, so
    that leg is an upper bound."""
    import numpy as np
    import oracle as O
    cores = blas_threads()
    if npairs_sample <= 0:
        t0 = time.perf_counter()
        H = O.setup_hierarchy(prob)
        t1 = time.perf_counter()
        X, its, cond, _ = O.solve_problem(prob, rtol=rtol, H=H)
        t2 = time.perf_counter()
        n_pairs = sum(len(L.pairs) for L in H.levels)
        return dict(value=t2 - t0, unit="s", cores=cores, kind="oracle",
                    setup_s=t1 - t0, solve_s=t2 - t1,
                    sample=(f"{prob.name}: the whole method in the FP64 oracle (dense Schur "
                            f"complements, {n_pairs} dense pair eigensolves, enriched BDDC, "
                            f"PCG to {rtol:g} in {int(its[0])} its), {cores} BLAS threads; "
                            f"nothing scaled"))
    from oracle.substructure import build_level, coarse_basis, level1_input
    from oracle.adaptive import enrich_level
    from oracle.bddc import _prepare_full_space, Hierarchy, bddc_apply, pcg
    from oracle import fem
    import scipy.linalg as sla
    t0 = time.perf_counter()
    inp = level1_input(prob)
    L = build_level(inp)
    L.Kglob = fem.assemble_global(prob)
    t1 = time.perf_counter()
    n_pairs = len(L.pairs)
    sample = list(range(0, n_pairs, max(1, n_pairs // npairs_sample)))[:npairs_sample]
    enrich_level(L, prob.tau, prob.nev_max, pairs=sample)
    t2 = time.perf_counter()
    coarse_basis(L)
    _prepare_full_space(L)
    H = Hierarchy(levels=[L])
    nC = L.n_coarse
    Kt = np.zeros((nC, nC))
    for s in range(L.inp.n_sub):
        Kt[np.ix_(L.Rc[s], L.Rc[s])] += L.Kc[s]
    H.top_chol = sla.cho_factor(Kt, lower=True)
    t3 = time.perf_counter()
    x, its, *_ = pcg(L.Kglob, prob.rhs[:, 0], lambda v: bddc_apply(H, v), rtol, 1000)
    t4 = time.perf_counter()
    per_pair = (t2 - t1) / max(1, len(sample))
    total_est = (t1 - t0) + per_pair * n_pairs + (t3 - t2) + (t4 - t3)
    return dict(value=total_est, unit="s", cores=cores, kind="oracle",
                measured_s=t4 - t0,
                sample=(f"{prob.name}: oracle level set-up, dense pair eigensolves for "
                        f"{len(sample)} of {n_pairs} pairs (time scaled to all pairs), "
                        f"enriched BDDC with the sampled constraints only, PCG to {rtol:g} "
                        f"({its} its, an upper bound); {cores} BLAS threads"))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    from paper_1301_0191_amd import Handle

    dev = torch.device("cuda:0")
    prob = W.CONFIGS[args.config](args.seed)
    coeff = torch.from_numpy(prob.coeff).to(dev)
    nu = None if prob.nu is None else torch.from_numpy(prob.nu).to(dev)
    rhs = torch.from_numpy(np.ascontiguousarray(prob.rhs.T)).to(dev)
    x = torch.empty_like(rhs)

    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr)
        del src, dst

    def run(precision):
        """Warm-up and timed steps with one handle; returns the measurements."""
        t0 = time.perf_counter()
        h = Handle.from_problem(prob, precision=precision)
        analysis_s = time.perf_counter() - t0

        def step():
            h.setup(coeff, nu)
            return h.solve(rhs, rtol=args.rtol, maxit=2000, x=x)

        for i in range(args.warmup):
            step()
            print(f"precision {precision}: warmup step {i + 1}/{args.warmup} done",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        h.timing_enable(TIMED)
        setup_s, solve_s = [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            res = step()
            st = h.stats()
            setup_s.append(st["t_phase"][6])
            solve_s.append(st["t_phase"][7])
            print(f"precision {precision}: step {i + 1}/{args.steps} done", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        timed = {c: h.timing_read(c) for c in TIMED}
        h.timing_enable(None)
        st = h.stats()
        h.close()
        return dict(T=T, res=res, st=st, timed=timed, setup_s=setup_s, solve_s=solve_s,
                    analysis_s=analysis_s)

    def kernel_table(m):
        kernels = {}
        for c, t in m["timed"].items():
            if t["launches"] == 0 or t["ms"] <= 0:
                continue
            sec = t["ms"] * 1e-3
            kernels[c] = {"launches": t["launches"], "avg_launch_us": 1e3 * t["ms"] / t["launches"],
                          "share_of_step": sec / m["T"],
                          "alg_flops_per_launch": t["flops"] / t["launches"],
                          "alg_bytes_per_launch": t["bytes"] / t["launches"],
                          "tflops": t["flops"] / sec / 1e12, "gbps": t["bytes"] / sec / 1e9}
        return kernels

    main_m = run(args.precision)
    other_m = run(1 - args.precision) if not args.no_compare else None
    timed, T, res, st = main_m["timed"], main_m["T"], main_m["res"], main_m["st"]
    kernels = kernel_table(main_m)
    dom = max((c for c in SINGLE_KERNEL if c in kernels), key=lambda c: timed[c]["ms"],
              default=None)
    roofline = None
    if dom is not None:
        name, bound, peak, unit = SINGLE_KERNEL[dom]
        t = timed[dom]
        achieved = t["flops"] / (t["ms"] * 1e-3)
        roofline = {"kernel": name, "class": dom, "bound": bound,
                    "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
                    "frac": achieved / peak, "traffic": traffic_for(dom),
                    "launches": t["launches"], "avg_launch_us": 1e3 * t["ms"] / t["launches"],
                    "alg_flops_per_launch": t["flops"] / t["launches"],
                    "alg_bytes_per_launch": t["bytes"] / t["launches"]}
    ms = 1e3 * T / args.steps
    n_pairs = sum(st["n_pairs"])
    lob = st["t_phase"][2]

    def mode_summary(m):
        k = kernel_table(m)
        r = m["res"]
        return {"ms_per_step": 1e3 * m["T"] / args.steps,
                "setup_s": float(np.mean(m["setup_s"])), "solve_s": float(np.mean(m["solve_s"])),
                "pcg_iterations": r.iterations,
                "true_residual_max": max(r.true_residual) if r.true_residual else None,
                "adaptive_constraints": m["st"]["n_adaptive"],
                "lobpcg_iterations": m["st"]["lobpcg_iters"],
                "bddc_apply": {kk: k["bddc_apply"][kk] for kk in ("avg_launch_us", "gbps")}
                if "bddc_apply" in k else None}

    modes = None
    if other_m is not None:
        by_p = {args.precision: main_m, 1 - args.precision: other_m}
        modes = {"fp64": mode_summary(by_p[0]), "fp32_stored_preconditioners": mode_summary(by_p[1])}
        modes["speedup_fp32_stored_vs_fp64"] = (modes["fp64"]["ms_per_step"]
                                                / modes["fp32_stored_preconditioners"]["ms_per_step"])
    out = {
        "metric": METRIC,
        "value": T / args.steps,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64 (preconditioner operators stored f32)",
        "data": "synthetic",
        "config": {"workload": prob.name, "n_free": st["n_free"], "subdomains": st["n_sub"],
                   "pairs": st["n_pairs"], "levels": prob.levels, "tau": prob.tau,
                   "nrhs": int(rhs.shape[0]), "rtol": args.rtol, "precision": args.precision},
        "pair_eigenproblems_per_s": n_pairs / lob if lob > 0 else None,
        "setup_s": float(np.mean(main_m["setup_s"])),
        "solve_s": float(np.mean(main_m["solve_s"])),
        "analysis_s": main_m["analysis_s"],
        "pcg_iterations": res.iterations,
        "true_residual_max": max(res.true_residual) if res.true_residual else None,
        "cond": res.cond,
        "lobpcg_iterations": st["lobpcg_iters"],
        "adaptive_constraints": st["n_adaptive"],
        "omega_tilde": st["omega_tilde"],
        "phase_s": {"schur": st["t_phase"][0], "bddc_init": st["t_phase"][1],
                    "lobpcg_select": st["t_phase"][2], "enriched_bddc": st["t_phase"][4],
                    "coarse": st["t_phase"][5]},
        "roofline": roofline,
        "kernels": kernels,
        "precision_modes": modes,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_pairs, args.rtol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
