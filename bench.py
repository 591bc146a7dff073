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
# Kernel classes timed with HIP events inside the library during one extra,
# untimed step after the timed ones (the timed steps run as a user runs the
# library, with no events between the launches).  The roofline is reported
# for the single-kernel class with the most time; the others are listed for
# context.
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
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1, 2],
                    help="mode of the timed headline steps: 0 = FP64 throughout, 1 = the PCG "
                         "preconditioner's dense subdomain operators stored in FP32, 2 = also "
                         "the pair LOBPCG's operator products in FP32 (MFMA, FP32 "
                         "accumulation) before an FP64 polish")
    ap.add_argument("--compare", default="0,1,2",
                    help="precision modes also timed on the same workload (comma-separated; "
                         "empty for none)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="subdomains (and about as many pairs) the oracle handles for a "
                         "sampled CPU baseline, scaled to the whole workload by operation "
                         "counts; 0 = run the whole method in the oracle (default: 0 for "
                         "C1/C2/C5, 24 for C3/C4)")
    ap.add_argument("--table5", action="store_true",
                    help="instead of the benchmark: the level comparison of Section 8.1 "
                         "(Tab. 5) on the synthetic 64^3 elasticity cube, three levels, "
                         "tau^2 = 25, 16, 9, 4, 2.25, and the non-adaptive c+e+f and c+e runs")
    ap.add_argument("--table5-n", type=int, default=64, help="elements per side for --table5")
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


def host_info():
    """CPU model (/proc/cpuinfo), BLAS library and threads of the oracle's host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{d.get('internal_api')} {d.get('version')}" for d in threadpool_info()
                if d.get("user_api") == "blas"]
        blas = ", ".join(libs) if libs else None
    except Exception:
        pass
    return {"cpu_model": model, "blas": blas, "cores": blas_threads(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline_full(prob, rtol):
    """The whole method in the FP64 oracle, timed as it runs."""
    import oracle as O
    hi = host_info()
    t0 = time.perf_counter()
    H = O.setup_hierarchy(prob)
    t1 = time.perf_counter()
    X, its, cond, _ = O.solve_problem(prob, rtol=rtol, H=H)
    t2 = time.perf_counter()
    n_pairs = sum(len(L.pairs) for L in H.levels)
    return dict(value=t2 - t0, unit="s", cores=hi["cores"], kind="oracle",
                setup_s=t1 - t0, solve_s=t2 - t1, host=hi,
                sample=(f"{prob.name}: the whole method in the FP64 oracle (dense Schur "
                        f"complements, {n_pairs} dense pair eigensolves, enriched BDDC, "
                        f"PCG to {rtol:g} in {int(its[0])} its), nothing scaled"))


def cpu_baseline_sampled(prob, nsamp, pcg_its):
    """The FP64 oracle on a bounded sample of a level-1 workload, scaled.

    Timed as the oracle runs them: the level input (whole), the dense
    subdomain matrices and Schur complements of nsamp subdomains, the dense
    pair eigenproblems of about nsamp pairs among them, and the per-subdomain
    steps of the oracle's Alg. 1 (interior Cholesky, LU of the saddle-point
    Neumann system, its coarse basis; then one application's solves) for the
    same subdomains.  Each part is scaled to all subdomains / pairs by the
    ratio of its operation counts (n_I^3/3 + n_I^2 n_G + n_I n_G^2 for a
    Schur complement, n^3 for a pair eigensolve or a factorisation, n^2 for
    a solve); PCG = setup factorisations + pcg_its x (scaled solves + three
    sparse products with K, timed whole)."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import fem
    from oracle.adaptive import pair_eigenproblem
    from oracle.substructure import build_level, level1_input
    hi = host_info()
    t0 = time.perf_counter()
    inp = level1_input(prob)
    t_input = time.perf_counter() - t0
    Ls = build_level(inp, only=())           # structure only (untimed part of the sample)
    nsub = Ls.inp.n_sub
    nI = np.array(Ls.n_I, float)
    nG = np.array(Ls.n_G, float)
    # pairs spread over the list; their subdomains form the subdomain sample
    npair = len(Ls.pairs)
    want_p = max(1, nsamp // 2)
    psel = sorted(set(np.linspace(0, npair - 1, want_p).round().astype(int).tolist()))
    subs = sorted({s for p in psel for s in Ls.pairs[p][:2]})
    t0 = time.perf_counter()
    L = build_level(inp, only=set(subs))
    t_schur_s = time.perf_counter() - t0
    w_schur = nI ** 3 / 3 + nI ** 2 * nG + nI * nG ** 2
    schur_all = t_schur_s * w_schur.sum() / w_schur[subs].sum()
    t0 = time.perf_counter()
    pn = []
    for p in psel:
        s, t, g = L.pairs[p]
        r = pair_eigenproblem(L, s, t, L.globs[g], prob.tau, prob.nev_max)
        pn.append(r["n"])
    t_pairs_s = time.perf_counter() - t0
    pn_all = np.array([nG[s] + nG[t] for s, t, _ in L.pairs])
    pairs_all = t_pairs_s * (pn_all ** 3).sum() / (np.array(pn, float) ** 3).sum()
    # Alg. 1 per subdomain, as the oracle does it: factorisations, then solves
    t0 = time.perf_counter()
    facs = []
    for s in subs:
        K = L.K[s]
        ni = L.n_I[s]
        n = K.shape[0]
        nc = L.C[s].shape[0]
        ch = sla.cho_factor(K[:ni, :ni], lower=True) if ni else None
        A = np.zeros((n + nc, n + nc))
        A[:n, :n] = K
        A[ni:n, n:] = L.C[s].T
        A[n:, ni:n] = L.C[s]
        lu = sla.lu_factor(A)
        rhs = np.zeros((n + nc, nc))
        rhs[n:, :] = np.eye(nc)
        Phi = sla.lu_solve(lu, rhs)[:n]
        facs.append((ch, lu, Phi, ni, n, nc))
    t_fac_s = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    for ch, lu, Phi, ni, n, nc in facs:
        x = rng.standard_normal(n)
        if ch is not None:
            sla.cho_solve(ch, x[:ni])
        sla.lu_solve(lu, np.concatenate([x, np.zeros(nc)]))
        if nc:
            Phi.T @ x
            Phi @ rng.standard_normal(nc)
        if ch is not None:
            sla.cho_solve(ch, x[:ni])
    t_sol_s = time.perf_counter() - t0
    ncs = np.array([len(c) for c in Ls.C], float)
    nn = nI + nG
    w_fac = nI ** 3 / 3 + (nn + ncs) ** 3 * (2.0 / 3.0)
    w_sol = 2 * nI ** 2 + (nn + ncs) ** 2
    fac_all = t_fac_s * w_fac.sum() / w_fac[subs].sum()
    sol_all = t_sol_s * w_sol.sum() / w_sol[subs].sum()
    Kg = fem.assemble_global(prob)
    x = rng.standard_normal(Kg.shape[0])
    t0 = time.perf_counter()
    for _ in range(3):
        Kg @ x
    t_mv = time.perf_counter() - t0
    pcg_all = fac_all + pcg_its * (sol_all + t_mv)
    total = t_input + schur_all + pairs_all + pcg_all
    measured = t_input + t_schur_s + t_pairs_s + t_fac_s + t_sol_s + t_mv
    return dict(value=total, unit="s", cores=hi["cores"], kind="oracle", host=hi,
                measured_s=measured,
                parts_s={"level_input": t_input, "schur": schur_all, "pair_eigs": pairs_all,
                         "pcg": pcg_all},
                pair_eigenproblems_per_s=npair / pairs_all,
                sample=(f"{prob.name}: FP64 oracle on a sample, scaled by operation counts: "
                        f"level input whole; dense Schur complements of {len(subs)} of "
                        f"{nsub} subdomains; dense pair eigensolves of {len(psel)} of {npair} "
                        f"pairs; the oracle's Alg. 1 factorisations and one application's "
                        f"solves on the same {len(subs)} subdomains, x {pcg_its} PCG "
                        f"iterations (the GPU's count) with three sparse K products each; "
                        f"{measured:.1f} s measured"
                        + ("; level 1 only (the higher levels are not timed)"
                           if prob.levels > 2 else "")))


def run_table5(args):
    """Tab. 5 on the synthetic cube: one set-up + solve (rtol 1e-8, as the
    paper's serial runs) per row; prints one JSON line with the rows."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1301_0191_amd import Handle
    dev = torch.device("cuda:0")
    rows = []
    variants = [(t2, "c+e", dict()) for t2 in (25.0, 16.0, 9.0, 4.0, 2.25)]
    variants += [(None, "c+e+f", dict(initial="c+e+f", tau=0.0)),
                 (None, "c+e", dict(tau=0.0))]
    for t2, init, kw in variants:
        prob = W.cube_tab5(t2 if t2 else 4.0, n=args.table5_n)
        t0 = time.perf_counter()
        h = Handle.from_problem(prob, precision=args.precision, **kw)
        print(f"table5: handle for tau2={t2} {init} in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        coeff = torch.from_numpy(prob.coeff).to(dev)
        nu = torch.from_numpy(prob.nu).to(dev)
        rhs = torch.from_numpy(np.ascontiguousarray(prob.rhs.T)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.setup(coeff, nu)
        res = h.solve(rhs, rtol=1e-8, maxit=5000, raise_on_noconv=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t0
        st = h.stats()
        om = st["omega_tilde"]
        row = {"tau2": t2, "initial": init, "n_free": st["n_free"],
               "pairs": st["n_pairs"], "adaptive_constraints": st["n_adaptive"],
               "constraints_per_pair": [a / p if p else 0.0
                                        for a, p in zip(st["n_adaptive"], st["n_pairs"])],
               "omega_tilde_levels": om,
               "omega_tilde": float(np.prod([o for o in om if o > 0])) if t2 else None,
               "its": res.iterations[0], "cond": res.cond[0],
               "lobpcg_iterations": st["lobpcg_iters"], "n_unconverged": st["n_unconverged"],
               "setup_s": st["t_phase"][6], "solve_s": st["t_phase"][7], "wall_s": t1}
        rows.append(row)
        print("table5 row", json.dumps(row), file=sys.stderr, flush=True)
        h.close()
    print(json.dumps({"table5": rows, "workload": f"cube_tab5 n={args.table5_n}",
                      "precision": args.precision}), flush=True)


def main():
    args = parse()
    if args.table5:
        run_table5(args)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); "
              "a multi-GPU path is not built.", file=sys.stderr)
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
            return h.solve(rhs, rtol=args.rtol, maxit=2000, x=x, raise_on_noconv=False)

        for i in range(args.warmup):
            step()
            print(f"precision {precision}: warmup step {i + 1}/{args.warmup} done",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        # timed steps as a user runs them (no kernel-class events)
        setup_s, solve_s, step_s = [], [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            ts = time.perf_counter()
            res = step()
            torch.cuda.synchronize()
            step_s.append(time.perf_counter() - ts)
            st = h.stats()
            setup_s.append(st["t_phase"][6])
            solve_s.append(st["t_phase"][7])
            print(f"precision {precision}: step {i + 1}/{args.steps} done", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = h.stats()
        # one more, untimed step with HIP events around every launch of the
        # kernel classes (their rooflines)
        h.timing_enable(TIMED)
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        T_instr = time.perf_counter() - ts
        timed = {c: h.timing_read(c) for c in TIMED}
        h.timing_enable(None)
        h.close()
        print(f"precision {precision}: instrumented step done", file=sys.stderr, flush=True)
        return dict(T=T, res=res, st=st, timed=timed, setup_s=setup_s, solve_s=solve_s,
                    step_s=step_s, analysis_s=analysis_s, T_instr=T_instr)

    def kernel_table(m):
        kernels = {}
        for c, t in m["timed"].items():
            if t["launches"] == 0 or t["ms"] <= 0:
                continue
            sec = t["ms"] * 1e-3
            kernels[c] = {"launches": t["launches"], "avg_launch_us": 1e3 * t["ms"] / t["launches"],
                          "share_of_step": sec / m["T_instr"],
                          "alg_flops_per_launch": t["flops"] / t["launches"],
                          "alg_bytes_per_launch": t["bytes"] / t["launches"],
                          "tflops": t["flops"] / sec / 1e12, "gbps": t["bytes"] / sec / 1e9}
        return kernels

    main_m = run(args.precision)
    others = {}
    for tok in (args.compare or "").split(","):
        if tok.strip() and int(tok) != args.precision:
            others[int(tok)] = run(int(tok))
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
                "median_step_s": float(np.median(m["step_s"])),
                "setup_s": float(np.mean(m["setup_s"])), "solve_s": float(np.mean(m["solve_s"])),
                "pcg_iterations": r.iterations,
                "true_residual_max": max(r.true_residual) if r.true_residual else None,
                "adaptive_constraints": m["st"]["n_adaptive"],
                "omega_tilde": m["st"]["omega_tilde"],
                "lobpcg_iterations": m["st"]["lobpcg_iters"],
                "lobpcg_iterations_fp32": m["st"]["lobpcg_iters_fp32"],
                "lobpcg_select_s": m["st"]["t_phase"][2],
                "pair_apply": {kk: k["pair_apply"][kk] for kk in ("avg_launch_us", "tflops")}
                if "pair_apply" in k else None,
                "bddc_apply": {kk: k["bddc_apply"][kk] for kk in ("avg_launch_us", "gbps")}
                if "bddc_apply" in k else None}

    modes = None
    names = {0: "fp64", 1: "fp32_stored_preconditioners", 2: "fp32_lobpcg_and_preconditioners"}
    if others:
        by_p = dict(others)
        by_p[args.precision] = main_m
        modes = {names[pm]: mode_summary(mm) for pm, mm in sorted(by_p.items())}
        if 0 in by_p:
            t64 = float(np.median(by_p[0]["step_s"]))
            for pm, mm in by_p.items():
                if pm != 0:
                    modes[f"speedup_{names[pm]}_vs_fp64"] = t64 / float(np.median(mm["step_s"]))
    out = {
        "metric": METRIC,
        "value": float(np.median(main_m["step_s"])),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 1: "f64 (preconditioner operators stored f32)",
                  2: "f32 MFMA (pair LOBPCG products, preconditioner operators) + f64 (Gram, "
                     "Rayleigh-Ritz, polish, Schur, PCG residuals)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": prob.name, "n_free": st["n_free"], "subdomains": st["n_sub"],
                   "pairs": st["n_pairs"], "levels": prob.levels, "tau": prob.tau,
                   "nrhs": int(rhs.shape[0]), "rtol": args.rtol, "precision": args.precision},
        "pair_eigenproblems_per_s": n_pairs / lob if lob > 0 else None,
        "step_s": main_m["step_s"],
        "setup_s": float(np.mean(main_m["setup_s"])),
        "solve_s": float(np.mean(main_m["solve_s"])),
        "analysis_s": main_m["analysis_s"],
        "pcg_iterations": res.iterations,
        "pcg_residual_replacements": st["pcg_replacements"],
        "pcg_converged": bool(res.true_residual) and max(res.true_residual) <= args.rtol,
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
        nsamp = args.cpu_sample
        if nsamp is None:
            nsamp = 24 if args.config in ("c3", "c4") else 0
        if nsamp > 0:
            out["cpu_baseline"] = cpu_baseline_sampled(prob, nsamp, int(max(res.iterations)))
        else:
            out["cpu_baseline"] = cpu_baseline_full(prob, args.rtol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
