#!/usr/bin/env python3
"""Throughput of the sampled-trial AFQMC step on one MI355X.

One step = green -> Cholesky contraction (force bias + local energy) ->
estimator -> fields -> propagate (V build, Taylor, ratio, weight) ->
Metropolis sweep of every path with hand-off -> QR every 10 steps -> comb,
for the FP64 workload M=64, N=16 per spin, 256 Cholesky vectors, K=64
Gaussian hidden variables, 512 walkers x 8 paths, tau=0.005, random-walk
proposal of step 0.3 (the FP64 random-walk form whose energy error fixes the
reference error bar), in the stabilised form (local-energy weights, force-bias
and local-energy caps, see STABLE).  Inputs are synthetic (seeded generator,
see afqmc_inputs) and resident in HBM before the timed region.

Prints one JSON line.  The roofline object refers to the dominant kernel, the
Cholesky contraction, timed with HIP events on the library's stream around
every afqmc_local_energy call of the timed steps; cpu_baseline is the FP64
numpy oracle on a bounded walker sample of the same workload, run as
independent walker chunks in parallel processes on the host's cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker-steps/s at fixed energy error; contraction TFLOP/s vs MFMA peak"
PEAK_FP64_MFMA = 78.6   # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2500.0  # TFLOP/s, MI355X dense BF16 matrix

# name -> (workload index of afqmc_inputs.workload, contraction precision, peak, dtype label)
WORKLOADS = {
    "fp64": (1, 0, PEAK_FP64_MFMA, "f64"),
    "fp64-prior": (1, 0, PEAK_FP64_MFMA, "f64"),
    # mixed forms: the contraction's products in the named type, the trial series,
    # V build and propagation on FP32 products, complex64 walkers, LU / log-det /
    # Theta / QR / sums in FP64
    "mixed": (2, 1, PEAK_FP32_MFMA, "f32-products/c64-walkers/f64-lu"),
    "mixed-fp64": (2, 0, PEAK_FP64_MFMA, "f64"),
    # BF16 products: roofline against the dense BF16 peak with the algorithmic flops
    # (the split form executes three products per algorithmic one)
    "mixed-bf16x3": (2, 3, PEAK_BF16_MFMA, "bf16x3-contraction/f32-products/c64-walkers/f64-lu"),
    "mixed-bf16": (2, 2, PEAK_BF16_MFMA, "bf16-contraction/f32-products/c64-walkers/f64-lu"),
    "slices": (5, 0, PEAK_FP64_MFMA, "f64"),
}


# HBM bytes per contraction launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by
# the plain-copy calibration (profiles/traffic_k_contract_*.md), valid while the
# kernel source is the one measured: workload -> (source file, sha256 prefix, bytes)
TRAFFIC = {
    "fp64": ("k_contract.hip", "911cdc519ab8f700", 454536192),
    "fp64-prior": ("k_contract.hip", "911cdc519ab8f700", 454536192),
}

# Proposal of each per-step workload: the default FP64 leg runs the random walk
# of step 0.3 (the form the fixed energy error is defined on); "fp64-prior" the
# paper's independence sampler from p_T.  Others keep their RunConfig's.
RW_STEP_FP64 = 0.3
PROPOSAL_OVERRIDE = {"fp64": (1, RW_STEP_FP64), "fp64-prior": (0, None)}

# The stabilised form of the runs (a reading outside the paper, which states no
# stabilisation): the hybrid weight's overlap-ratio estimator sum_p O_p(phi') /
# |O_p(phi)| / sum_p S_p has a denominator that approaches zero as the paths'
# phases spread, so a few walkers take the whole weight and the comb collapses
# the population; local-energy weights with the usual caps keep the runs
# stationary.  Stated beside every figure of the per-step workloads.
STABLE = {"weights": "local energy", "xbar_cap": 1.0,
          "eloc_cap": "Re E_L within E_T +- sqrt(2/tau)",
          "e_t_schedule": "0 and no cap for steps 0..19, then the mixed estimate of the last "
                          "<= 100 steps, refreshed after step 19 and every 100 steps",
          "comb_every": 1, "comb_weights_reset_to": 1.0, "weight_cap": 0.0}


def oracle_form(proposal, rw_step, n_pc, dtau):
    """Keyword arguments of the oracle's step for the stabilised form (the
    CPU baseline's E_L cap sits at 0: its cost does not depend on the centre)."""
    import math
    return dict(proposal=proposal, rw_step=rw_step, n_pc=n_pc, weight_mode=3,
                xbar_cap=STABLE["xbar_cap"], eloc_cap=(0.0, math.sqrt(2.0 / dtau)))


# The departures of the synthetic inputs and run loop from the configurations
# as written, stated beside every figure of the per-step workloads.
L_SCALE = "0.3*sqrt(8/M)/sqrt(g+1)"
L_SCALE_NOTE = ("the configurations write 0.3/sqrt(g+1); the extra sqrt(8/M) keeps the "
                "two-body scale per orbital independent of M (exactly 1 at M = 8)")


def measured_traffic(workload):
    import hashlib
    if workload not in TRAFFIC:
        return None
    src, sha, nbytes = TRAFFIC[workload]
    path = os.path.join(ROOT, "paper_2505_18519_amd", "csrc", src)
    with open(path, "rb") as f:
        ok = hashlib.sha256(f.read()).hexdigest().startswith(sha)
    return nbytes if ok else None


def contraction_flops(M, N, G, complex_trial=False):
    """Algorithmic flops of the contraction per (walker, path): the real
    half-rotation Phi_T^T L_g (2 N M^2), its product with both spins' Theta
    (2 x 4 M N^2) and tr(f f) (2 x 8 N^2), for each of the G vectors.  A
    complex trial doubles the first two: Re and Im Phi_T^T L_g (4 N M^2), a
    complex-by-complex product per spin (2 x 8 M N^2)."""
    if complex_trial:
        return G * (4 * N * M * M + 2 * (8 * M * N * N + 8 * N * N))
    return G * (2 * N * M * M + 2 * (4 * M * N * N + 8 * N * N))


def _oracle_chunk(args):
    """One host process of the CPU baseline: the oracle's whole steps on its own
    walker chunk (one BLAS thread), one untimed step first.  Returns the time
    of the timed steps."""
    widx, n_walkers, seed, n_steps, form = args
    from threadpoolctl import threadpool_limits
    import afqmc_inputs as ai
    from oracle import afqmc_oracle as O
    sys_, run = ai.workload(widx)
    with threadpool_limits(limits=1):
        st = O.init_state(sys_, n_walkers, run.P, seed)
        Eh = O.half_kinetic(sys_, run.dtau)
        h1p = O.h1_eff(sys_)
        kw = dict(n_taylor=run.n_taylor, n_sweep=run.n_sweep, n_qr=run.n_qr, Eh=Eh, h1p=h1p,
                  **form)
        st, _ = O.step(sys_, st, seed, 0, run.dtau, **kw)
        t0 = time.perf_counter()
        for i in range(1, 1 + n_steps):
            st, _ = O.step(sys_, st, seed, i, run.dtau, **kw)
        return time.perf_counter() - t0


def host_cores():
    """CPU threads this process may use, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(widx, seed, form, per_core=4, n_steps=6):
    """Time the oracle's whole steps on a bounded walker sample: per_core
    walkers (all paths) on each host core, as independent chunks in separate
    processes (walkers are independent within a step; each chunk combs its own
    walkers), one untimed step, then n_steps timed steps.  form: the oracle
    step's keyword arguments of the run's form (proposal, weights, caps)."""
    import multiprocessing as mp
    import afqmc_inputs as ai
    sys_, run = ai.workload(widx)
    cores = host_cores()
    jobs = [(widx, per_core, seed + 7919 * c, n_steps, form) for c in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        times = pool.map(_oracle_chunk, jobs)
    wall = time.perf_counter() - t0
    dt = max(times)
    n_walkers = per_core * cores
    flops = n_walkers * n_steps * run.P * contraction_flops(sys_.M, sys_.N, sys_.n_chol)
    return {"value": n_walkers * n_steps / dt, "unit": "walker-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n_walkers} walkers x {run.P} paths ({per_core} per process on {cores} "
                      f"processes, one BLAS thread each), {n_steps} whole steps of the same "
                      f"workload after one untimed step (numpy FP64/complex128); slowest "
                      f"process {dt:.1f} s, {sum(times):.1f} s of CPU work, pool {wall:.1f} s",
            "gflops": flops / dt / 1e9,
            "gflops_counts": "the contraction's algorithmic flops over the whole steps' time"}


def reblock(x):
    """Standard error of the mean of a correlated series (Flyvbjerg-Petersen
    blocking): the largest error over blocking levels with >= 16 blocks."""
    x = np.asarray(x, dtype=np.float64)
    best = x.std(ddof=1) / np.sqrt(len(x))
    while len(x) >= 32:
        x = 0.5 * (x[0:len(x) // 2 * 2:2] + x[1:len(x) // 2 * 2:2])
        best = max(best, x.std(ddof=1) / np.sqrt(len(x)))
    return float(best)


def learned_study(args):
    """Learned-proposal workload (M=96, N=24, 384 vectors, K=128, 2048 walkers x
    4 paths), stabilised form (STABLE): the learned/mixed form (BF16 network
    trained during the warm-up on the random-walk moves, then frozen;
    FP32-product contraction) against the plain FP64 random-walk form, both
    whole AFQMC steps from the same walkers and seeds.  Step throughput and
    acceptance; the energies at fixed error come from the fixed-error
    workload (independent seeds), not from these short runs."""
    import torch
    import afqmc_inputs as ai
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D

    sys_, run = ai.workload(4)
    nw, P, seed = run.W, run.P, 2004
    xbar_cap, n_pc = STABLE["xbar_cap"], STABLE["comb_every"]
    s_train, rw_step, n_sweep_eq = 0.5, 0.3, 2

    def leg(kind):
        prec = A.PREC_FP32 if kind == "learned" else A.PREC_FP64
        common = dict(n_taylor=run.n_taylor, max_walkers=nw, xbar_cap=xbar_cap, precision=prec,
                      weight_mode=A.WEIGHT_LOCAL)
        if kind == "learned":
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_LEARNED, rw_step=s_train,
                            **common)
            p = ai.mlp_params(np.random.default_rng(8), sys_.M, sys_.K, last_scale=0.0)
            p["b3"][sys_.K:] = 4 * np.arctanh(np.log(s_train * s_train) / 4)
            A.afqmc_mlp_init(ctx, A.PREC_BF16, A.mlp_pack(p), lr=1e-3)
            A.afqmc_mlp_set_training(ctx, True)
        else:
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_RW, rw_step=rw_step, **common)
        st = D.init_walkers(ctx, sys_.phi0, nw, seed)
        est = torch.zeros(args.warmup + args.steps, 2, dtype=torch.float64, device="cuda")
        ref = D.EnergyReference(ctx)
        for i in range(args.warmup):
            D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=n_sweep_eq,
                   n_qr=run.n_qr, n_pc=n_pc)
            ref.update(i, est)
        if kind == "learned":          # freeze: network moves only from here on
            trained = A.afqmc_mlp_get_params(ctx)
            ctx.close()
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_LEARNED, rw_step=0.0, **common)
            A.afqmc_mlp_init(ctx, A.PREC_BF16, trained)
            ref.attach(ctx)
        nacc = torch.zeros(nw, dtype=torch.int64, device="cuda")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            i = args.warmup + k
            D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=1, n_qr=run.n_qr,
                   contract_events=evs[k], n_pc=n_pc)
            ref.update(i, est)
            nacc += st.nacc
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e = est.cpu().numpy()[args.warmup:]
        en = e[:, 0] / e[:, 1]
        ctx.close()
        print(f"{kind}: {1e3 * dt / args.steps:.2f} ms/step, E = {en.mean():.5f}",
              file=sys.stderr, flush=True)
        return {"walker_steps_per_s": nw * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
                "contraction_ms": float(np.mean([a.elapsed_time(b) for a, b in evs])),
                "acceptance": float(nacc.sum().item()) / (args.steps * nw * P),
                "energy_timed_steps": float(en.mean()),
                "finite": bool(np.all(np.isfinite(en)))}

    L = leg("learned")
    R = leg("rw")
    if not (L["finite"] and R["finite"]):
        print("non-finite energy in the learned study", L, R, file=sys.stderr)
        sys.exit(1)
    flops = contraction_flops(sys_.M, sys_.N, sys_.n_chol) * nw * P
    achieved = flops / (L["contraction_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": L["walker_steps_per_s"],
        "unit": "walker-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": L["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-contraction/bf16-network/f64",
        "data": "synthetic",
        "config": {"workload": f"learned-gauss-M{sys_.M}-N{sys_.N}-G{sys_.n_chol}-K{sys_.K}"
                               f"-W{nw}-P{P}-dtau{run.dtau}",
                   "network_train_step": s_train, "warmup_sweeps_per_step": n_sweep_eq,
                   "L_scale": L_SCALE, **STABLE},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": None,
                     "kernel": "k_contract_sh, FP32 products (+ k_combine) in afqmc_local_energy",
                     "ms_per_launch": L["contraction_ms"], "flops_per_launch": flops},
        "learned_mixed": L,
        "random_walk_fp64": R,
        "step_throughput_ratio": L["walker_steps_per_s"] / R["walker_steps_per_s"],
    }
    print(json.dumps(out))


def scan_study(args):
    """Cost of one step against the number of tethered paths P and of
    Metropolis sweeps (the synthetic analogue of the paper's statement that the
    cost grows linearly with P and with the sweeps): the FP64 workload's
    Hamiltonian and walker count, P in {1, 2, 4, 8, 16} at one sweep and
    n_sweep in {1, 2, 4} at P = 8, each timed over the same number of steps."""
    import torch
    import afqmc_inputs as ai
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D

    sys_, run = ai.workload(1)
    nw, seed = run.W, 2001
    rows = []
    for P, ns in [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (8, 2), (8, 4)]:
        ctx = A.Context(sys_, P, run.dtau, n_taylor=run.n_taylor, max_walkers=nw,
                        xbar_cap=STABLE["xbar_cap"], weight_mode=A.WEIGHT_LOCAL,
                        proposal=A.PROPOSAL_RW, rw_step=RW_STEP_FP64)
        st = D.init_walkers(ctx, sys_.phi0, nw, seed)
        est = torch.zeros(2, dtype=torch.float64, device="cuda")
        for i in range(args.warmup):
            D.step(ctx, st, seed, i, est, n_sweep=ns, n_qr=run.n_qr, n_pc=1)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            D.step(ctx, st, seed, args.warmup + k, est, n_sweep=ns, n_qr=run.n_qr,
                   contract_events=evs[k], n_pc=1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        rows.append({"P": P, "n_sweep": ns, "ms_per_step": 1e3 * dt / args.steps,
                     "walker_steps_per_s": nw * args.steps / dt, "contraction_ms": cms})
        print(f"P={P} n_sweep={ns}: {1e3 * dt / args.steps:.3f} ms/step (contraction {cms:.3f} ms)",
              file=sys.stderr, flush=True)
        ctx.close()
    one = [r for r in rows if r["n_sweep"] == 1]
    slope, icept = np.polyfit([r["P"] for r in one], [r["ms_per_step"] for r in one], 1)
    ref = next(r for r in rows if r["P"] == 8 and r["n_sweep"] == 1)
    flops = contraction_flops(sys_.M, sys_.N, sys_.n_chol) * nw * 8
    achieved = flops / (ref["contraction_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": ref["walker_steps_per_s"], "unit": "walker-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ref["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"scan-gauss-M{sys_.M}-N{sys_.N}-G{sys_.n_chol}-K{sys_.K}-W{nw}",
                   "walkers": nw, "proposal": "random walk", "rw_step": RW_STEP_FP64,
                   "L_scale": L_SCALE, "weights": STABLE["weights"],
                   "xbar_cap": STABLE["xbar_cap"], "comb_every": 1,
                   "eloc_cap": "none (E_T is not tracked in this cost scan)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA, "traffic": None,
                     "kernel": "k_contract (+ k_combine) in afqmc_local_energy, P = 8",
                     "ms_per_launch": ref["contraction_ms"], "flops_per_launch": flops},
        "scan": rows,
        "linear_fit_ms_per_step_vs_P": {"slope_ms": float(slope), "intercept_ms": float(icept)},
    }
    print(json.dumps(out))


def fixed_error_study(args):
    """Walker-steps/s at fixed energy error on the FP64 workload's system (M=64,
    N=16, 256 vectors, K=64, 512 walkers x 8 paths, tau = 0.005), every run in
    the stabilised form (STABLE), n_seeds independent runs of warmup + steps
    steps per configuration; a run's energy is its mixed estimate over the
    measured steps and sigma is the spread of those energies over the seeds.

    The energy depends on the Metropolis sweeps per step: with few sweeps the
    paths lag the walkers and the estimate is biased (the paper's one sweep
    assumes the chains re-equilibrate quickly).  So each form is run at a
    range of sweeps: the FP64 random walk (step 0.3; its one-sweep sigma is
    the error eps), the mixed-precision random walks at one sweep, and the
    learned proposal (BF16 network trained on the GPU during the warm-up, then
    frozen; FP32 contraction products).  E_inf, the converged energy, is the
    mean of the two most-swept configurations of the two samplers, which must
    agree.  eps is the statistical error of one run, sigma pooled over every
    configuration.  A configuration reaches eps if its bias |E - E_inf| is
    below eps; its time to eps is then T (sigma^2 / (eps^2 - bias^2)) with T
    the wall time of one run's measured steps, and its walker-steps/s at
    fixed error is walkers x measured steps / time to eps.  The line's value
    is the best configuration's rate; configurations that never reach eps
    report none."""
    import torch
    import afqmc_inputs as ai
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D

    sys_, run = ai.workload(1)
    nw, P = run.W, run.P
    n_seeds, n_eq, n_meas = args.seeds, args.warmup, args.steps
    s_train = 0.5

    def one(form, ns, seed):
        prec = {"fp64": A.PREC_FP64, "fp32": A.PREC_FP32, "bf16x3": A.PREC_BF16X3,
                "bf16": A.PREC_BF16, "learned": A.PREC_FP32}[form]
        common = dict(n_taylor=run.n_taylor, max_walkers=nw, xbar_cap=STABLE["xbar_cap"],
                      precision=prec, walker_c64=form in ("fp32", "bf16x3", "bf16"),
                      weight_mode=A.WEIGHT_LOCAL)
        if form == "learned":
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_LEARNED, rw_step=s_train,
                            **common)
            p = ai.mlp_params(np.random.default_rng(8), sys_.M, sys_.K, last_scale=0.0)
            p["b3"][sys_.K:] = 4 * np.arctanh(np.log(s_train * s_train) / 4)
            A.afqmc_mlp_init(ctx, A.PREC_BF16, A.mlp_pack(p), lr=1e-3)
            A.afqmc_mlp_set_training(ctx, True)
        else:
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_RW, rw_step=RW_STEP_FP64,
                            **common)
        st = D.init_walkers(ctx, sys_.phi0, nw, seed)
        est = torch.zeros(n_eq + n_meas, 2, dtype=torch.float64, device="cuda")
        ref = D.EnergyReference(ctx)
        for i in range(n_eq):
            D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=ns, n_qr=run.n_qr,
                   n_pc=1)
            ref.update(i, est)
        if form == "learned":  # freeze: network moves only from here on
            trained = A.afqmc_mlp_get_params(ctx)
            ctx.close()
            ctx = A.Context(sys_, P, run.dtau, proposal=A.PROPOSAL_LEARNED, rw_step=0.0,
                            **common)
            A.afqmc_mlp_init(ctx, A.PREC_BF16, trained)
            ref.attach(ctx)
        nacc = torch.zeros(nw, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_eq, n_eq + n_meas):
            D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=ns, n_qr=run.n_qr,
                   n_pc=1)
            ref.update(i, est)
            nacc += st.nacc
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        e = est[n_eq:].cpu().numpy()
        en = float(e[:, 0].sum() / e[:, 1].sum())
        return {"energy": en, "seconds": dt, "reblocked": reblock(e[:, 0] / e[:, 1]),
                "acceptance": float(nacc.sum().item()) / (n_meas * nw * P * ns),
                "finite": bool(np.all(np.isfinite(e)))}

    plan = [("fp64", ns) for ns in args.fe_sweeps_rw] + \
           [("fp32", 1), ("bf16x3", 1), ("bf16", 1)] + \
           [("learned", ns) for ns in args.fe_sweeps_learned]
    res = {}
    for form, ns in plan:
        runs = []
        for k in range(n_seeds):
            r = one(form, ns, 7001 + 97 * k)
            runs.append(r)
            print(f"{form} sweeps {ns} seed {k}: E = {r['energy']:.4f} (reblocked +- "
                  f"{r['reblocked']:.4f}), {1e3 * r['seconds'] / n_meas:.2f} ms/step, "
                  f"acceptance {r['acceptance']:.3f}", file=sys.stderr, flush=True)
        en = np.array([r["energy"] for r in runs])
        T = float(np.mean([r["seconds"] for r in runs]))
        res[f"{form}-sweeps{ns}"] = {
            "form": form, "sweeps": ns, "energies": en.tolist(), "energy": float(en.mean()),
            "sigma_run": float(en.std(ddof=1)),
            "error_of_mean": float(en.std(ddof=1) / np.sqrt(n_seeds)),
            "reblocked_sigma_run_mean": float(np.mean([r["reblocked"] for r in runs])),
            "seconds_per_run": T, "ms_per_step": 1e3 * T / n_meas,
            "walker_steps_per_s": nw * n_meas / T,
            "acceptance": float(np.mean([r["acceptance"] for r in runs])),
            "finite": all(r["finite"] for r in runs)}
    rw_top = f"fp64-sweeps{max(args.fe_sweeps_rw)}"
    ln_top = f"learned-sweeps{max(args.fe_sweeps_learned)}"
    a, b = res[rw_top], res[ln_top]
    e_inf = 0.5 * (a["energy"] + b["energy"])
    e_inf_err = 0.5 * float(np.hypot(a["error_of_mean"], b["error_of_mean"]))
    samplers_agree = bool(abs(a["energy"] - b["energy"])
                          <= 3 * np.hypot(a["error_of_mean"], b["error_of_mean"]))
    # the statistical error of one run: the seed-to-seed spread pooled over every
    # configuration (a few seeds per configuration make each spread alone a poor
    # estimate; reblocking single runs understates it: reblocked_over_pooled)
    pooled_var = float(np.mean([d["sigma_run"] ** 2 for d in res.values()]))
    sigma = float(np.sqrt(pooled_var))
    eps = sigma
    best = None
    for key, d in res.items():
        bias = d["energy"] - e_inf
        d["bias_vs_converged"] = bias
        d["reaches_eps"] = bool(abs(bias) < eps)
        if d["reaches_eps"]:
            d["time_to_eps_s"] = d["seconds_per_run"] * sigma ** 2 / (eps ** 2 - bias ** 2)
            d["walker_steps_per_s_at_eps"] = nw * n_meas / d["time_to_eps_s"]
            if best is None or d["walker_steps_per_s_at_eps"] > res[best]["walker_steps_per_s_at_eps"]:
                best = key
        else:
            d["time_to_eps_s"] = None
            d["walker_steps_per_s_at_eps"] = None
    per_form = {}
    for key, d in res.items():
        f = d["form"]
        if d["walker_steps_per_s_at_eps"] is not None and (
                f not in per_form or d["walker_steps_per_s_at_eps"] > per_form[f][1]):
            per_form[f] = (key, d["walker_steps_per_s_at_eps"])
    out = {
        "metric": METRIC,
        "value": res[best]["walker_steps_per_s_at_eps"] if best else None,
        "unit": "walker-steps/s",
        "n_gpus": 1, "steps": n_meas, "warmup": n_eq,
        "ms_per_step": res[best]["ms_per_step"] if best else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed (see configurations)", "data": "synthetic",
        "config": {"workload": f"fixed-error-gauss-M{sys_.M}-N{sys_.N}-G{sys_.n_chol}-K{sys_.K}"
                               f"-W{nw}-P{P}-dtau{run.dtau}", "walkers": nw, "paths": P,
                   "seeds_per_configuration": n_seeds, "rw_step": RW_STEP_FP64,
                   "network_train_step": s_train, "L_scale": L_SCALE, **STABLE},
        "value_configuration": best,
        "eps": eps, "eps_is": "the statistical error of one run (seed-to-seed spread pooled over "
                              "every configuration); a configuration reaches it if its bias "
                              "against the converged energy is smaller",
        "sigma_run_pooled": sigma,
        "reblocked_over_pooled": float(np.sqrt(np.mean([d["reblocked_sigma_run_mean"] ** 2
                                                          for d in res.values()])) / sigma),
        "converged_energy": e_inf, "converged_energy_error": e_inf_err,
        "converged_from": [rw_top, ln_top], "samplers_agree_within_3_sigma": samplers_agree,
        "best_per_form": {f: {"configuration": k, "walker_steps_per_s_at_eps": v}
                          for f, (k, v) in per_form.items()},
        "configurations": res,
    }
    print(json.dumps(out))


def uneven_study(args):
    """Uneven batch (32 systems, M in [24, 160], N = M/4, 4M vectors, K = M/2,
    walkers log-uniform in [64, 1024], 4 paths): aggregate walker-steps/s of the
    autotuned batch (replays of one captured graph with parallel branches)
    against the same systems stepped one after another through the per-system
    calls on one stream, and per-system agreement: a batch with the default
    kernel families against each system alone, estimator sums step by step."""
    import torch
    import afqmc_inputs as ai
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D

    systems, runs = ai.workload(3)
    # local-energy weights with the force-bias cap (STABLE without the E_L cap: the
    # replayed graph fixes every kernel argument, so E_T cannot move during the run)
    specs = [(s, r.P, r.dtau, dict(xbar_cap=STABLE["xbar_cap"], weight_mode=A.WEIGHT_LOCAL))
             for s, r in zip(systems, runs)]
    walkers = [r.W for r in runs]
    total_w = sum(walkers)
    flops = sum(contraction_flops(s.M, s.N, s.n_chol) * r.W * r.P for s, r in zip(systems, runs))
    seed = 2003
    t_build = time.perf_counter()
    b = A.Batch(specs, walkers, seed=seed, n_sweep=1, n_qr=10, n_pc=1, w_cap=0.0,
                max_branches=4, autotune=True, history=64)
    print(f"uneven batch built and tuned in {time.perf_counter() - t_build:.1f} s, cycle "
          f"{b.cycle} steps", file=sys.stderr, flush=True)
    n_cycles = max(1, args.steps // b.cycle)
    b.run(1)
    torch.cuda.synchronize()
    _, steps0 = b.estimates()
    t0 = time.perf_counter()
    b.run(n_cycles)
    sums, steps = b.estimates()
    dt = time.perf_counter() - t0
    n_steps = n_cycles * b.cycle
    fam, br, ms, nb = b.plan()
    energies = []
    for i in range(b.n):     # mean and spread of the per-step energies of the timed steps
        idx = [t % b.history for t in range(int(steps0[i]), int(steps[i]))][-b.history:]
        e = sums[i, idx, 0] / sums[i, idx, 1]
        energies.append({"M": systems[i].M, "N": systems[i].N, "walkers": walkers[i],
                         "energy": float(np.mean(e)),
                         "energy_err": float(np.std(e, ddof=1) / np.sqrt(len(e)))})
    b.close()
    print(f"batch: {1e3 * dt / n_steps:.1f} ms/step", file=sys.stderr, flush=True)

    # agreement: a batch with each system's default kernel family (no tuner)
    # and each system alone through the per-system calls, same seeds, 20 steps
    n_check = 20
    bv = A.Batch(specs, walkers, seed=seed, n_sweep=1, n_qr=10, n_pc=1, w_cap=0.0,
                 max_branches=4, autotune=False, history=64)
    bv.run(n_check // bv.cycle)
    vsums, _ = bv.estimates()
    bv.close()
    agree, seq_ms = [], 0.0
    for i, (s, P, dtau, kw) in enumerate(specs):
        ctx = A.Context(s, P, dtau, max_walkers=walkers[i], **kw)
        st = D.init_walkers(ctx, s.phi0, walkers[i], seed + i)
        est = torch.zeros(n_check, 2, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(n_check):
            D.step(ctx, st, seed + i, k, est[k], n_pc=1)
        torch.cuda.synchronize()
        seq_ms += 1e3 * (time.perf_counter() - t1) / n_check
        ref = est.cpu().numpy()
        got = vsums[i, :n_check]
        scale = np.maximum(np.abs(ref), 1e-300)
        agree.append(float(np.max(np.abs(got - ref) / scale)))
        ctx.close()
    print(f"sequential: {seq_ms:.1f} ms/step; per-system max relative difference of the "
          f"estimator sums, batch vs alone: {max(agree):.1e}", file=sys.stderr, flush=True)

    step_s = dt / n_steps
    achieved = flops / step_s / 1e12
    out = {
        "metric": METRIC,
        "value": total_w / step_s,
        "unit": "walker-steps/s",
        "n_gpus": 1, "steps": n_steps, "warmup": b.cycle,
        "ms_per_step": 1e3 * step_s,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "uneven-32-systems-M24-160", "systems": len(specs),
                   "M_range": [min(s.M for s in systems), max(s.M for s in systems)],
                   "walkers": total_w, "paths": 4, "cycle_steps": b.cycle,
                   "branches": nb, "families": [int(f) for f in fam],
                   "L_scale": L_SCALE, "weights": "local energy", "xbar_cap": STABLE["xbar_cap"],
                   "eloc_cap": "none (the replayed graph fixes E_T)", "comb_every": 1,
                   "comb_weights_reset_to": 1.0, "weight_cap": 0.0},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA, "traffic": None,
                     "kernel": "all systems' contractions per whole step (a lower bound on the "
                               "contraction kernels' rate: the step's other kernels are included)",
                     "flops_per_step": flops},
        "sequential_ms_per_step": seq_ms,
        "speedup_vs_sequential": seq_ms * 1e-3 / step_s,
        "per_system_agreement": {
            "what": f"max relative difference of the per-step estimator sums over {n_check} "
                    "steps, batch (default kernel families) vs each system alone through the "
                    "per-system calls; 0 = bit-identical",
            "max": max(agree), "per_system": agree},
        "per_system_energies": energies,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="fp64",
                    choices=sorted(WORKLOADS) + ["learned", "uneven", "scan", "fixed-error"])
    ap.add_argument("--seeds", type=int, default=4,
                    help="independent runs per configuration (fixed-error workload)")
    ap.add_argument("--fe-sweeps-rw", type=int, nargs="+", default=[1, 2, 4, 8, 16, 32],
                    help="sweeps per step of the FP64 random walk (fixed-error workload)")
    ap.add_argument("--fe-sweeps-learned", type=int, nargs="+", default=[1, 2, 4, 8],
                    help="sweeps per step of the learned proposal (fixed-error workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (the plain copy kernel that "
                         "calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on exactly one GPU (one-GPU build); --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import afqmc_inputs as ai
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D

    # the CPU baseline runs first, in processes started before anything here
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline and args.workload == "fp64" and not args.copy_calibration:
        prop, rws = PROPOSAL_OVERRIDE["fp64"]
        cpu = cpu_baseline(1, 2001, oracle_form(prop, rws, 1, ai.workload(1)[1].dtau))
        print(f"cpu baseline: {cpu['value']:.2f} walker-steps/s on {cpu['cores']} cores",
              file=sys.stderr, flush=True)
    if not torch.cuda.is_available():
        print("no GPU: the HIP path cannot run", file=sys.stderr)
        sys.exit(1)
    A.load_library()
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 5}))
        return
    if args.workload == "learned":
        learned_study(args)
        return
    if args.workload == "uneven":
        uneven_study(args)
        return
    if args.workload == "scan":
        scan_study(args)
        return
    if args.workload == "fixed-error":
        fixed_error_study(args)
        return

    widx, precision, peak, dtype = WORKLOADS[args.workload]
    sys_, run = ai.workload(widx)
    nw, P, seed = run.W, run.P, 2001
    proposal, rw_step = PROPOSAL_OVERRIDE.get(
        args.workload, (run.proposal, run.rw_step if run.proposal == A.PROPOSAL_RW else None))
    # the stabilised form of every per-step leg: local-energy weights, force-bias
    # modulus capped at 1, Re E_L capped at E_T +- sqrt(2 / tau) with the E_T
    # schedule of driver.EnergyReference, comb every step with the weights reset
    # to 1 (a common factor, which cancels in the mixed estimator)
    xbar_cap, n_pc, w_cap = STABLE["xbar_cap"], STABLE["comb_every"], 0.0
    c64 = precision != 0 and getattr(sys_, "trial_kind", 0) == 0
    ctx = A.Context(sys_, P, run.dtau, n_taylor=run.n_taylor, max_walkers=nw, xbar_cap=xbar_cap,
                    precision=precision, proposal=proposal, rw_step=rw_step, walker_c64=c64,
                    weight_mode=A.WEIGHT_LOCAL)
    st = D.init_walkers(ctx, sys_.phi0, nw, seed)
    est = torch.zeros(args.warmup + args.steps, 2, dtype=torch.float64, device="cuda")
    ref = D.EnergyReference(ctx)

    for i in range(args.warmup):
        D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=run.n_sweep,
               n_qr=run.n_qr, n_pc=n_pc, w_cap=w_cap)
        ref.update(i, est)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        i = args.warmup + k
        D.step(ctx, st, seed, i, est[i], e_shift=ref.e_shift, n_sweep=run.n_sweep,
               n_qr=run.n_qr, contract_events=evs[k], n_pc=n_pc, w_cap=w_cap)
        ref.update(i, est)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    contract_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    flops = contraction_flops(sys_.M, sys_.N, sys_.n_chol, ctx.ctrial) * nw * P
    achieved = flops / (contract_ms * 1e-3) / 1e12
    e = est.cpu().numpy()
    energies = e[:, 0] / e[:, 1]
    if not np.all(np.isfinite(energies)):
        w = st.w.cpu().numpy()
        print("non-finite energy in the benchmark run:", e.tolist(), "e_shift", ref.e_shift,
              "weights: min", w.min(), "max", w.max(), "n_zero", int((w == 0).sum()),
              "n_nonfinite", int((~np.isfinite(w)).sum()), file=sys.stderr)
        sys.exit(1)

    wname = (sys_.name if ctx.ctrial else
             f"gauss-M{sys_.M}-N{sys_.N}-G{sys_.n_chol}-K{sys_.K}")
    out = {
        "metric": METRIC,
        "value": nw * args.steps / dt,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{wname}-W{nw}-P{P}-dtau{run.dtau}-qr{run.n_qr}-"
                               + (f"rw{rw_step}" if proposal == A.PROPOSAL_RW else "prior"),
                   "walkers": nw, "paths": P, "M": sys_.M, "N": sys_.N,
                   "n_chol": sys_.n_chol, "K": sys_.K,
                   "proposal": "random walk" if proposal == A.PROPOSAL_RW else "prior",
                   "rw_step": rw_step if proposal == A.PROPOSAL_RW else None,
                   "L_scale": L_SCALE, "L_scale_note": L_SCALE_NOTE, **STABLE,
                   "walkers_complex64": c64},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload),
                     "kernel": ("k_contract" if sys_.M <= 64 and sys_.N <= 16 and precision == 0
                                and not ctx.ctrial else
                                "k_contract_sh" if precision in (1, 2, 3) and not ctx.ctrial
                                else "k_contract_g")
                               + (" (complex trial)" if ctx.ctrial else "")
                               + " (+ k_combine) in afqmc_local_energy",
                     "ms_per_launch": contract_ms, "flops_per_launch": flops},
        "energy_last": float(energies[-1]),
        "acceptance_last_step": float(st.nacc.sum().item()) / (nw * P * run.n_sweep),
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
