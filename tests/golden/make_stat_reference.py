"""Writes tests/golden/stat_m64_local.json: the oracle's long-run energy of the
FP64 M = 64 workload in the stabilised local-energy form, the reference that
the GPU's independent runs are compared with.

Run from the repository root (a few tens of minutes per seed on 8 cores):
    python tests/golden/make_stat_reference.py [--seeds 5001 5002 ...] [--procs 7]

Workload: M = 64, N = 16, 256 vectors, K = 64 Gaussian hidden fields
(afqmc_inputs.workload(1)), P = 8 paths, 64 walkers, tau = 0.005, 2000 steps;
random-walk proposal of step 0.3, one sweep; QR every 10 steps; comb every
step with the weights reset to 1; local-energy weights (Sec. III.A) with the
force-bias modulus capped at 1 and Re E_L capped at E_T +- sqrt(2 / tau).
E_T schedule: 0 and no cap for steps 0..19; after step 19, and after every
step i with (i + 1) % 100 == 0 from 99 on, E_T = the mixed estimate over the
last (at most) 100 steps.  Measured segment: steps 500..1999.

The population is stepped in walker chunks on a process pool (each chunk with
its place in the population, so its random streams are those of the whole
population's step); the parent forms the estimator sums and combs the whole
population.  Only oracle/ and the input generator are used.
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import afqmc_inputs as ai  # noqa: E402
from oracle import afqmc_oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "stat_m64_local.json")

NW, P, DTAU, N_STEPS, MEASURE_FROM = 64, 8, 0.005, 2000, 500
RW_STEP, N_QR, XBAR_CAP = 0.3, 10, 1.0
ECAP = math.sqrt(2.0 / DTAU)

_S = {}


def _init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    s, _ = ai.workload(1)
    _S["sys"] = s
    _S["Eh"] = O.half_kinetic(s, DTAU)
    _S["h1p"] = O.h1_eff(s)


def _chunk_step(args):
    phi, w, y, phiT, logov, w0, seed, i, e_t = args
    s = _S["sys"]
    st = O.State(phi, w, y, phiT, logov)
    cap = None if e_t is None else (e_t, ECAP)
    st, rec = O.step(s, st, seed, i, DTAU, n_qr=N_QR, e_shift=0.0 if e_t is None else e_t,
                     proposal=O.PROPOSAL_RW, rw_step=RW_STEP, weight_mode=O.WEIGHT_LOCAL,
                     Eh=_S["Eh"], h1p=_S["h1p"], xbar_cap=XBAR_CAP, n_pc=0, eloc_cap=cap,
                     w0=w0)
    return st.phi, st.w, st.y, st.phiT, st.logov, rec["e_num"], rec["e_den"], int(rec["nacc"].sum())


def run_seed(seed, pool, n_chunks, log):
    s, _ = ai.workload(1)
    st = O.init_state(s, NW, P, seed)
    bounds = np.linspace(0, NW, n_chunks + 1).astype(int)
    num, den = np.zeros(N_STEPS), np.zeros(N_STEPS)
    e_t = None
    t0 = time.time()
    for i in range(N_STEPS):
        jobs = [(st.phi[a:b], st.w[a:b], st.y[a:b], st.phiT[a:b], st.logov[a:b], int(a), seed, i,
                 e_t) for a, b in zip(bounds[:-1], bounds[1:])]
        res = pool.map(_chunk_step, jobs)
        phi = np.concatenate([r[0] for r in res])
        w = np.concatenate([r[1] for r in res])
        y = np.concatenate([r[2] for r in res])
        phiT = np.concatenate([r[3] for r in res])
        logov = np.concatenate([r[4] for r in res])
        num[i] = math.fsum(r[5] for r in res)
        den[i] = math.fsum(r[6] for r in res)
        parent, w = O.comb(w, seed, i, 0.0, True)
        st = O.State(phi[parent], w, y[parent], phiT[parent], logov[parent])
        if i == 19 or (i >= 99 and (i + 1) % 100 == 0):
            a = max(0, i - 99)
            if den[a:i + 1].sum() > 0:
                e_t = num[a:i + 1].sum() / den[a:i + 1].sum()
        if (i + 1) % 100 == 0:
            log(f"seed {seed} step {i + 1}: E(step) = {num[i] / den[i]:.4f}  E_T = {e_t:.4f}  "
                f"acc = {sum(r[7] for r in res) / (NW * P):.3f}  {time.time() - t0:.0f} s")
    seg = slice(MEASURE_FROM, N_STEPS)
    blocks = [float(num[a:a + 100].sum() / den[a:a + 100].sum())
              for a in range(MEASURE_FROM, N_STEPS, 100)]
    return {"seed": seed, "energy": float(num[seg].sum() / den[seg].sum()),
            "block_means_100": blocks, "seconds": time.time() - t0}


def main():
    global N_STEPS, MEASURE_FROM
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, nargs="+", default=[5001, 5002, 5003, 5004])
    ap.add_argument("--procs", type=int, default=7)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--steps", type=int, default=N_STEPS)
    ap.add_argument("--measure-from", type=int, default=MEASURE_FROM)
    args = ap.parse_args()
    N_STEPS, MEASURE_FROM = args.steps, args.measure_from
    log = lambda m: print(m, flush=True)  # noqa: E731
    doc = {
        "what": "oracle mixed-estimate energy of the FP64 M=64 workload, stabilised local-energy "
                "form, one value per independent seed over the measured segment",
        "workload": "afqmc_inputs.workload(1): M=64 N=16 n_chol=256 K=64 Gaussian",
        "walkers": NW, "paths": P, "dtau": DTAU, "steps": N_STEPS, "measured_from": MEASURE_FROM,
        "proposal": "random walk", "rw_step": RW_STEP, "n_sweep": 1, "n_qr": N_QR,
        "comb": "every step, weights reset to 1", "weight_mode": "local energy",
        "xbar_cap": XBAR_CAP, "eloc_cap_half_width": ECAP,
        "e_t_schedule": "0 and no cap for steps 0..19; after step 19 and after every step i "
                        "with (i+1) % 100 == 0 from 99 on: mixed estimate of the last <= 100 steps",
        "runs": [],
    }
    if os.path.exists(args.out):
        old = json.load(open(args.out))
        if all(old.get(k) == doc[k] for k in doc if k != "runs"):
            doc["runs"] = old["runs"]
    done = {r["seed"] for r in doc["runs"]}
    ctx = mp.get_context("fork")
    with ctx.Pool(args.procs, initializer=_init) as pool:
        for seed in args.seeds:
            if seed in done:
                continue
            doc["runs"].append(run_seed(seed, pool, args.procs, log))
            e = np.array([r["energy"] for r in doc["runs"]])
            doc["mean"] = float(e.mean())
            doc["sigma_seed"] = float(e.std(ddof=1)) if len(e) > 1 else None
            doc["sigma_mean"] = (float(e.std(ddof=1) / math.sqrt(len(e)))
                                 if len(e) > 1 else None)
            with open(args.out, "w") as f:
                json.dump(doc, f, indent=1)
            log(f"seed {seed}: E = {doc['runs'][-1]['energy']:.4f}; written {args.out}")


if __name__ == "__main__":
    main()
