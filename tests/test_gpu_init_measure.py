"""Initialisation from the trial and measurement with extra paths (App. B,
Initialization and Measurement) through the C ABI, against the FP64 oracle on
the same seeds: the walker fields, walkers, paths, log-overlaps and weights of
afqmc_init_metropolis, and the corrected mixed-estimator sums, correction
factors and local energies of the measurement; plus the beta = 0 energy of a
large GPU population against the exact variational energy of the tiny trial."""
import json
import math
import os
import sys

import numpy as np
import pytest

import afqmc_inputs as ai
from oracle import afqmc_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_18519_amd import afqmc as A
    A.load_library()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def check_logov(got, ref):
    ok = np.isfinite(ref.real)
    assert np.array_equal(np.isfinite(got.real), ok)
    d = np.abs(np.exp(got[ok] - ref[ok]) - 1.0)
    assert d.max(initial=0.0) <= TOL, d.max()


CASES = {
    # name: (system factory, P, nw, proposal, rw_step)
    "tiny-ising-M8": (lambda: ai.tiny_ising(), 4, 24, 0, 0.5),
    "gauss-M20-N5-ragged-prior": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5),
                                  3, 7, 0, 0.5),
    "gauss-M20-N5-ragged-rw": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5),
                               3, 7, 1, 0.3),
    "gauss-M72-N20-rw": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7),
                         2, 3, 1, 0.2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_init_metropolis_matches_oracle(case):
    from paper_2505_18519_amd import afqmc as A
    mk, P, nw, prop, rw = CASES[case]
    s = mk()
    _say("case", case)
    seed, n_pair, n_burn = 31, 3, 2
    ost, oyw = O.init_metropolis(s, nw, P, seed, n_pair, n_burn, proposal=prop, rw_step=rw)
    ctx = A.Context(s, P, 0.01, max_walkers=nw, proposal=prop, rw_step=rw)
    z = dict(device="cuda")
    yw = torch.zeros(nw, s.K, dtype=torch.float64, **z)
    phi = torch.zeros(nw, 2, s.M, s.N, dtype=torch.complex128, **z)
    y = torch.zeros(nw, P, s.K, dtype=torch.float64, **z)
    phiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, **z)
    logov = torch.zeros(nw, P, dtype=torch.complex128, **z)
    w = torch.zeros(nw, dtype=torch.float64, **z)
    A.afqmc_init_metropolis(ctx, nw, seed, n_pair, n_burn, yw, phi, y, phiT, logov, w)
    torch.cuda.synchronize()
    # accept decisions are exact; accepted Gaussian proposals carry the
    # device's Box-Muller normals, equal to the oracle's within a few ulp
    assert np.abs(host(yw) - oyw).max() <= 4e-15 * max(np.abs(oyw).max(), 1.0)
    assert np.abs(host(y) - ost.y).max() <= 4e-15 * max(np.abs(ost.y).max(), 1.0)
    assert rel(host(phiT), ost.phiT) <= 1e-12
    assert rel(host(phi), ost.phi) <= 1e-12
    check_logov(host(logov), ost.logov)
    assert np.abs(host(w) - ost.w).max() <= 1e-12 * P
    assert np.all(np.abs(ost.w - P) <= 1e-12 * P)


MEAS = {
    # name: (system factory, P, P', nw)
    "tiny-ising-M8": (lambda: ai.tiny_ising(), 4, 9, 10),
    "gauss-M48-N11": (lambda: ai.small_gaussian(M=48, N=11, n_chol=40, K=12, seed=6), 3, 8, 4),
    "cfg-M64-N16-G256": (lambda: ai.workload(1)[0], 8, 12, 3),
    "gauss-M96-N24": (lambda: ai.small_gaussian(M=96, N=24, n_chol=48, K=32, seed=8), 2, 5, 2),
}


@pytest.mark.parametrize("case", list(MEAS))
def test_measurement_with_extra_paths_matches_oracle(case):
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    mk, P, P2, nw = MEAS[case]
    s = mk()
    _say("case", case)
    rng = np.random.default_rng(17)
    phi = ai.random_walkers(rng, s, nw, spread=0.5)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    w = rng.uniform(0.5, 1.5, size=nw)
    seed, i, n_sweep, dtau = 77, 5, 2, 0.01
    num, den, e2, R = O.measure_extra(s, phi, y, phiT, logov, w, seed, O.MEASURE_STEP + i, P2,
                                      n_sweep, dtau)
    ctx = A.Context(s, P, dtau, max_walkers=nw)
    st = D.Walkers(ctx, nw)
    st.phi.copy_(dev(phi))
    st.y.copy_(dev(y))
    st.phiT.copy_(dev(phiT))
    st.logov.copy_(dev(logov))
    st.w.copy_(dev(w))
    mctx = A.Context(s, P2, dtau, max_walkers=nw)
    m = D.Measurement(mctx, nw)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    D.measure_extra(m, st, seed, i, out, n_sweep)
    torch.cuda.synchronize()
    g = host(out)
    assert abs(g[0] - num) <= TOL * max(abs(num), 1.0)
    assert abs(g[1] - den) <= TOL * max(abs(den), 1.0)
    assert np.abs(host(m.R) - R).max() <= TOL * max(np.abs(R).max(), 1.0)
    assert np.abs(host(m.eloc) - e2).max() <= TOL * max(np.abs(e2).max(), 1.0)
    # the walkers' own paths are untouched
    assert np.array_equal(host(st.y), y)


def test_beta_zero_energy_is_the_variational_energy():
    """A large GPU population initialised from the tiny trial: the mixed
    estimate at beta = 0, plain and with a measurement trial of 3P paths,
    equals the exact <Psi_T|H|Psi_T>/<Psi_T|Psi_T> within 4 sigma."""
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    g = json.load(open(os.path.join(GOLDEN, "tiny_ising_ed.json")))
    s = ai.tiny_ising()
    nw, P = 20000, 8
    ctx = A.Context(s, P, 0.01, max_walkers=nw)
    st = D.init_walkers_metropolis(ctx, nw, 5, n_pair=10, n_burn=2)
    A.afqmc_green(ctx, nw, st.phi, st.phiT, st.logov, st.theta)
    A.afqmc_local_energy(ctx, nw, st.phiT, st.theta, st.logov, st.eloc, None, st.xbar)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    A.afqmc_estimator(ctx, nw, st.w, st.eloc, out)
    m = D.Measurement(A.Context(s, 3 * P, 0.01, max_walkers=nw), nw)
    out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    D.measure_extra(m, st, 5, 0, out2, n_sweep=3)
    torch.cuda.synchronize()
    e = host(st.eloc).real
    e2 = host(m.eloc).real
    err = e.std(ddof=1) / math.sqrt(nw)
    err2 = e2.std(ddof=1) / math.sqrt(nw)
    o, o2 = host(out), host(out2)
    _say(f"E(beta=0) {o[0] / o[1]:.6f} +- {err:.6f}, with 3P paths {o2[0] / o2[1]:.6f} +- "
         f"{err2:.6f}, exact E_var {g['E_var']:.6f}")
    assert np.all(host(st.w) == P)
    assert abs(o[0] / o[1] - g["E_var"]) < 4 * err
    assert abs(o2[0] / o2[1] - g["E_var"]) < 4 * err2
