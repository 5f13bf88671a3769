"""Uneven batching through the C ABI: a batch of systems of different size,
stepped by replays of one captured graph with parallel branches (real and
complex trial families side by side), gives every
system exactly the per-step estimates of that system run alone through the
per-system calls with the same seed (the same kernels on the same inputs), and
the autotuned batch runs and reports a valid plan."""
import sys

import numpy as np
import pytest

import afqmc_inputs as ai
from oracle import afqmc_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_18519_amd import afqmc as A
    A.load_library()


SYSTEMS = [
    # (system, P, walkers, rw proposal?)  -- both kernel families, ragged sizes
    (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=71), 4, 23, False),
    (lambda: ai.small_gaussian(M=48, N=11, n_chol=40, K=12, seed=72), 3, 9, True),
    (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=73), 2, 5, False),
    (lambda: ai.tiny_ising(), 8, 16, False),
    # a multi-slice (complex) trial: trial determinants twice the size
    (lambda: ai.imaginary_time_trial(ai.tiny_ising(), 2, 0.05), 4, 12, True),
]
DTAU, XCAP, WCAP, SEED = 0.01, 1.0, 4.0, 900


def _specs():
    from paper_2505_18519_amd import afqmc as A
    out = []
    for mk, P, nw, rw in SYSTEMS:
        s = mk()
        kw = dict(xbar_cap=XCAP)
        if rw:
            kw.update(proposal=A.PROPOSAL_RW, rw_step=0.3)
        out.append((s, P, nw, kw))
    return out


def _alone(s, P, nw, kw, seed, n_steps):
    """The same system through the per-system calls (driver.step)."""
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    ctx = A.Context(s, P, DTAU, max_walkers=nw, **kw)
    st = D.init_walkers(ctx, s.phi0, nw, seed)
    est = torch.zeros(n_steps, 2, dtype=torch.float64, device="cuda")
    for i in range(n_steps):
        D.step(ctx, st, seed, i, est[i], e_shift=0.0, n_sweep=1, n_qr=10, n_pc=1, w_cap=WCAP,
               normalize=True)
    torch.cuda.synchronize()
    return est.cpu().numpy()


def test_batch_equals_each_system_alone():
    from paper_2505_18519_amd import afqmc as A
    specs = _specs()
    b = A.Batch([(s, P, DTAU, kw) for s, P, nw, kw in specs], [nw for _, _, nw, _ in specs],
                seed=SEED, n_sweep=1, n_qr=10, n_pc=1, w_cap=WCAP, max_branches=2,
                autotune=False, history=64)
    assert b.cycle == 10
    b.run(2)
    sums, steps = b.estimates()
    fam, br, ms, nb = b.plan()
    _say("plan: families", fam, "branches", br, "n_branches", nb)
    assert np.all(steps == 20) and nb == 2
    for i, (s, P, nw, kw) in enumerate(specs):
        ref = _alone(s, P, nw, kw, SEED + i, 20)
        got = sums[i, :20]
        _say(s.name, "E first/last", got[0, 0] / got[0, 1], got[-1, 0] / got[-1, 1])
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), np.abs(got - ref).max()
    b.close()


def test_autotuned_batch_runs_and_reports_its_plan():
    from paper_2505_18519_amd import afqmc as A
    specs = _specs()
    walkers = [4 * nw for _, _, nw, _ in specs]        # populations that live ~100 steps
    b = A.Batch([(s, P, DTAU, kw) for s, P, nw, kw in specs], walkers,
                seed=SEED, n_sweep=1, n_qr=10, n_pc=1, w_cap=WCAP, max_branches=4,
                autotune=True, history=64)
    fam, br, ms, nb = b.plan()
    _say("tuned plan: families", fam, "branches", br, "step ms", np.round(ms, 3), "n_branches", nb)
    assert nb in (1, 2, 4) and np.all((br >= 0) & (br < nb)) and np.all(ms > 0)
    for i, (s, P, nw, kw) in enumerate(specs):
        if not (s.M <= 64 and s.N <= 16):
            assert fam[i] == 1          # only the workgroup-per-path family applies
    _, steps0 = b.estimates()
    b.run(3)
    sums, steps = b.estimates()
    assert np.all(steps == steps0 + 3 * b.cycle)
    last = [(steps[i] - 1) % b.history for i in range(b.n)]
    den = np.array([sums[i, last[i], 1] for i in range(b.n)])
    num = np.array([sums[i, last[i], 0] for i in range(b.n)])
    _say("last weight sums", den, "energies", num / np.where(den > 0, den, 1))
    # a population the phaseless projection has killed keeps W = 0 exactly
    assert np.all(np.isfinite(den)) and np.all(den >= 0) and (den > 0).sum() >= b.n - 1
    assert np.all(np.isfinite(num[den > 0] / den[den > 0]))
    b.close()


ORACLE_SYSTEMS = [
    # (system, P, walkers, proposal): an uneven set that spans both kernel
    # families, Ising and Gaussian hidden variables, the prior and the random
    # walk, and a system past M = 128 and N = 32 (nine row tiles, three column
    # tiles), as the uneven batches of M in [24, 160] hold
    (lambda: ai.tiny_ising(), 4, 6, 0),
    (lambda: ai.small_gaussian(M=24, N=6, n_chol=12, K=12, seed=81), 3, 5, 1),
    (lambda: ai.small_gaussian(M=70, N=17, n_chol=20, K=16, seed=82), 2, 4, 0),
    (lambda: ai.small_gaussian(M=136, N=34, n_chol=16, K=24, seed=83), 2, 3, 1),
]


def test_batch_matches_the_oracle_step_for_step():
    """Each system of a batch (graph replays on two branches) against the
    oracle's whole steps from the same seed: the estimator sums of Eq.
    mixed_estimator at every one of 20 steps to 1e-9 relative (the comb, QR
    every 10 steps and the hand-off included), which also fixes the weights,
    since every comb draws its parents from them."""
    from paper_2505_18519_amd import afqmc as A
    specs, walkers = [], []
    for mk, P, nw, prop in ORACLE_SYSTEMS:
        s = mk()
        kw = dict(xbar_cap=XCAP)
        if prop == 1:
            kw.update(proposal=A.PROPOSAL_RW, rw_step=0.3)
        specs.append((s, P, DTAU, kw))
        walkers.append(nw)
    b = A.Batch(specs, walkers, seed=SEED, n_sweep=1, n_qr=10, n_pc=1, w_cap=WCAP,
                max_branches=2, autotune=False, history=64)
    b.run(2)
    sums, steps = b.estimates()
    b.close()
    assert np.all(steps == 20)
    for i, ((s, P, _, kw), nw) in enumerate(zip(specs, walkers)):
        _say("oracle batch system", s.name, "P", P, "walkers", nw)
        prop = ORACLE_SYSTEMS[i][3]
        st = O.init_state(s, nw, P, SEED + i)
        for t in range(20):
            st, rec = O.step(s, st, SEED + i, t, DTAU, n_taylor=10, n_sweep=1, n_qr=10,
                             proposal=prop, rw_step=0.3, xbar_cap=XCAP, n_pc=1, w_cap=WCAP,
                             normalize=True)
            num, den = sums[i, t]
            assert abs(den - rec["e_den"]) <= 1e-9 * rec["e_den"], (s.name, t)
            assert abs(num - rec["e_num"]) <= 1e-9 * max(abs(rec["e_num"]), rec["e_den"]), \
                (s.name, t, num, rec["e_num"])
