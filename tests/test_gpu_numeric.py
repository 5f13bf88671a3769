"""Numerical events through the C ABI: non-finite inputs fed from the host
(a NaN auxiliary field, a NaN Green's-function entry, an infinite hand-off
reference) give the oracle's data-level outcome (W = 0, E_L left out of the
estimator sums) for the walker concerned, leave every other walker equal to
the oracle, and raise that walker's AFQMC_NUMERIC_* flag bits, which
afqmc_numeric_flags reports as AFQMC_E_NUMERIC and clears.  With the numeric
check on, the per-step call itself returns AFQMC_E_NUMERIC."""
import sys

import numpy as np
import pytest

import afqmc_inputs as ai
from oracle import afqmc_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


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


CASES = {
    "tiny-ising-M8": (lambda: ai.tiny_ising(), 4, 6),
    "gauss-M72-N20": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 3, 5),
}


def _inputs(s, P, nw, seed):
    rng = np.random.default_rng(seed)
    phi = ai.random_walkers(rng, s, nw, spread=0.5)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    return rng, phi, phiT


@pytest.mark.parametrize("case", list(CASES))
def test_nan_field_kills_one_walker_and_is_flagged(case):
    _say("numeric: NaN field", case)
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw)
    rng, phi, phiT = _inputs(s, P, nw, 1)
    eloc, xbar, _, _, ell = O.local_energy(s, phi, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    xi[2, 3] = np.nan
    w0 = rng.uniform(0.5, 1.5, size=nw)
    with np.errstate(invalid="ignore", over="ignore"):
        phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, w0, dtau, 10, -0.5)
    assert wn[2] == 0.0
    dw = dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dev(phi), dev(xi), dev(xbar), dev(phiT), dev(ell), -0.5, dw, dref,
                      dln)
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 1 and flags[2] & A.NUMERIC_WEIGHT, flags
    assert np.count_nonzero(flags) == 1
    gw = host(dw)
    assert gw[2] == 0.0
    keep = np.arange(nw) != 2
    assert np.abs(gw[keep] - wn[keep]).max() <= TOL * np.abs(wn[keep]).max()
    # read and cleared: a second read reports nothing
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 0 and not flags.any()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_nan_green_function_flags_local_energy(case, prec):
    _say("numeric: NaN Theta", case, "precision", prec)
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw, precision=prec)
    rng, phi, phiT = _inputs(s, P, nw, 2)
    ell, theta = O.green(phiT, phi)
    theta[1, 0, 1, 2, 0] = np.nan
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, None, d_xb)
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 1, flags
    assert flags[1] & A.NUMERIC_ELOC and flags[1] & A.NUMERIC_XBAR, flags
    g_el = host(d_el)
    assert not np.isfinite(g_el[1])
    # the estimator leaves the flagged walker out, as the oracle's does
    w = rng.uniform(0.5, 1.5, size=nw)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    A.afqmc_estimator(ctx, nw, dev(w), d_el, out)
    num, den = O.estimator(w, g_el)
    g = host(out)
    assert np.isfinite(g).all()
    assert abs(g[0] - num) <= 1e-13 * abs(num) and abs(g[1] - den) <= 1e-13 * den
    assert abs(den - (w.sum() - w[1])) <= 1e-13 * den


@pytest.mark.parametrize("mode", [0, 2])
def test_non_finite_handoff_reference(mode):
    _say("numeric: hand-off reference, mode", mode)
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 3, 6
    ctx = A.Context(s, P, 0.01, max_walkers=nw, weight_mode=mode, proposal=A.PROPOSAL_RW,
                    rw_step=0.3)
    rng, phi, phiT = _inputs(s, P, nw, 3)
    y = ai.random_hidden(np.random.default_rng(3), s, nw, P)
    phiT = O.trial_det(s, y)
    ell = O.log_overlap(phiT, phi)
    ref = np.exp(1j * rng.uniform(-0.3, 0.3, size=nw))
    ref[4] = complex(np.inf, 0.0)
    w0 = rng.uniform(0.5, 1.5, size=nw)
    _, _, _, w2, _ = O.metropolis(s, phi, y, phiT, ell, ref, w0, 5, 1, 1, proposal=O.PROPOSAL_RW,
                                  rw_step=0.3, weight_mode=mode)
    assert w2[4] == 0.0
    dw = dev(w0)
    A.afqmc_metropolis_x(ctx, nw, dev(phi), dev(y), dev(phiT), dev(ell), dev(ref), dw, 5, 1, 1)
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 1 and flags[4] & A.NUMERIC_HANDOFF, flags
    assert np.array_equal(host(dw) == 0.0, w2 == 0.0)
    assert np.abs(host(dw) - w2).max() <= TOL * np.abs(w2).max()


def test_numeric_check_makes_the_call_report():
    _say("numeric: check mode")
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = ai.tiny_ising(), 4, 6
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw)
    A.afqmc_set_numeric_check(ctx, True)
    rng, phi, phiT = _inputs(s, P, nw, 4)
    eloc, xbar, _, _, ell = O.local_energy(s, phi, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    # finite inputs: no report
    A.afqmc_propagate(ctx, nw, dev(phi), dev(xi), dev(xbar), dev(phiT), dev(ell), 0.0,
                      dev(np.ones(nw)), dref, dln)
    xi[5, 0] = np.inf
    with pytest.raises(A.AfqmcError) as ei:
        A.afqmc_propagate(ctx, nw, dev(phi), dev(xi), dev(xbar), dev(phiT), dev(ell), 0.0,
                          dev(np.ones(nw)), dref, dln)
    assert ei.value.status == A.E_NUMERIC and "walker 5" in str(ei.value)
    # the flags stay readable after the report; each checking call reports its own
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 1 and flags[5] & A.NUMERIC_WEIGHT
    xi[5, 0] = 0.3
    A.afqmc_propagate(ctx, nw, dev(phi), dev(xi), dev(xbar), dev(phiT), dev(ell), 0.0,
                      dev(np.ones(nw)), dref, dln)
    A.afqmc_set_numeric_check(ctx, False)
    xi[0, 0] = np.nan
    A.afqmc_propagate(ctx, nw, dev(phi), dev(xi), dev(xbar), dev(phiT), dev(ell), 0.0,
                      dev(np.ones(nw)), dref, dln)    # asynchronous: no report by the call
    flags, n = A.afqmc_numeric_flags(ctx, nw)
    assert n == 1 and flags[0] & A.NUMERIC_WEIGHT
