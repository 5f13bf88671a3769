"""Multi-slice (complex) trials through the C ABI against the FP64 oracle
(Sec. II.C, Eqs. trial and trial-AF; Sec. III.B): trial determinants, overlaps
and Green's functions, the Cholesky contraction (FP64 and FP32 products), the
walker move and weight, the Metropolis update of the paths, population
control of complex trial rows, and a short trajectory, on the same seeded
inputs.  Tolerances as for the real trial family: FP64 1e-10, accept
decisions exact, FP32 products 1e-4."""
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


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def check_logov(got, ref):
    ok = np.isfinite(ref.real)
    assert np.array_equal(np.isfinite(got.real), ok)
    d = np.abs(np.exp(got[ok] - ref[ok]) - 1.0)
    assert d.max(initial=0.0) <= TOL, d.max()


CASES = {
    # name: (system factory, P, nw) -- imaginary-time trials e^{-m tau_T H} Phi_0
    "tiny-M8-m2": (lambda: ai.imaginary_time_trial(ai.tiny_ising(), 2, 0.05), 6, 5),
    "gauss-M20-N5-m1": (lambda: ai.imaginary_time_trial(
        ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 1, 0.05, n_gen=8), 3, 4),
    "gauss-M48-N24-m2": (lambda: ai.imaginary_time_trial(
        ai.small_gaussian(M=48, N=24, n_chol=16, K=8, seed=6), 2, 0.02), 2, 2),
    "cfg-M64-N16-G256-m2": (lambda: ai.imaginary_time_trial(ai.workload(1)[0], 2, 0.01, n_gen=32),
                            4, 2),
    "gauss-M96-N16-m1": (lambda: ai.imaginary_time_trial(
        ai.small_gaussian(M=96, N=16, n_chol=24, K=8, seed=8), 1, 0.02, n_gen=12), 2, 2),
}


def make_ctx(s, P, nw, **kw):
    from paper_2505_18519_amd import afqmc as A
    return A.Context(s, P, 0.01, max_walkers=nw, **kw)


def state(s, P, nw, seed, spread=0.5):
    rng = np.random.default_rng(seed)
    phi = ai.random_walkers(rng, s, nw, spread=spread)
    y = 0.7 * rng.normal(size=(nw, P, s.K))
    return rng, phi, y


@pytest.mark.parametrize("case", list(CASES))
def test_trial_overlap_green(case):
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    _say("case", case)
    ctx = make_ctx(s, P, nw)
    rng, phi, y = state(s, P, nw, 1)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    dT = torch.zeros(nw, P, s.M, s.N, dtype=torch.complex128, device="cuda")
    A.afqmc_trial_build(ctx, nw, dev(y), dT)
    dl = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    dth = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, device="cuda")
    A.afqmc_green(ctx, nw, dev(phi), dT, dl, dth)
    torch.cuda.synchronize()
    assert rel(host(dT), phiT) <= 1e-12
    check_logov(host(dl), ell)
    for w in range(nw):
        assert rel(host(dth)[w], theta[w]) <= TOL


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_contraction(case, prec):
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    _say("case", case, "precision", prec)
    tol = TOL if prec == 0 else 1e-4
    ctx = make_ctx(s, P, nw, precision=prec)
    rng, phi, y = state(s, P, nw, 2)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, 0.01)
    _, theta = O.green(phiT, phi)
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_ep = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    d_vb = torch.zeros(nw, P, s.n_chol, dtype=torch.complex128, device="cuda")
    d_xb2 = torch.zeros_like(d_xb)
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, d_ep, d_xb)
    A.afqmc_force_bias(ctx, nw, dev(phiT), dev(theta), dev(ell), d_xb2, d_vb)
    torch.cuda.synchronize()
    assert np.abs(host(d_ep) - ep).max() <= tol * max(np.abs(ep).max(), 1)
    assert np.abs(host(d_el) - eloc).max() <= tol * max(np.abs(eloc).max(), 1)
    for w in range(nw):
        assert rel(host(d_xb)[w], xbar[w]) <= tol
        assert rel(host(d_xb2)[w], xbar[w]) <= tol
        for p in range(P):
            assert rel(host(d_vb)[w, p], vb[w, p]) <= tol


@pytest.mark.parametrize("case", list(CASES))
def test_propagate(case):
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    _say("case", case)
    ctx = make_ctx(s, P, nw)
    rng, phi, y = state(s, P, nw, 3)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, 0.01)
    xi = rng.normal(size=(nw, s.n_chol))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, w0, 0.01, 10, -1.1)
    dphi, dw = dev(phi), dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), dev(xbar), dev(phiT), dev(ell), -1.1, dw, dref, dln)
    torch.cuda.synchronize()
    for w in range(nw):
        assert rel(host(dphi)[w], phin[w]) <= TOL
    check_logov(host(dln), elln)
    assert np.abs(host(dw) - wn).max() <= TOL * np.abs(wn).max()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("proposal", [0, 1])
def test_metropolis_and_population_control(case, proposal):
    from paper_2505_18519_amd import afqmc as A
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    _say("case", case, "proposal", proposal)
    ctx = make_ctx(s, P, nw, proposal=proposal, rw_step=0.15)
    rng, phi, y = state(s, P, nw, 4)
    phiT = O.trial_det(s, y)
    ell = O.log_overlap(phiT, phi)
    ref = np.exp(1j * rng.uniform(-0.3, 0.3, size=nw)) * rng.uniform(0.5, 2, size=nw)
    w0 = rng.uniform(0.5, 1.5, size=nw)
    seed, stp, nsw = 4321, 3, 2
    y2, phiT2, ell2, w2, nacc = O.metropolis(s, phi, y, phiT, ell, ref, w0, seed, stp, nsw,
                                             proposal=proposal, rw_step=0.15)
    dy, dT, dl, dw = dev(y), dev(phiT), dev(ell), dev(w0)
    dacc = torch.zeros(nw, dtype=torch.int32, device="cuda")
    A.afqmc_metropolis_x(ctx, nw, dev(phi), dy, dT, dl, dev(ref), dw, seed, stp, nsw, dacc)
    torch.cuda.synchronize()
    _say("accepted", nacc, "of", nw * P * nsw)
    assert np.array_equal(host(dacc), nacc)
    assert np.abs(host(dy) - y2).max() <= 4e-15 * max(np.abs(y2).max(), 1.0)
    assert rel(host(dT), phiT2) <= 1e-12
    check_logov(host(dl), ell2)
    assert np.abs(host(dw) - w2).max() <= TOL * np.abs(w2).max()
    # comb: complex trial rows (and y, logov) follow their parents bit for bit
    gT, gy, gl, gw = host(dT), host(dy), host(dl), host(dw)
    par = torch.zeros(nw, dtype=torch.int32, device="cuda")
    A.afqmc_population_control(ctx, nw, dev(phi), dw, dy, dT, dl, seed, stp, 0.0, parent=par)
    torch.cuda.synchronize()
    pa, _ = O.comb(gw, seed, stp)
    assert np.array_equal(host(par), pa)
    assert np.array_equal(host(dT), gT[pa])
    assert np.array_equal(host(dy), gy[pa])
    assert np.array_equal(host(dl), gl[pa])


def test_trajectory_matches_oracle():
    """Ten steps of the tiny workload with an m = 2 imaginary-time trial
    (prior proposal, comb every step) through driver.step against O.step."""
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    s = ai.imaginary_time_trial(ai.tiny_ising(), 2, 0.05)
    nw, P, dtau, seed = 16, 6, 0.01, 55
    ctx = A.Context(s, P, dtau, max_walkers=nw, proposal=A.PROPOSAL_RW, rw_step=0.3)
    st = D.init_walkers(ctx, s.phi0, nw, seed)
    ost = O.init_state(s, nw, P, seed)
    Eh, h1p = O.half_kinetic(s, dtau), O.h1_eff(s)
    est = torch.zeros(10, 2, dtype=torch.float64, device="cuda")
    for i in range(10):
        D.step(ctx, st, seed, i, est[i], n_sweep=1, n_qr=5, n_pc=1, w_cap=4.0)
        ost, rec = O.step(s, ost, seed, i, dtau, n_qr=5, proposal=O.PROPOSAL_RW, rw_step=0.3,
                          Eh=Eh, h1p=h1p, n_pc=1, w_cap=4.0)
        e = host(est[i])
        assert abs(e[0] / e[1] - rec["e_num"] / rec["e_den"]) <= 1e-9 * abs(e[0] / e[1]), i
    torch.cuda.synchronize()
    assert rel(host(st.phi), ost.phi) <= 1e-9
    assert rel(host(st.phiT), ost.phiT) <= 1e-9
    assert np.abs(host(st.w) - ost.w).max() <= 1e-9


def test_unsupported_combinations_are_refused():
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    s = ai.imaginary_time_trial(ai.tiny_ising(), 1, 0.05)
    with pytest.raises(A.AfqmcError):
        A.Context(s, 4, 0.01, proposal=A.PROPOSAL_LEARNED)
    big = ai.imaginary_time_trial(ai.small_gaussian(M=128, N=32, n_chol=8, K=4, seed=3), 1, 0.02)
    with pytest.raises(A.AfqmcError):
        A.Context(big, 2, 0.01)
    ctx = A.Context(s, 4, 0.01, max_walkers=4)
    with pytest.raises(A.AfqmcError):
        D.init_walkers_metropolis(ctx, 4, 1)
