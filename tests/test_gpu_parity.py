"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Same seeded inputs on both sides; tolerances are those of the FP64 path:
log-overlaps |exp(l - l_ref) - 1| <= 1e-10, force bias normwise 1e-10 per
walker, energies |E - E_ref| <= 1e-10 max(|E_ref|, 1), determinants
normwise 1e-10, integer and accept decisions exact.
"""
import math
import sys

import numpy as np
import pytest

import afqmc_inputs as ai
from oracle import afqmc_oracle as O
from oracle import philox as PH

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


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    # name: (system factory, P, nw)
    "tiny-ising-M8": (lambda: ai.tiny_ising(), 8, 5),
    "gauss-M20-N5-ragged": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 3, 6),
    "gauss-M48-N11": (lambda: ai.small_gaussian(M=48, N=11, n_chol=40, K=12, seed=6), 4, 3),
    "cfg-M64-N16-G256": (lambda: ai.workload(1)[0], 8, 3),
    # edge shapes of the wavefront-per-path kernels: a single Cholesky vector and a
    # single path; 17 vectors (one flush of 16 staged diagonals plus a ragged one)
    # with 15 paths (a last workgroup with idle wavefronts)
    "gauss-M32-N8-G1-P1": (lambda: ai.small_gaussian(M=32, N=8, n_chol=1, K=4, seed=10), 1, 4),
    "gauss-M64-N16-G17-P5": (lambda: ai.small_gaussian(M=64, N=16, n_chol=17, K=8, seed=11), 5, 3),
    # one electron per spin: 1 x 1 overlaps in a single tile of rows (M = 3) and in
    # the workgroup-per-path kernels just past M = 64
    "gauss-M3-N1": (lambda: ai.small_gaussian(M=3, N=1, n_chol=5, K=2, seed=12), 2, 3),
    "gauss-M70-N1": (lambda: ai.small_gaussian(M=70, N=1, n_chol=9, K=4, seed=13), 3, 2),
    # every orbital occupied (N = M) in both kernel families
    "gauss-M16-N16": (lambda: ai.small_gaussian(M=16, N=16, n_chol=6, K=4, seed=14), 2, 3),
    "gauss-M32-N32": (lambda: ai.small_gaussian(M=32, N=32, n_chol=6, K=4, seed=15), 2, 2),
    # workgroup-per-path kernels (M > 64 or N > 16)
    "gauss-M72-N20-ragged": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 3, 3),
    "gauss-M96-N24": (lambda: ai.small_gaussian(M=96, N=24, n_chol=48, K=32, seed=8), 4, 2),
    "gauss-M128-N32": (lambda: ai.small_gaussian(M=128, N=32, n_chol=32, K=32, seed=9), 2, 2),
    # five row tiles (a padded 32-wide k block in BF16) by four packed column tiles
    # with ragged columns: the reduced-precision contraction's one-path form
    "gauss-M80-N27-ragged": (lambda: ai.small_gaussian(M=80, N=27, n_chol=20, K=12, seed=19), 3, 3),
    # past M = 128 and N = 32 (the uneven batches' largest systems): nine and ten
    # row tiles, three column tiles, ragged
    "gauss-M136-N34": (lambda: ai.small_gaussian(M=136, N=34, n_chol=24, K=40, seed=16), 2, 2),
    "gauss-M150-N20": (lambda: ai.small_gaussian(M=150, N=20, n_chol=20, K=24, seed=17), 3, 2),
    "gauss-M160-N40": (lambda: ai.small_gaussian(M=160, N=40, n_chol=24, K=40, seed=18), 2, 2),
}


def make_ctx(s, P, nw, dtau=0.01, **kw):
    from paper_2505_18519_amd import afqmc as A
    return A.Context(s, P, dtau, max_walkers=nw, **kw)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def check_logov(got, ref):
    ok_ref = np.isfinite(ref.real)
    assert np.array_equal(np.isfinite(got.real), ok_ref)
    d = np.abs(np.exp(got[ok_ref] - ref[ok_ref]) - 1.0)
    assert d.max(initial=0.0) <= TOL, d.max()


def state(s, P, nw, seed, spread=0.5):
    rng = np.random.default_rng(seed)
    phi = ai.random_walkers(rng, s, nw, spread=spread)
    y = ai.random_hidden(rng, s, nw, P)
    return rng, phi, y


@pytest.mark.parametrize("case", list(CASES))
def test_trial_build_overlap_green(case):
    _say("case", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, P, nw)
    rng, phi, y = state(s, P, nw, 1)
    phiT_ref = O.trial_det(s, y)
    dy = dev(y)
    dphiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, device="cuda")
    A.afqmc_trial_build(ctx, nw, dy, dphiT)
    torch.cuda.synchronize()
    assert rel(host(dphiT), phiT_ref) <= 1e-12
    ell_ref, theta_ref = O.green(phiT_ref, phi)
    dphi = dev(phi)
    dl = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    dth = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, device="cuda")
    A.afqmc_green(ctx, nw, dphi, dev(phiT_ref), dl, dth)
    dl2 = torch.zeros_like(dl)
    A.afqmc_overlap(ctx, nw, dphi, dev(phiT_ref), dl2)
    torch.cuda.synchronize()
    check_logov(host(dl), ell_ref)
    check_logov(host(dl2), ell_ref)
    for w in range(nw):
        for p in range(P):
            assert rel(host(dth)[w, p], theta_ref[w, p]) <= TOL


@pytest.mark.parametrize("case", list(CASES))
def test_force_bias_and_local_energy(case):
    _say("case", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    ctx = make_ctx(s, P, nw, dtau=dtau)
    rng, phi, y = state(s, P, nw, 2)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, dtau)
    _, theta = O.green(phiT, phi)
    dphiT, dth, dl = dev(phiT), dev(theta), dev(ell)
    G = s.n_chol
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_ep = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, G, dtype=torch.complex128, device="cuda")
    d_xb2 = torch.zeros(nw, G, dtype=torch.complex128, device="cuda")
    d_vb = torch.zeros(nw, P, G, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dphiT, dth, dl, d_el, d_ep, d_xb)
    A.afqmc_force_bias(ctx, nw, dphiT, dth, dl, d_xb2, d_vb)
    torch.cuda.synchronize()
    g_el, g_ep, g_xb, g_xb2, g_vb = map(host, (d_el, d_ep, d_xb, d_xb2, d_vb))
    assert np.abs(g_ep - ep).max() <= TOL * max(np.abs(ep).max(), 1)
    assert np.abs(g_el - eloc).max() <= TOL * max(np.abs(eloc).max(), 1)
    for w in range(nw):
        assert rel(g_xb[w], xbar[w]) <= TOL
        assert rel(g_xb2[w], xbar[w]) <= TOL
        for p in range(P):
            assert rel(g_vb[w, p], vb[w, p]) <= TOL


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_propagate(case, mode):
    _say("case", case, "mode", mode)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    ctx = make_ctx(s, P, nw, dtau=dtau, weight_mode=mode)
    rng, phi, y = state(s, P, nw, 3)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    e_shift = -1.3
    phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, w0, dtau, 10, e_shift, mode,
                                      eloc=eloc)
    dphi, dw = dev(phi), dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), dev(xbar), dev(phiT), dev(ell), e_shift, dw, dref, dln,
                      dev(eloc))
    torch.cuda.synchronize()
    for w in range(nw):
        assert rel(host(dphi)[w], phin[w]) <= TOL
    check_logov(host(dln), elln)
    assert np.abs(host(dw) - wn).max() <= TOL * np.abs(wn).max()
    assert np.abs(host(dref) - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("proposal", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_metropolis_and_handoff(case, proposal, mode):
    """Metropolis moves of the paths, then the hand-off projection of the
    weight mode: the cosine (SEPARATE, COMBINED) or the half-plane rule.  For
    modes 1 and 2 the reference phases span the whole circle, so walkers on
    both sides of the half-plane boundary occur."""
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    if s.hidden_kind == 0 and proposal == 1:
        pytest.skip("random walk is for Gaussian hidden variables")
    _say("case", case, "proposal", proposal, "mode", mode)
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, P, nw, proposal=proposal, rw_step=0.3, weight_mode=mode)
    rng, phi, y = state(s, P, nw, 4)
    phiT = O.trial_det(s, y)
    ell = O.log_overlap(phiT, phi)
    spread = 0.3 if mode == 0 else math.pi
    ref = np.exp(1j * rng.uniform(-spread, spread, size=nw)) * rng.uniform(0.5, 2, size=nw)
    w0 = rng.uniform(0.5, 1.5, size=nw)
    seed, stp, nsw = 1234, 7, 2
    y2, phiT2, ell2, w2, nacc = O.metropolis(s, phi, y, phiT, ell, ref, w0, seed, stp, nsw,
                                             proposal=proposal, rw_step=0.3, weight_mode=mode)
    dy, dphiT, dl, dw = dev(y), dev(phiT), dev(ell), dev(w0)
    dacc = torch.zeros(nw, dtype=torch.int32, device="cuda")
    A.afqmc_metropolis_x(ctx, nw, dev(phi), dy, dphiT, dl, dev(ref), dw, seed, stp, nsw, dacc)
    torch.cuda.synchronize()
    assert np.array_equal(host(dacc), nacc), (host(dacc), nacc)
    # accept decisions are exact; accepted Gaussian proposals carry the
    # device's Box-Muller normals, equal to the oracle's within a few ulp
    assert np.abs(host(dy) - y2).max() <= 4e-15 * max(np.abs(y2).max(), 1.0)
    assert rel(host(dphiT), phiT2) <= 1e-12
    check_logov(host(dl), ell2)
    assert np.array_equal(host(dw) == 0.0, w2 == 0.0)
    assert np.abs(host(dw) - w2).max() <= TOL * max(np.abs(w2).max(), 1e-300)


def test_half_plane_handoff_both_outcomes():
    """Half-plane hand-off over many walkers whose reference phases span the
    circle: the kept set and the weights equal the oracle's exactly, and both
    outcomes occur."""
    _say("half-plane hand-off")
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5)
    P, nw = 4, 96
    ctx = make_ctx(s, P, nw, proposal=A.PROPOSAL_RW, rw_step=0.3,
                   weight_mode=A.WEIGHT_HALFPLANE)
    rng, phi, y = state(s, P, nw, 14)
    phiT = O.trial_det(s, y)
    ell = O.log_overlap(phiT, phi)
    ref = np.exp(1j * rng.uniform(-math.pi, math.pi, size=nw))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    _, _, _, w2, _ = O.metropolis(s, phi, y, phiT, ell, ref, w0, 99, 3, 1,
                                  proposal=O.PROPOSAL_RW, rw_step=0.3,
                                  weight_mode=O.WEIGHT_HALFPLANE)
    dw = dev(w0)
    A.afqmc_metropolis_x(ctx, nw, dev(phi), dev(y), dev(phiT), dev(ell), dev(ref), dw, 99, 3, 1)
    torch.cuda.synchronize()
    assert 20 < (w2 > 0).sum() < nw - 20
    assert np.array_equal(host(dw), w2)


@pytest.mark.parametrize("case", list(CASES))
def test_reorthogonalize(case):
    _say("case", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, P, nw)
    rng, phi, y = state(s, P, nw, 5, spread=2.0)
    phi = phi * 3.0
    ell = O.log_overlap(O.trial_det(s, y), phi)
    q, lq = O.reorthogonalize(phi, ell)
    dphi, dl = dev(phi), dev(ell)
    A.afqmc_reorthogonalize(ctx, nw, dphi, dl)
    torch.cuda.synchronize()
    for w in range(nw):
        assert rel(host(dphi)[w], q[w]) <= TOL
    assert np.abs(host(dl).real - lq.real).max() <= TOL * np.abs(lq.real).max()


def test_philox_streams_and_prior():
    _say("philox")
    s = ai.tiny_ising()
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, 8, 40)
    out = torch.zeros(37, 61, dtype=torch.float64, device="cuda")
    A.afqmc_philox_normal(ctx, 99, 5, A.TAG_FIELD, 37, 61, out)
    dy = torch.zeros(40, 8, s.K, dtype=torch.float64, device="cuda")
    A.afqmc_sample_prior(ctx, 40, 77, dy)
    torch.cuda.synchronize()
    ref = PH.field_normals(99, 5, 37, 61)
    assert np.abs(host(out) - ref).max() <= 4e-15 * np.abs(ref).max()
    assert np.array_equal(host(dy), PH.init_hidden(77, 40, 8, s.K, 0))
    g = ai.small_gaussian()
    ctx2 = make_ctx(g, 3, 10)
    dy2 = torch.zeros(10, 3, g.K, dtype=torch.float64, device="cuda")
    A.afqmc_sample_prior(ctx2, 10, 78, dy2)
    torch.cuda.synchronize()
    r2 = PH.init_hidden(78, 10, 3, g.K, 1)
    assert np.abs(host(dy2) - r2).max() <= 4e-15 * np.abs(r2).max()


def test_estimator_sums():
    _say("estimator")
    s = ai.tiny_ising()
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, 2, 4)
    rng = np.random.default_rng(0)
    nw = 1000
    w = rng.uniform(0, 2, size=nw)
    e = rng.normal(size=nw) + 1j * rng.normal(size=nw)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    A.afqmc_estimator(ctx, nw, dev(w), dev(e), out)
    torch.cuda.synchronize()
    num, den = O.estimator(w, e)
    assert abs(host(out)[0] - num) <= 1e-14 * abs(num) + 1e-14
    assert abs(host(out)[1] - den) <= 1e-14 * den
    # walkers with a non-finite local energy drop out of both sums
    e[[3, 500]] = [np.nan, np.inf + 0j]
    A.afqmc_estimator(ctx, nw, dev(w), dev(e), out)
    torch.cuda.synchronize()
    num, den = O.estimator(w, e)
    assert np.isfinite(host(out)).all()
    assert abs(host(out)[0] - num) <= 1e-14 * abs(num) + 1e-14
    assert abs(host(out)[1] - den) <= 1e-14 * den


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("case", ["tiny-ising-M8", "gauss-M72-N20-ragged"])
def test_singular_paths_are_excluded(case, prec):
    """Paths of zero overlap (l = -inf) carry no force bias or energy, in every
    contraction form; with P = 3 a workgroup of the two-path kernels holds one
    such path beside a live one, and 9 paths leave the last workgroup half empty."""
    _say("singular", case, "precision", prec)
    s = CASES[case][0]()
    P, nw = 3, 3
    from paper_2505_18519_amd import afqmc as A
    ctx = make_ctx(s, P, nw, precision=prec)
    rng, phi, y = state(s, P, nw, 6)
    phi[1, 0, :, 0] = 0.0
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, 0.01)
    dl = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    dth = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, device="cuda")
    A.afqmc_green(ctx, nw, dev(phi), dev(phiT), dl, dth)
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dev(phiT), dth, dl, d_el, None, d_xb)
    torch.cuda.synchronize()
    g = host(dl)
    assert np.all(np.isneginf(g[1].real))
    assert host(d_el)[1] == 0 and np.all(host(d_xb)[1] == 0)
    bound = TOL if prec == 0 else MIXED_TOL if prec in (1, 3) else BF16_TOL
    for w in (0, 2):
        assert abs(host(d_el)[w] - eloc[w]) <= bound * max(abs(eloc[w]), 1)
        assert rel(host(d_xb)[w], xbar[w]) <= bound


TRAJ = {
    # name: (system factory, P, walkers, tau, proposal, rw step)
    "tiny-ising": (lambda: ai.workload(0)[0], 8, 16, 0.01, 0, 0.0),
    "gauss-M20-rw": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 4, 12, 0.01,
                     1, 0.3),
    "gauss-M72-prior": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 3, 6,
                        0.005, 0, 0.0),
}


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("name", list(TRAJ))
def test_trajectory_matches_oracle(name, mode):
    """30 whole steps (QR every 10) in every weight formalism, identical
    streams: per-step estimator sums, then paths and weights, against the
    oracle's steps.  The local-energy formalism (mode 3) runs with the
    shift E_T at the first step's energy, as production runs do."""
    _say("trajectory", name, "mode", mode)
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    fac, P, nw, dtau, prop, rw = TRAJ[name]
    s = fac()
    seed = 2001
    ctx = A.Context(s, P, dtau, max_walkers=nw, weight_mode=mode, proposal=prop, rw_step=rw)
    st = D.init_walkers(ctx, s.phi0, nw, seed)
    ost = O.init_state(s, nw, P, seed)
    est = torch.zeros(30, 2, dtype=torch.float64, device="cuda")
    e_shift = 0.0
    for i in range(30):
        D.step(ctx, st, seed, i, est[i], e_shift=e_shift, n_sweep=1, n_qr=10)
        ost, rec = O.step(s, ost, seed, i, dtau, n_taylor=10, n_sweep=1, n_qr=10,
                          e_shift=e_shift, proposal=prop, rw_step=rw, weight_mode=mode)
        torch.cuda.synchronize()
        g = host(est[i])
        e_ref = rec["e_num"] / rec["e_den"]
        assert abs(g[0] / g[1] - e_ref) <= TOL * max(abs(e_ref), 1.0), (i, g, e_ref)
        assert abs(g[1] - rec["e_den"]) <= TOL * rec["e_den"], i
        if i == 0 and mode == 3:
            e_shift = e_ref
    assert np.abs(host(st.y) - ost.y).max() <= 1e-12 * max(np.abs(ost.y).max(), 1.0)
    gw = host(st.w)
    assert np.array_equal(gw == 0.0, ost.w == 0.0)
    assert np.abs(gw - ost.w).max() <= TOL * np.abs(ost.w).max()


# plain BF16 products (8 significant bits) are reported, not held to the mixed bar
BF16_TOL = 5e-2

FULL = {
    # name: (workload index, contraction precision, tolerance)
    "M64-N16-G256-512x8-fp64": (1, 0, TOL),
    "M128-N32-G512-1024x4-fp64": (2, 0, TOL),
    "M128-N32-G512-1024x4-fp32": (2, 1, 1e-4),
    "M96-N24-G384-2048x4-fp64": (4, 0, TOL),
    "M96-N24-G384-2048x4-fp32": (4, 1, 1e-4),
    "M128-N32-G512-1024x4-bf16x3": (2, 3, 1e-4),
    "M96-N24-G384-2048x4-bf16x3": (4, 3, 1e-4),
    "M128-N32-G512-1024x4-bf16": (2, 2, BF16_TOL),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled_walkers(name):
    """Trial build, Green's function, contraction and propagation on every path
    of a workload at its full size, with the launch shapes the benchmark times;
    a sample of walkers is checked against the oracle."""
    _say("full size", name)
    from paper_2505_18519_amd import afqmc as A
    widx, prec, tol = FULL[name]
    s, run = ai.workload(widx)
    nw, P = run.W, run.P
    ctx = A.Context(s, P, run.dtau, max_walkers=nw, precision=prec)
    rng, phi, y = state(s, P, nw, 8)
    dy = dev(y)
    dphiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, device="cuda")
    A.afqmc_trial_build(ctx, nw, dy, dphiT)
    dl = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    dth = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, device="cuda")
    dphi = dev(phi)
    A.afqmc_green(ctx, nw, dphi, dphiT, dl, dth)
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dphiT, dth, dl, d_el, None, d_xb)
    # propagation with the GPU's own x-bar (compared below with the oracle's
    # propagation from the same x-bar)
    xi = rng.normal(size=(nw, s.n_chol))
    w = rng.uniform(0.5, 1.5, size=nw)
    dw, dref = dev(w), torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), d_xb, dphiT, dl, 0.3, dw, dref, dln)
    torch.cuda.synchronize()
    pick = np.array([0, 1, nw // 3, nw - 1])
    phiT_o = O.trial_det(s, y[pick])
    e_tr = rel(host(dphiT)[pick], phiT_o)
    # mixed-precision contexts build the trial with FP32 (BF16 contexts: split-
    # BF16) products and propagate with FP32 products: the later checks start
    # from the GPU's own trial determinants, against
    # which the FP64 LU, log-det and Theta still hold to the FP64 bound
    phiT_g = host(dphiT)[pick]
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi[pick], phiT_g, run.dtau)
    check_logov(host(dl)[pick], ell)
    g_el = host(d_el)[pick]
    e_el = np.abs(g_el - eloc).max() / np.abs(eloc).max()
    e_xb = max(rel(host(d_xb)[w_], xbar[k]) for k, w_ in enumerate(pick))
    xb_gpu = host(d_xb)[pick]
    phin, wn, ref, elln = O.propagate(s, phi[pick], xi[pick], xb_gpu, phiT_g, ell, w[pick],
                                      run.dtau, run.n_taylor, 0.3)
    e_phi = max(rel(host(dphi)[w_], phin[k]) for k, w_ in enumerate(pick))
    gw = host(dw)[pick]
    assert np.array_equal(gw == 0.0, wn == 0.0)        # the phaseless cosine's zeros
    e_w = np.abs(gw - wn).max() / max(np.abs(wn).max(), 1e-300)
    _say(f"  Phi_T {e_tr:.2e}  E_L {e_el:.2e}  xbar {e_xb:.2e}  phi' {e_phi:.2e}  W {e_w:.2e}")
    assert e_el <= tol and e_xb <= tol
    if prec == 0:
        assert e_tr <= TOL and e_phi <= TOL and e_w <= TOL
    else:
        trial_tol = BF16_TRIAL_TOL if prec == 2 else MIXED_TRIAL_TOL
        prop_tol = BF16_PROP_TOL if prec == 2 else MIXED_PROP_TOL
        assert e_tr <= trial_tol and e_phi <= prop_tol and e_w <= MIXED_TOL


def test_population_control_matches_oracle_comb():
    _say("population control")
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5)
    P, nw = 3, 37
    ctx = make_ctx(s, P, nw)
    rng, phi, y = state(s, P, nw, 9)
    phiT = O.trial_det(s, y)
    ell = O.log_overlap(phiT, phi)
    w = rng.exponential(size=nw)
    w[[3, 10]] = 0.0
    w[5] = 40.0
    for w_cap, norm in ((0.0, False), (4.0, False), (4.0, True)):
        parent, wn = O.comb(w, 55, 3, w_cap, norm)
        dphi, dw, dy, dphiT, dl = dev(phi), dev(w), dev(y), dev(phiT), dev(ell)
        dpar = torch.zeros(nw, dtype=torch.int32, device="cuda")
        A.afqmc_population_control(ctx, nw, dphi, dw, dy, dphiT, dl, 55, 3, w_cap, dpar,
                                   normalize=norm)
        torch.cuda.synchronize()
        assert np.array_equal(host(dpar), parent)
        assert np.abs(host(dw) - wn).max() <= 1e-14 * wn.max()
        assert np.array_equal(host(dphi), phi[parent])
        assert np.array_equal(host(dy), y[parent])
        assert np.array_equal(host(dphiT), phiT[parent])
        assert np.array_equal(host(dl), ell[parent])


def test_force_bias_cap():
    _say("xbar cap")
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5)
    P, nw, dtau, cap = 3, 6, 0.05, 0.05
    ctx = make_ctx(s, P, nw, dtau=dtau, xbar_cap=cap)
    rng, phi, y = state(s, P, nw, 10, spread=1.0)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(s, phiT, theta, ell)
    xbar, eloc = O.walker_estimates(vb, ep, ell, dtau, xbar_cap=cap)
    assert np.abs(xbar).max() <= cap * (1 + 1e-12)
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, None, d_xb)
    torch.cuda.synchronize()
    for w in range(nw):
        assert rel(host(d_xb)[w], xbar[w]) <= TOL



def test_local_energy_cap():
    """Re E_L clipped to E_T +- d in the context (afqmc_set_eloc_cap) against
    the oracle's capped walker estimates, with a window narrow enough that
    walkers fall on both sides of it; Im E_L, the force bias and the per-path
    E_p are unchanged; width 0 turns the cap off again."""
    _say("eloc cap")
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5)
    P, nw, dtau = 3, 12, 0.05
    ctx = make_ctx(s, P, nw, dtau=dtau)
    rng, phi, y = state(s, P, nw, 12, spread=1.5)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(s, phiT, theta, ell)
    _, e0 = O.walker_estimates(vb, ep, ell, dtau)
    et, d = float(np.median(e0.real)), 0.4 * float(np.std(e0.real))
    xbar, eloc = O.walker_estimates(vb, ep, ell, dtau, eloc_cap=(et, d))
    inside = np.abs(e0.real - et) <= d
    assert 0 < inside.sum() < nw
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_ep = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_set_eloc_cap(ctx, et, d)
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, d_ep, d_xb)
    torch.cuda.synchronize()
    g = host(d_el)
    assert np.abs(g - eloc).max() <= TOL * max(np.abs(eloc).max(), 1.0)
    assert np.all(g.real[~inside] == eloc.real[~inside])  # the bounds themselves
    assert np.abs(host(d_ep) - ep).max() <= TOL * max(np.abs(ep).max(), 1.0)
    for w in range(nw):
        assert rel(host(d_xb)[w], xbar[w]) <= TOL
    A.afqmc_set_eloc_cap(ctx, et, 0.0)
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, None, None)
    torch.cuda.synchronize()
    assert np.abs(host(d_el) - e0).max() <= TOL * max(np.abs(e0).max(), 1.0)
    with pytest.raises(A.AfqmcError):
        A.afqmc_set_eloc_cap(ctx, et, -1.0)
    with pytest.raises(A.AfqmcError):
        A.afqmc_set_eloc_cap(ctx, float("nan"), 1.0)


@pytest.mark.parametrize("name", ["gauss-M20-rw", "cfg-M64-rw"])
def test_stabilised_trajectory_matches_oracle(name):
    """40 whole steps of the stabilised local-energy form (force-bias modulus
    capped at 1, Re E_L capped around E_T, comb every step with weights reset
    to 1): E_T and a deliberately narrow cap window are set after steps 4 and
    19 from the run's own estimates, so that walkers are clipped; per-step
    estimator sums, then paths and weights, against the oracle's steps."""
    _say("stabilised trajectory", name)
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    if name == "gauss-M20-rw":
        s, P, nw, dtau = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 4, 12, 0.01
    else:
        s, P, nw, dtau = ai.workload(1)[0], 8, 6, 0.005
    seed, width = 2003, 0.3
    ctx = A.Context(s, P, dtau, max_walkers=nw, weight_mode=3, proposal=1, rw_step=0.3,
                    xbar_cap=1.0)
    st = D.init_walkers(ctx, s.phi0, nw, seed)
    ost = O.init_state(s, nw, P, seed)
    est = torch.zeros(40, 2, dtype=torch.float64, device="cuda")
    e_t, clipped = None, 0
    for i in range(40):
        cap = None if e_t is None else (e_t, width)
        D.step(ctx, st, seed, i, est[i], e_shift=e_t or 0.0, n_sweep=1, n_qr=10, n_pc=1)
        ost, rec = O.step(s, ost, seed, i, dtau, n_taylor=10, n_sweep=1, n_qr=10,
                          e_shift=e_t or 0.0, proposal=1, rw_step=0.3, weight_mode=3,
                          xbar_cap=1.0, n_pc=1, eloc_cap=cap)
        torch.cuda.synchronize()
        g = host(est[i])
        e_ref = rec["e_num"] / rec["e_den"]
        assert abs(g[0] / g[1] - e_ref) <= TOL * max(abs(e_ref), 1.0), (i, g, e_ref)
        assert abs(g[1] - rec["e_den"]) <= TOL * rec["e_den"], i
        if cap is not None:
            clipped += int(np.sum(np.abs(rec["eloc"].real - e_t) >= width * (1 - 1e-12)))
        if i in (4, 19):
            e_t = e_ref
            A.afqmc_set_eloc_cap(ctx, e_t, width)
    assert clipped > 0
    assert np.abs(host(st.y) - ost.y).max() <= 1e-12 * max(np.abs(ost.y).max(), 1.0)
    gw = host(st.w)
    assert np.abs(gw - ost.w).max() <= TOL * np.abs(ost.w).max()


@pytest.mark.parametrize("case", ["gauss-M72-N20-ragged", "gauss-M96-N24", "gauss-M128-N32",
                                  "gauss-M150-N20", "gauss-M70-N1", "gauss-M32-N32"])
def test_streamed_contraction_variant(case):
    """The FP64 contraction with its operands streamed from L2
    (afqmc_set_contraction_variant 1; the batch tuner's third family) against
    the oracle's per-path vb, E_p and walker estimates, at the shapes the
    register-resident kernel serves by default."""
    _say("streamed contraction", case)
    from paper_2505_18519_amd import afqmc as A
    fac, P, nw = CASES[case]
    s = fac()
    ctx = make_ctx(s, P, nw)
    A.afqmc_set_contraction_variant(ctx, 1)
    rng, phi, y = state(s, P, nw, 31)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(s, phiT, theta, ell)
    xbar, eloc = O.walker_estimates(vb, ep, ell, 0.01)
    d_vb = torch.zeros(nw, P, s.n_chol, dtype=torch.complex128, device="cuda")
    d_ep = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, s.n_chol, dtype=torch.complex128, device="cuda")
    A.afqmc_force_bias(ctx, nw, dev(phiT), dev(theta), dev(ell), d_xb, d_vb)
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, d_ep, None)
    torch.cuda.synchronize()
    assert rel(host(d_vb), vb) <= TOL
    assert np.abs(host(d_ep) - ep).max() <= TOL * max(np.abs(ep).max(), 1.0)
    assert np.abs(host(d_el) - eloc).max() <= TOL * max(np.abs(eloc).max(), 1.0)
    for w in range(nw):
        assert rel(host(d_xb)[w], xbar[w]) <= TOL
    with pytest.raises(A.AfqmcError):
        A.afqmc_set_contraction_variant(ctx, 2)


MIXED_TOL = 1e-4
MIXED = {"fp32": (1, MIXED_TOL), "bf16x3": (3, MIXED_TOL), "bf16": (2, BF16_TOL)}
# FP32-product trial series and walker propagation (mixed-precision contexts):
# normwise against the FP64 oracle
MIXED_TRIAL_TOL = 1e-5
MIXED_PROP_TOL = 1e-5


@pytest.mark.parametrize("case", ["tiny-ising-M8", "gauss-M3-N1", "gauss-M20-N5-ragged",
                                  "gauss-M32-N32", "cfg-M64-N16-G256", "gauss-M70-N1",
                                  "gauss-M72-N20-ragged", "gauss-M96-N24", "gauss-M128-N32"])
def test_mixed_precision_trial_and_propagation(case):
    """Mixed-precision contexts (here FP32 products) build Phi_T(y) and
    propagate the walkers with FP32 matrix-core products: Phi_T and phi'
    within 1e-5 normwise of the FP64 oracle; the move's log-overlaps (FP64 LU
    of the GPU's phi') to the FP64 bound against the oracle's LU of the same
    matrices; the weights within 1e-4."""
    _say("mixed trial/propagation", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw, precision=A.PREC_FP32)
    rng, phi, y = state(s, P, nw, 3)
    dphiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, device="cuda")
    A.afqmc_trial_build(ctx, nw, dev(y), dphiT)
    torch.cuda.synchronize()
    phiT_o = O.trial_det(s, y)
    e_tr = max(rel(host(dphiT)[w], phiT_o[w]) for w in range(nw))
    phiT = host(dphiT)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, w0, dtau, 10, -1.3)
    dphi, dw = dev(phi), dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), dev(xbar), dphiT, dev(ell), -1.3, dw, dref, dln)
    torch.cuda.synchronize()
    e_phi = max(rel(host(dphi)[w], phin[w]) for w in range(nw))
    check_logov(host(dln), O.log_overlap(phiT, host(dphi)))
    e_w = np.abs(host(dw) - wn).max() / np.abs(wn).max()
    _say(f"  errors vs FP64 oracle: Phi_T {e_tr:.2e}  phi' {e_phi:.2e}  W {e_w:.2e}")
    assert e_tr <= MIXED_TRIAL_TOL and e_phi <= MIXED_PROP_TOL and e_w <= MIXED_TOL
    assert max(e_tr, e_phi) > 1e-12     # the FP32 products are really in use


# BF16 contexts past M = 64 or N = 16 build the trial on split-BF16 products
# (FP32 accumulation, the running sum in FP64)
BF16_TRIAL_TOL = 2e-5


@pytest.mark.parametrize("prec", ["bf16"])
@pytest.mark.parametrize("case", ["gauss-M32-N32", "gauss-M70-N1", "gauss-M72-N20-ragged",
                                  "gauss-M80-N27-ragged", "gauss-M96-N24", "gauss-M128-N32"])
def test_bf16_contexts_build_the_trial_on_split_bf16_products(case, prec):
    """Phi_T(y) of a BF16 context within 2e-5 normwise of the
    FP64 oracle, and further from it than FP32 products would be (so the
    split-BF16 series is the one that ran)."""
    _say("bf16 trial", case, prec)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    ctx = A.Context(s, P, 0.01, max_walkers=nw, precision=MIXED[prec][0])
    rng, phi, y = state(s, P, nw, 3)
    dphiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, device="cuda")
    A.afqmc_trial_build(ctx, nw, dev(y), dphiT)
    torch.cuda.synchronize()
    phiT_o = O.trial_det(s, y)
    e_tr = max(rel(host(dphiT)[w], phiT_o[w]) for w in range(nw))
    _say(f"  Phi_T vs FP64 oracle: {e_tr:.2e}")
    assert 5e-7 < e_tr <= BF16_TRIAL_TOL  # FP32 products stay below 3e-7 on these shapes


# ... and propagate the walkers on split-BF16 products
BF16_PROP_TOL = 5e-5


@pytest.mark.parametrize("case", ["gauss-M32-N32", "gauss-M70-N1", "gauss-M72-N20-ragged",
                                  "gauss-M80-N27-ragged", "gauss-M96-N24", "gauss-M128-N32"])
def test_bf16_contexts_propagate_on_split_bf16_products(case):
    """The move of a BF16 context (V build, T_n(V) and the one-body factors on
    split-BF16 products, V stored split between them) from the oracle's trial and
    x-bar: phi' within 5e-5 normwise of the FP64 oracle and further from it
    than FP32 products would be; the log-overlaps of the GPU's phi' to the
    FP64 bound against the oracle's LU of the same matrices; the weights
    within 1e-4."""
    _say("bf16 propagation", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw, precision=A.PREC_BF16)
    rng, phi, y = state(s, P, nw, 3)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, w0, dtau, 10, -1.3)
    dphi, dw = dev(phi), dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), dev(xbar), dev(phiT), dev(ell), -1.3, dw, dref,
                      dln)
    torch.cuda.synchronize()
    e_phi = max(rel(host(dphi)[w], phin[w]) for w in range(nw))
    check_logov(host(dln), O.log_overlap(phiT, host(dphi)))
    e_w = np.abs(host(dw) - wn).max() / np.abs(wn).max()
    _say(f"  errors vs FP64 oracle: phi' {e_phi:.2e}  W {e_w:.2e}")
    assert 4e-7 < e_phi <= BF16_PROP_TOL and e_w <= MIXED_TOL


@pytest.mark.parametrize("prec", list(MIXED))
@pytest.mark.parametrize("case", ["tiny-ising-M8", "gauss-M3-N1", "gauss-M20-N5-ragged",
                                  "gauss-M32-N32", "gauss-M48-N11", "cfg-M64-N16-G256",
                                  "gauss-M70-N1", "gauss-M72-N20-ragged", "gauss-M96-N24",
                                  "gauss-M128-N32", "gauss-M80-N27-ragged"])
def test_mixed_precision_contraction(case, prec):
    """FP32, split-BF16 and BF16 matrix-core contractions (FP64 traces and
    sums) against the FP64 oracle: per-path vb and E_p, per-walker force bias
    and E_L within 1e-4 (FP32, split BF16) or the plain-BF16 bound."""
    _say("mixed", case, prec)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    code, bound = MIXED[prec]
    ctx = A.Context(s, P, dtau, max_walkers=nw, precision=code)
    rng, phi, y = state(s, P, nw, 2)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, dtau)
    _, theta = O.green(phiT, phi)
    G = s.n_chol
    d_el = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    d_ep = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    d_xb = torch.zeros(nw, G, dtype=torch.complex128, device="cuda")
    d_vb = torch.zeros(nw, P, G, dtype=torch.complex128, device="cuda")
    A.afqmc_local_energy(ctx, nw, dev(phiT), dev(theta), dev(ell), d_el, d_ep, d_xb)
    A.afqmc_force_bias(ctx, nw, dev(phiT), dev(theta), dev(ell), d_xb, d_vb)
    torch.cuda.synchronize()
    e_ep = np.abs(host(d_ep) - ep).max() / max(np.abs(ep).max(), 1)
    e_el = np.abs(host(d_el) - eloc).max() / max(np.abs(eloc).max(), 1)
    e_xb = max(rel(host(d_xb)[w], xbar[w]) for w in range(nw))
    e_vb = max(rel(host(d_vb)[w, p], vb[w, p]) for w in range(nw) for p in range(P))
    _say(f"  errors vs FP64 oracle: E_p {e_ep:.2e} E_L {e_el:.2e} xbar {e_xb:.2e} vb {e_vb:.2e}")
    for e in (e_ep, e_el, e_xb, e_vb):
        assert e <= bound
    # the reduced-precision products are really in use (FP64 would agree to ~1e-14)
    assert max(e_ep, e_xb) > 1e-10


def test_large_systems_take_the_fp64_contraction_and_plain_proposals():
    """Past M = 128 or N = 32 only the FP64 contraction and the prior and
    random-walk proposals are built; the rest is refused, not run."""
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=136, N=34, n_chol=4, K=8, seed=16)
    A.Context(s, 2, 0.01, proposal=A.PROPOSAL_RW).close()
    for kw in (dict(precision=A.PREC_FP32), dict(precision=A.PREC_BF16X3),
               dict(proposal=A.PROPOSAL_LEARNED)):
        with pytest.raises(A.AfqmcError) as ei:
            A.Context(s, 2, 0.01, **kw)
        assert ei.value.status == 6, kw


def test_bf16_contraction_needs_real_trials():
    from paper_2505_18519_amd import afqmc as A
    s = ai.imaginary_time_trial(ai.tiny_ising(), 1, 0.05)
    for prec in (A.PREC_BF16, A.PREC_BF16X3):
        with pytest.raises(A.AfqmcError):
            A.Context(s, 4, 0.01, precision=prec)
    with pytest.raises(A.AfqmcError):
        A.Context(ai.tiny_ising(), 4, 0.01, precision=4)


@pytest.mark.parametrize("case", ["gauss-M20-N5-ragged", "cfg-M64-N16-G256", "gauss-M72-N20-ragged",
                                  "gauss-M128-N32"])
def test_complex64_walkers(case):
    """Walkers stored as complex64 (mixed-precision contexts): the calls widen
    them exactly, so overlaps and Theta equal the oracle's for the stored
    walkers to the FP64 bound; a move returns walkers within 1e-5 of the FP64
    oracle (FP32 products plus rounding to complex64) whose stored log-overlaps
    are the FP64 LU of the rounded walkers; QR returns the rounded FP64 QR;
    the comb copies rows bit for bit."""
    _say("complex64 walkers", case)
    s, P, nw = CASES[case][0](), CASES[case][1], CASES[case][2]
    from paper_2505_18519_amd import afqmc as A
    dtau = 0.01
    ctx = A.Context(s, P, dtau, max_walkers=nw, precision=A.PREC_FP32, walker_c64=True)
    rng, phi, y = state(s, P, nw, 11, spread=1.0)
    phi64 = phi.astype(np.complex64)
    phi_w = phi64.astype(np.complex128)                 # what the library works on
    phiT = O.trial_det(s, y)
    ell_ref, theta_ref = O.green(phiT, phi_w)
    dl = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    dth = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, device="cuda")
    dphi = dev(phi64)
    assert dphi.dtype == torch.complex64
    A.afqmc_green(ctx, nw, dphi, dev(phiT), dl, dth)
    torch.cuda.synchronize()
    check_logov(host(dl), ell_ref)
    for w in range(nw):
        for p in range(P):
            assert rel(host(dth)[w, p], theta_ref[w, p]) <= TOL
    # a move
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi_w, phiT, dtau)
    xi = rng.normal(size=(nw, s.n_chol))
    w0 = rng.uniform(0.5, 1.5, size=nw)
    phin, wn, ref, elln = O.propagate(s, phi_w, xi, xbar, phiT, ell, w0, dtau, 10, -1.3)
    dw = dev(w0)
    dref = torch.zeros(nw, dtype=torch.complex128, device="cuda")
    dln = torch.zeros(nw, P, dtype=torch.complex128, device="cuda")
    A.afqmc_propagate(ctx, nw, dphi, dev(xi), dev(xbar), dev(phiT), dev(ell), -1.3, dw, dref, dln)
    torch.cuda.synchronize()
    g_phi = host(dphi).astype(np.complex128)
    e_phi = max(rel(g_phi[w], phin[w]) for w in range(nw))
    check_logov(host(dln), O.log_overlap(phiT, g_phi))
    e_w = np.abs(host(dw) - wn).max() / np.abs(wn).max()
    _say(f"  errors vs FP64 oracle: phi' {e_phi:.2e}  W {e_w:.2e}")
    assert e_phi <= MIXED_PROP_TOL and e_w <= MIXED_TOL
    # re-orthonormalisation of the stored walkers
    q_ref, lq_ref = O.reorthogonalize(g_phi, ell)
    dl2 = dev(ell)
    A.afqmc_reorthogonalize(ctx, nw, dphi, dl2)
    torch.cuda.synchronize()
    g_q = host(dphi)
    assert g_q.dtype == np.complex64
    for w in range(nw):
        assert rel(g_q[w].astype(np.complex128), q_ref[w]) <= 2e-7
    assert np.abs(host(dl2).real - lq_ref.real).max() <= TOL * np.abs(lq_ref.real).max()
    # the comb moves complex64 rows
    wts = rng.exponential(size=nw)
    parent, _ = O.comb(wts, 3, 1)
    before = host(dphi).copy()
    A.afqmc_population_control(ctx, nw, dphi, dev(wts), dev(y), dev(phiT), dev(ell), 3, 1, 0.0)
    torch.cuda.synchronize()
    assert np.array_equal(host(dphi), before[parent])


def test_complex64_walkers_need_a_mixed_context():
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5)
    with pytest.raises(A.AfqmcError) as ei:
        A.Context(s, 2, 0.01, walker_c64=True)          # FP64 contraction
    assert ei.value.status == 6
    ctx = A.Context(s, 2, 0.01, max_walkers=2, precision=A.PREC_BF16X3, walker_c64=True)
    z = dict(device="cuda")
    with pytest.raises(A.AfqmcError) as ei:
        A.afqmc_init_metropolis(ctx, 2, 1, 1, 1, torch.zeros(2, s.K, dtype=torch.float64, **z),
                                torch.zeros(2, 2, s.M, s.N, dtype=torch.complex64, **z),
                                torch.zeros(2, 2, s.K, dtype=torch.float64, **z),
                                torch.zeros(2, 2, s.M, s.N, dtype=torch.float64, **z),
                                torch.zeros(2, 2, dtype=torch.complex128, **z),
                                torch.zeros(2, dtype=torch.float64, **z))
    assert ei.value.status == 6
