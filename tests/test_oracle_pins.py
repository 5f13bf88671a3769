"""Pins of the CPU oracle against exact references (no GPU).

Every check compares the oracle with something other than itself: Fock-space
brute force and exact diagonalisation on tiny systems, Gauss-Hermite
quadrature of the Hubbard-Stratonovich identity, closed forms of an exactly
solvable Hamiltonian, numpy's own Philox, and limits in which the method
reduces to plain single-determinant phaseless AFQMC.
"""
import copy
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

import afqmc_inputs as ai
from oracle import afqmc_oracle as O
from oracle import fock as F
from oracle import philox as PH

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tiny():
    return ai.tiny_ising()


@pytest.fixture(scope="module")
def tiny_H(tiny):
    return F.hamiltonian(tiny)


# -- RNG -------------------------------------------------------------------

def test_philox_matches_numpy_bit_exact():
    """Counter c of our Philox4x64-10 equals numpy's Philox started at c - 1
    (numpy increments the counter before producing a block)."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        key = int(rng.integers(0, 2**63))
        ctr = [int(v) for v in rng.integers(1, 2**62, size=4)]
        bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64),
                              counter=np.array([ctr[0] - 1] + ctr[1:], dtype=np.uint64))
        ref = [int(v) for v in bg.random_raw(4)]
        assert list(PH.philox4x64_scalar(ctr, [key, 0])) == ref
        vec = PH.philox4x64(np.array(ctr, dtype=np.uint64), key)
        assert [int(v) for v in vec] == ref


def test_philox_streams_layout():
    """Uniforms in [0,1), normals with unit variance, streams independent of nw."""
    u = PH.accept_uniforms(7, 3, 16, 4, 9, 0)
    assert u.min() >= 0.0 and u.max() < 1.0
    z = PH.field_normals(11, 5, 256, 257)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    z_sub = PH.field_normals(11, 5, 3, 257)
    assert np.array_equal(z[:3], z_sub)
    # normal i of a stream is element i % 4 of block i // 4 (counter word 0)
    words = PH.philox4x64(np.array([2, 1, 5, PH.word3(PH.TAG_FIELD)], dtype=np.uint64), 11)
    ua = (int(words[0]) >> 11) * 2.0**-53
    ub = (int(words[1]) >> 11) * 2.0**-53
    assert z[1, 8] == pytest.approx(math.sqrt(-2 * math.log(1 - ua)) * math.cos(2 * math.pi * ub),
                                    rel=1e-14)


# -- Thouless and the propagator -------------------------------------------

def test_thouless_trial_determinant(tiny):
    """exp(U-hat)|Phi_0> equals the determinant of exp(U) Phi_0 (Eq. spo) for
    the trial generator U = c sum_k y_k A_k, Ising and Gaussian."""
    gs = ai.small_gaussian(M=7, N=3, n_chol=4, K=5, seed=9)
    for s in (tiny, gs):
        y = ai.random_hidden(np.random.default_rng(4), s, 2, 3)
        phiT = O.trial_det(s, y)
        v0 = F.det_vector_sector(s.phi0)
        for w in range(2):
            for p in range(3):
                U = s.coupling * np.einsum("k,kij->ij", y[w, p], s.A)
                ref = expm(F.one_body_sector(U, s.N)) @ v0
                got = F.det_vector_sector(phiT[w, p])
                assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_thouless_walker_propagator(tiny):
    """e^{-tau h1/2} T_n(V) e^{-tau h1/2} Phi with a long series equals the
    Fock-space exp of the same one-body operators acting on |Phi>."""
    rng = np.random.default_rng(5)
    phi = ai.random_walkers(rng, tiny, 1, spread=0.7)
    xi = rng.normal(size=(1, tiny.n_chol))
    xbar = 0.1 * (rng.normal(size=(1, tiny.n_chol)) + 1j * rng.normal(size=(1, tiny.n_chol)))
    tau = 0.01
    got = O.propagate_dets(tiny, phi, xi, xbar, tau, 40)
    V = O.field_matrix(tiny, xi, xbar, tau)[0]
    H1 = F.one_body_full(tiny.h1, tiny.N)
    Vf = F.one_body_full(V, tiny.N)
    ref = expm(-tau / 2 * H1) @ expm(Vf) @ expm(-tau / 2 * H1) @ F.det_vector(phi[0, 0], phi[0, 1])
    g = F.det_vector(got[0, 0], got[0, 1])
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_taylor_order_ten_truncation(tiny):
    """The fixed 10-term series is within its truncation bound of exp(V)."""
    sysg, _ = ai.workload(1)
    rng = np.random.default_rng(6)
    xi = rng.normal(size=(2, sysg.n_chol))
    V = O.field_matrix(sysg, xi, np.zeros((2, sysg.n_chol)), 0.005)
    X = rng.normal(size=(2, sysg.M, 3)) + 0j
    got = O.taylor_apply(V, X, 10)
    for w in range(2):
        ref = expm(V[w]) @ X[w]
        nv = np.linalg.norm(V[w], 2)
        bound = nv ** 11 / math.factorial(11) * math.exp(nv) * np.linalg.norm(X[w], 2)
        assert np.linalg.norm(got[w] - ref, 2) <= bound + 1e-12


def test_hs_quadrature_pins_the_coupling_convention(tiny):
    """Gauss-Hermite sum over one field of the oracle's propagator equals
    e^{-tau H1/2} e^{-tau L^2/2} e^{-tau H1/2} (Eqs. HS-V, HS); the factor i
    in V = i sqrt(tau) x L is what makes this hold for real L."""
    s1 = copy.deepcopy(tiny)
    s1.n_chol = 1
    s1.L = tiny.L[2:3].copy()
    phi = ai.random_walkers(np.random.default_rng(1), tiny, 1, spread=0.8)
    x, wq = np.polynomial.hermite_e.hermegauss(40)
    wq = wq / math.sqrt(2 * math.pi)
    tau = 0.01
    acc = 0
    for xq, ww in zip(x, wq):
        ph = O.propagate_dets(s1, phi, np.array([[xq]]), np.zeros((1, 1), complex), tau, 80)
        acc = acc + ww * F.det_vector(ph[0, 0], ph[0, 1])
    Lf = F.one_body_full(s1.L[0], tiny.N)
    H1 = F.one_body_full(tiny.h1, tiny.N)
    ref = (expm(-tau / 2 * H1) @ expm(-tau / 2 * Lf @ Lf) @ expm(-tau / 2 * H1)
           @ F.det_vector(phi[0, 0], phi[0, 1]))
    assert np.abs(acc - ref).max() <= 1e-12 * np.abs(ref).max()


# -- One determinant pair against Fock space --------------------------------

@pytest.mark.parametrize("which", ["ising", "gauss"])
def test_det_pair_overlap_forcebias_energy(which, tiny, tiny_H):
    """exp(l) = <Phi_T|Phi_w>, vb_g = <L_g>, E_p = <H> for a determinant pair
    (Cauchy-Binet, Wick with h1' = h1 + 1/2 sum L^2, spin factorisation)."""
    if which == "ising":
        s, H = tiny, tiny_H
    else:
        s = ai.small_gaussian(M=6, N=2, n_chol=5, K=3, seed=12)
        H = F.hamiltonian(s)
    rng = np.random.default_rng(3)
    phi = ai.random_walkers(rng, s, 2, spread=0.8)
    y = ai.random_hidden(rng, s, 2, 3)
    phiT = O.trial_det(s, y)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, phiT, 0.01)
    Lf = [F.one_body_full(s.L[g], s.N) for g in range(s.n_chol)]
    for w in range(2):
        vw = F.det_vector(phi[w, 0], phi[w, 1])
        for p in range(3):
            vt = F.det_vector(phiT[w, p], phiT[w, p])
            ov = vt.conj() @ vw
            assert abs(np.exp(ell[w, p]) - ov) <= 1e-12 * abs(ov)
            assert abs((vt.conj() @ H @ vw) / ov - ep[w, p]) <= 1e-12 * max(1, abs(ep[w, p]))
            for g in range(s.n_chol):
                ref = (vt.conj() @ Lf[g] @ vw) / ov
                assert abs(ref - vb[w, p, g]) <= 1e-12 * max(1, abs(ref))


def test_ising_trial_bruteforce_local_energy(tiny, tiny_H):
    """With all 2^K Ising states the trial is exact: <Psi_T| = 2^-K sum_y <Phi_T(y)|.
    E_L and the force bias of Eq. local-obs, with every state weighted by its
    |O_y| (the density the paths sample), equal the exact Fock-space values."""
    K = tiny.K
    ys = np.array([[1.0 if (b >> k) & 1 else -1.0 for k in range(K)] for b in range(2**K)])
    rng = np.random.default_rng(8)
    phi = ai.random_walkers(rng, tiny, 1, spread=0.6)
    phiT = O.trial_det(tiny, ys[None])
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(tiny, phiT, theta, ell)
    vw = F.det_vector(phi[0, 0], phi[0, 1])
    psi = sum(F.det_vector(phiT[0, p], phiT[0, p]) for p in range(2**K)) / 2**K
    ov = psi @ vw
    e_exact = (psi @ tiny_H @ vw) / ov
    L0 = F.one_body_full(tiny.L[0], tiny.N)
    l0_exact = (psi @ L0 @ vw) / ov
    O_y = np.exp(ell[0])
    # S-weighted average over samples with multiplicity |O_y| (Eq. local-obs)
    S = O.phases(ell)[0]
    m = np.abs(O_y)
    e_est = (m * S * ep[0]).sum() / (m * S).sum()
    l0_est = (m * S * vb[0, :, 0]).sum() / (m * S).sum()
    assert abs(e_est - e_exact) <= 1e-12 * abs(e_exact)
    assert abs(l0_est - l0_exact) <= 1e-12 * max(1, abs(l0_exact))


def test_metropolis_samples_the_path_density(tiny):
    """The Ising single-flip chain at fixed phi visits y with frequency
    |O(y; phi)| / sum |O| (Eq. PDF-Y with uniform p_T)."""
    K = tiny.K
    rng = np.random.default_rng(21)
    phi = ai.random_walkers(rng, tiny, 1, spread=1.5)
    P = 64
    y = ai.random_hidden(rng, tiny, 1, P)
    phiT = O.trial_det(tiny, y)
    logov = O.log_overlap(phiT, phi)
    ref = np.ones(1, complex)
    counts = np.zeros((P, 2**K))
    n_steps = 400
    for st in range(n_steps):
        y, phiT, logov, _, _ = O.metropolis(tiny, phi, y, phiT, logov, ref, np.ones(1), 99, st, 1)
        if st >= 20:
            idx = ((y[0] > 0) * (1 << np.arange(K))).sum(-1).astype(int)
            counts[np.arange(P), idx] += 1
    ys = np.array([[1.0 if (b >> k) & 1 else -1.0 for k in range(K)] for b in range(2**K)])
    pr = np.abs(np.exp(O.log_overlap(O.trial_det(tiny, ys[None]), phi)[0]))
    pr /= pr.sum()
    # the P chains are independent: their spread gives the error of the mean
    f = counts / counts.sum(1, keepdims=True)
    z = (f.mean(0) - pr) / (f.std(0, ddof=1) / np.sqrt(P))
    assert np.abs(z).max() < 5.0, z


def test_path_estimator_converges_to_exact_local_energy(tiny, tiny_H):
    """Eq. local-obs evaluated on the paths the chain produces converges to the
    exact <Psi_T|H|phi>/<Psi_T|phi> of the 2^K-state Ising trial."""
    K = tiny.K
    rng = np.random.default_rng(31)
    phi = ai.random_walkers(rng, tiny, 1, spread=1.2)
    P = 32
    y = ai.random_hidden(rng, tiny, 1, P)
    phiT = O.trial_det(tiny, y)
    logov = O.log_overlap(phiT, phi)
    ests = []
    for st in range(220):
        y, phiT, logov, _, _ = O.metropolis(tiny, phi, y, phiT, logov, np.ones(1, complex),
                                            np.ones(1), 17, st, 1)
        if st >= 20:
            ell, theta = O.green(phiT, phi)
            vb, ep = O.sample_contraction(tiny, phiT, theta, ell)
            _, eloc = O.walker_estimates(vb, ep, ell, 0.01)
            ests.append(eloc[0])
    ys = np.array([[1.0 if (b >> k) & 1 else -1.0 for k in range(K)] for b in range(2**K)])
    pt = O.trial_det(tiny, ys[None])
    psi = sum(F.det_vector(pt[0, p], pt[0, p]) for p in range(2**K))
    vw = F.det_vector(phi[0, 0], phi[0, 1])
    e_exact = (psi @ tiny_H @ vw) / (psi @ vw)
    ests = np.array(ests)
    blocks = ests.reshape(20, -1).mean(1)
    err = blocks.std(ddof=1) / math.sqrt(len(blocks))
    assert abs(ests.mean() - e_exact) < 5 * abs(err) + 1e-3 / P, (ests.mean(), e_exact, err)


def test_gaussian_random_walk_detailed_balance():
    """Random-walk chain on a K=2 Gaussian-hidden toy: the mean of y under the
    chain matches quadrature of p_T(y)|O(y; phi)| on a grid."""
    s = ai.small_gaussian(M=6, N=2, n_chol=3, K=2, seed=4)
    s.coupling = 0.8
    rng = np.random.default_rng(2)
    phi = ai.random_walkers(rng, s, 1, spread=0.8)
    P = 128
    y = rng.normal(size=(1, P, 2))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    acc = []
    for st in range(300):
        y, phiT, logov, _, _ = O.metropolis(s, phi, y, phiT, logov, np.ones(1, complex),
                                            np.ones(1), 5, st, 1, proposal=O.PROPOSAL_RW,
                                            rw_step=0.8)
        if st >= 30:
            acc.append(y[0].copy())
    samp = np.concatenate(acc)
    g = np.linspace(-7, 7, 141)
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    lo = O.log_overlap(O.trial_det(s, Y[None]), phi)[0]
    dens = np.exp(lo.real - lo.real.max() - 0.5 * (Y * Y).sum(-1))
    dens /= dens.sum()
    mean_ref = (dens[:, None] * Y).sum(0)
    sd = np.sqrt((dens[:, None] * (Y - mean_ref) ** 2).sum(0))
    # effective sample size: generous autocorrelation allowance of 20
    err = sd / math.sqrt(len(samp) / 20)
    assert np.all(np.abs(samp.mean(0) - mean_ref) < 5 * err), (samp.mean(0), mean_ref, err)


def _quadrature_moments(s, phi, a, b, half=8.0, n=161):
    """Mean and second moment per coordinate of the 2-D density
    exp(a Re l(y; phi) - b |y|^2 / 2) on a grid, with their standard deviations."""
    g = np.linspace(-half, half, n)
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    lo = O.log_overlap(O.trial_det(s, Y[None]), phi)[0].real
    dens = np.exp(a * (lo - lo.max()) - 0.5 * b * (Y * Y).sum(-1))
    dens /= dens.sum()
    m1 = (dens[:, None] * Y).sum(0)
    m2 = (dens[:, None] * Y ** 2).sum(0)
    m4 = (dens[:, None] * Y ** 4).sum(0)
    return m1, m2, np.sqrt(m2 - m1 ** 2), np.sqrt(m4 - m2 ** 2)


def test_gaussian_prior_proposal_detailed_balance():
    """The independence sampler of App. B (Propagation, step 2; Sec. III.A,
    leapfrog step 2): y' drawn from the prior N(0, 1), accepted with
    min{1, |O(y')| / |O(y)|}, must leave p_T(y) |O(y; phi)| = N(y) |O(y; phi)|
    of Eq. PDF-Y invariant.  On a K = 2 toy the chain's first and second
    moments match 2-D quadrature of that density, and they are far from the
    densities a plausible slip would sample instead: an extra prior ratio
    N(y')/N(y) in alpha (density N^2 |O|), the inverted ratio (N / |O|), or
    the squared ratio (N |O|^2)."""
    s = ai.small_gaussian(M=6, N=2, n_chol=3, K=2, seed=4)
    s.coupling = 1.5
    rng = np.random.default_rng(2)
    phi = ai.random_walkers(rng, s, 1, spread=1.5)
    P = 128
    y = rng.normal(size=(1, P, 2))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    acc, n_acc = [], 0
    for st in range(300):
        y, phiT, logov, _, nacc = O.metropolis(s, phi, y, phiT, logov, np.ones(1, complex),
                                               np.ones(1), 5, st, 1,
                                               proposal=O.PROPOSAL_PRIOR)
        n_acc += int(nacc[0])
        if st >= 30:
            acc.append(y[0].copy())
    samp = np.concatenate(acc)
    assert 0.2 < n_acc / (300 * P) < 0.99          # the test exercises rejections
    n_eff = len(samp) / 20                          # autocorrelation allowance of 20

    def zscores(a, b):
        m1, m2, sd1, sd2 = _quadrature_moments(s, phi, a, b)
        z1 = (samp.mean(0) - m1) / (sd1 / math.sqrt(n_eff))
        z2 = ((samp ** 2).mean(0) - m2) / (sd2 / math.sqrt(n_eff))
        return np.abs(np.concatenate([z1, z2]))

    assert zscores(1.0, 1.0).max() < 4.0, zscores(1.0, 1.0)
    for a, b in ((1.0, 2.0), (-1.0, 1.0), (2.0, 1.0)):
        assert zscores(a, b).max() > 5.0, (a, b, zscores(a, b))


def test_handoff_half_plane_and_cosine_closed_forms():
    """Hand-off projection (Sec. III.A, after Eq. AFQMC_Metro_constraint_cos;
    App. B step 3): with the angle dtheta_T = arg sum_p S'_p - arg ref,
    the cosine rule multiplies W by max(0, cos dtheta_T) and the half-plane
    rule keeps W exactly when the new sign sum lies within pi/2 of the
    reference.  Both are checked against the inner-product form
    cos dtheta_T = Re(a conj(b)) / (|a| |b|) (a = sum S', b = ref), which holds
    for any branch of arg, and on single-path cases whose answer is plain."""
    pi = math.pi
    # one path of phase theta against a reference of phase phi0 and modulus 2.5
    cases = [(0.49 * pi, 0.0, True), (0.51 * pi, 0.0, False), (-0.51 * pi, 0.0, False),
             (1.6 * pi, 0.0, True), (-1.6 * pi, 0.0, True), (pi, 0.0, False),
             (0.9 * pi, -0.9 * pi, True), (0.2 * pi, 0.75 * pi, False), (0.0, 0.0, True)]
    for th, ph, kept in cases:
        logov = np.array([[0.3 + 1j * th]])
        ref = np.array([2.5 * np.exp(1j * ph)])
        w = np.array([1.7])
        w_hp = O.handoff(w, logov, ref, O.WEIGHT_HALFPLANE)
        w_cos = O.handoff(w, logov, ref, O.WEIGHT_SEPARATE)
        assert w_hp[0] == (1.7 if kept else 0.0), (th, ph)
        assert abs(w_cos[0] - 1.7 * max(0.0, math.cos(th - ph))) <= 1e-15, (th, ph)
        assert (w_cos[0] > 0.0) == kept
    # many walkers, P = 5 paths with one singular path, arbitrary phases
    rng = np.random.default_rng(11)
    nw, P = 400, 5
    logov = rng.normal(size=(nw, P)) + 1j * rng.uniform(-8, 8, size=(nw, P))
    logov[:, 2] = complex(-np.inf, 0.0)
    ref = rng.normal(size=nw) + 1j * rng.normal(size=nw)
    w = rng.uniform(0.5, 2.0, size=nw)
    a = np.exp(1j * logov[:, [0, 1, 3, 4]].imag).sum(-1)
    inner = (a * np.conj(ref)).real / (np.abs(a) * np.abs(ref))
    w_hp = O.handoff(w, logov, ref, O.WEIGHT_HALFPLANE)
    w_cos = O.handoff(w, logov, ref, O.WEIGHT_SEPARATE)
    w_comb = O.handoff(w, logov, ref, O.WEIGHT_COMBINED)
    assert np.array_equal(w_hp, np.where(inner > 0, w, 0.0))
    assert np.abs(w_cos - w * np.maximum(inner, 0.0)).max() <= 1e-13
    assert np.array_equal(w_comb, w_cos)           # the same projection, another reference
    assert 100 < (w_hp > 0).sum() < 300            # both outcomes occur
    # a walker whose new paths are all singular, or whose reference is 0, dies
    logov[7] = complex(-np.inf, 0.0)
    ref[9] = 0.0
    for mode in (O.WEIGHT_HALFPLANE, O.WEIGHT_SEPARATE):
        out = O.handoff(w, logov, ref, mode)
        assert out[7] == 0.0 and out[9] == 0.0


# -- Exactly solvable: zero-variance trial ----------------------------------

def test_zero_variance_exact_trial():
    """L_g annihilates the occupied space and the trial generators keep it
    invariant, so Phi_0 is the exact ground state with E_0 = 2 sum_occ eps,
    every E_p and E_L equals E_0, xbar = 0, and a run keeps E = E_0 with
    constant weights when the shift is E_0."""
    s = ai.exact_trial_system()
    E0_ed = F.ground_energy(s)
    eps = np.linalg.eigvalsh(s.h1)
    E0 = 2 * eps[: s.N].sum()
    assert abs(E0_ed - E0) <= 1e-10
    rng = np.random.default_rng(3)
    phi = ai.random_walkers(rng, s, 4, spread=0.9)
    y = ai.random_hidden(rng, s, 4, 5)
    eloc, xbar, ep, vb, ell = O.local_energy(s, phi, O.trial_det(s, y), 0.01)
    assert np.abs(ep - E0).max() <= 1e-10 * abs(E0)
    assert np.abs(eloc - E0).max() <= 1e-10 * abs(E0)
    assert np.abs(xbar).max() <= 1e-12
    st = O.init_state(s, 8, 4, seed=3)
    for i in range(12):
        st, rec = O.step(s, st, 3, i, 0.01, e_shift=E0, n_qr=5)
        assert abs(rec["e_num"] / rec["e_den"] - E0) <= 1e-10 * abs(E0)
    assert np.abs(st.w - 1.0).max() <= 1e-10
    # with E_T = E_0 + d both formalisms grow every weight by exactly e^{tau d}
    # per step: the hybrid through the overlap ratio e^{-tau E_0}, the
    # local-energy form through E_L = E_0 (sign and scale of both pinned)
    for mode in (O.WEIGHT_SEPARATE, O.WEIGHT_LOCAL):
        st = O.init_state(s, 8, 4, seed=4)
        for i in range(6):
            st, rec = O.step(s, st, 4, i, 0.01, e_shift=E0 + 0.7, n_qr=5, weight_mode=mode)
        assert np.abs(st.w / math.exp(0.01 * 0.7 * 6) - 1.0).max() <= 1e-12, (mode, st.w)


# -- Reductions and invariances ---------------------------------------------

def _single_det_reference_weight(s, phi, w, xi, dtau):
    """Plain single-determinant ph-AFQMC weight from Fock-space overlaps."""
    v0 = F.det_vector(s.phi0, s.phi0)
    vw = F.det_vector(phi[0, 0], phi[0, 1])
    ov = v0 @ vw
    xbar = np.array([-1j * math.sqrt(dtau) * (v0 @ F.one_body_full(s.L[g], s.N) @ vw) / ov
                     for g in range(s.n_chol)])[None]
    phin = O.propagate_dets(s, phi, xi, xbar, dtau, 10)
    ovn = v0 @ F.det_vector(phin[0, 0], phin[0, 1])
    r = ovn / ov
    I = np.exp((xi * xbar - 0.5 * xbar * xbar).sum()) * r
    return xbar, w * abs(I) * max(0.0, math.cos(np.angle(r)))


def test_frozen_trial_reduces_to_single_determinant(tiny):
    """coupling = 0: every path carries Phi_0, the composite-walker step equals
    single-determinant phaseless AFQMC and the hand-off factor is exactly 1."""
    s = copy.deepcopy(tiny)
    s.coupling = 0.0
    rng = np.random.default_rng(4)
    phi = ai.random_walkers(rng, s, 1, spread=0.5)
    y = ai.random_hidden(rng, s, 1, 4)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(s, phiT, theta, ell)
    xbar, eloc = O.walker_estimates(vb, ep, ell, 0.01)
    xi = rng.normal(size=(1, s.n_chol))
    xbar_ref, w_ref = _single_det_reference_weight(s, phi, 1.0, xi, 0.01)
    assert np.abs(xbar - xbar_ref).max() <= 1e-12
    phin, wn, ref, elln = O.propagate(s, phi, xi, xbar, phiT, ell, np.ones(1), 0.01, 10)
    assert abs(wn[0] - w_ref) <= 1e-12 * w_ref
    _, _, _, w2, nacc = O.metropolis(s, phin, y, phiT, elln, ref, wn, 1, 0, 1)
    assert abs(w2[0] - wn[0]) <= 1e-14 * wn[0]


def test_handoff_is_one_for_single_path_without_moves(tiny):
    """P = 1 and no Metropolis move: R of Eq. AFQMC_Metro_correction has zero phase."""
    rng = np.random.default_rng(7)
    phi = ai.random_walkers(rng, tiny, 3, spread=0.8)
    y = ai.random_hidden(rng, tiny, 3, 1)
    phiT = O.trial_det(tiny, y)
    eloc, xbar, ep, vb, ell = O.local_energy(tiny, phi, phiT, 0.01)
    xi = rng.normal(size=(3, tiny.n_chol))
    phin, wn, ref, elln = O.propagate(tiny, phi, xi, xbar, phiT, ell, np.ones(3), 0.01, 10)
    _, _, _, w2, _ = O.metropolis(tiny, phin, y, phiT, elln, ref, wn, 1, 0, 0)
    assert np.abs(w2 - wn).max() <= 1e-14


def test_combined_angle_is_the_sum_of_the_two_angles(tiny):
    """arg sum S' - arg sum S = arg r + (arg sum S' - arg num_r)."""
    rng = np.random.default_rng(9)
    phi = ai.random_walkers(rng, tiny, 4, spread=1.2)
    y = ai.random_hidden(rng, tiny, 4, 6)
    phiT = O.trial_det(tiny, y)
    eloc, xbar, ep, vb, ell = O.local_energy(tiny, phi, phiT, 0.05)
    xi = rng.normal(size=(4, tiny.n_chol))
    _, _, num_r, elln = O.propagate(tiny, phi, xi, xbar, phiT, ell, np.ones(4), 0.05, 10)
    _, _, den, _ = O.propagate(tiny, phi, xi, xbar, phiT, ell, np.ones(4), 0.05, 10,
                               weight_mode=O.WEIGHT_COMBINED)
    assert np.allclose(den, O.phases(ell).sum(-1))
    Sn = O.phases(elln).sum(-1)
    lhs = np.exp(1j * (np.angle(Sn) - np.angle(den)))
    rhs = np.exp(1j * (np.angle(num_r / den) + np.angle(Sn) - np.angle(num_r)))
    assert np.abs(lhs - rhs).max() <= 1e-13


def test_scale_and_qr_invariance(tiny):
    """E_L, xbar and overlap ratios do not depend on the walker's scale or on
    re-orthogonalisation (Eq. WF-imp); QR keeps span and shifts l by -log det R."""
    rng = np.random.default_rng(10)
    phi = ai.random_walkers(rng, tiny, 3, spread=1.0)
    y = ai.random_hidden(rng, tiny, 3, 4)
    phiT = O.trial_det(tiny, y)
    e1, x1, _, _, l1 = O.local_energy(tiny, phi, phiT, 0.01)
    c = 3.7 * np.exp(0.4j)
    e2, x2, _, _, l2 = O.local_energy(tiny, phi * c, phiT, 0.01)
    assert np.abs(e1 - e2).max() <= 1e-12 * np.abs(e1).max()
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()
    assert np.abs(np.exp(l2 - l1 - 2 * tiny.N * np.log(c)) - 1).max() <= 1e-12
    q, lq = O.reorthogonalize(phi, l1)
    for w in range(3):
        for s in range(2):
            assert np.abs(q[w, s].conj().T @ q[w, s] - np.eye(tiny.N)).max() <= 1e-13
    e3, x3, _, _, l3 = O.local_energy(tiny, q, phiT, 0.01)
    assert np.abs(e1 - e3).max() <= 1e-12 * np.abs(e1).max()
    assert np.abs(x1 - x3).max() <= 1e-12 * np.abs(x1).max()
    assert np.abs(np.exp(l3 - lq) - 1).max() <= 1e-12


def test_force_bias_cancels_first_order_field_dependence(tiny):
    """With the force bias of Eq. shift1 (and the i of Eq. HS-V), d log I / d xi
    at xi = 0 scales as tau^(3/2); with the opposite sign it scales as tau^(1/2)."""
    rng = np.random.default_rng(1)
    phi = ai.random_walkers(rng, tiny, 1, spread=0.8)
    y = ai.random_hidden(np.random.default_rng(2), tiny, 1, 1)
    phiT = O.trial_det(tiny, y)
    for sign, expo in ((1, 1.5), (-1, 0.5)):
        norms = []
        for tau in (1e-2, 1e-3, 1e-4):
            _, xbar, _, _, ell = O.local_energy(tiny, phi, phiT, tau)
            xbar = sign * xbar

            def log_i(xi):
                phn = O.propagate_dets(tiny, phi, xi, xbar, tau, 30)
                return ((xi * xbar - 0.5 * xbar * xbar).sum(-1)[0]
                        + (O.log_overlap(phiT, phn) - ell)[0, 0])
            h = 1e-3
            g = []
            for k in range(tiny.n_chol):
                e = np.zeros((1, tiny.n_chol))
                e[0, k] = h
                g.append((log_i(e) - log_i(-e)) / (2 * h))
            norms.append(np.linalg.norm(g))
        slopes = [math.log10(norms[i] / norms[i + 1]) for i in range(2)]
        assert all(abs(sl - expo) < 0.1 for sl in slopes), (sign, slopes)


# -- Failure handling --------------------------------------------------------

def test_singular_overlap_is_excluded(tiny):
    """A walker column orthogonal to Phi_T makes l = -inf: S = 0, the sample is
    left out of every sum; with every sample singular the walker dies."""
    rng = np.random.default_rng(11)
    phi = ai.random_walkers(rng, tiny, 2, spread=0.5)
    phi[1, 0, :, 0] = 0.0          # walker 1: zero column -> singular for every path
    y = ai.random_hidden(rng, tiny, 2, 3)
    phiT = O.trial_det(tiny, y)
    eloc, xbar, ep, vb, ell = O.local_energy(tiny, phi, phiT, 0.01)
    assert np.all(np.isneginf(ell[1].real)) and np.all(np.isfinite(ell[0].real))
    assert eloc[1] == 0 and np.all(xbar[1] == 0)
    xi = rng.normal(size=(2, tiny.n_chol))
    _, wn, _, _ = O.propagate(tiny, phi, xi, xbar, phiT, ell, np.ones(2), 0.01, 10)
    assert wn[1] == 0.0 and wn[0] > 0.0


# -- Exact diagonalisation fixture --------------------------------------------

def test_tiny_ed_fixture(tiny_H):
    """The stored ED ground energy of the tiny workload (written by
    tests/golden/make_golden.py from the oracle's Fock-space code)."""
    with open(os.path.join(GOLDEN, "tiny_ising_ed.json")) as f:
        g = json.load(f)
    assert tiny_H.shape[0] == g["dim"] == 784
    assert abs(np.linalg.eigvalsh(tiny_H)[0] - g["E0"]) <= 1e-10


def test_estimator_exact_sum():
    w = np.array([1e16, 1.0, -1e16 + 2.0, 3.0])
    e = np.array([1.0, 1.0, 1.0, 1.0]) + 0j
    num, den = O.estimator(np.abs(w), e)
    assert num == math.fsum(np.abs(w))


def test_non_finite_walkers_drop_out(tiny):
    """A walker with a non-finite local energy adds nothing to either sum of
    Eq. mixed_estimator, and a non-finite weight update sets W = 0 while the
    other walkers' weights are those of the same move without it."""
    w = np.array([1.0, 2.0, 0.5])
    e = np.array([-1.0, np.nan, -3.0]) + 0j
    num, den = O.estimator(w, e)
    assert num == -1.0 - 1.5 and den == 1.5
    rng = np.random.default_rng(3)
    phi = ai.random_walkers(rng, tiny, 3, spread=0.4)
    y = ai.random_hidden(rng, tiny, 3, 4)
    phiT = O.trial_det(tiny, y)
    eloc, xbar, _, _, ell = O.local_energy(tiny, phi, phiT, 0.01)
    xi = rng.normal(size=(3, tiny.n_chol))
    _, w_ref, _, _ = O.propagate(tiny, phi, xi, xbar, phiT, ell, np.ones(3), 0.01, 10)
    xbar_bad = xbar.copy()
    xbar_bad[1, 0] = np.inf
    with np.errstate(all="ignore"):
        _, w_bad, _, _ = O.propagate(tiny, phi, xi, xbar_bad, phiT, ell, np.ones(3), 0.01, 10)
    assert w_bad[1] == 0.0 and w_bad[0] == w_ref[0] and w_bad[2] == w_ref[2]


def test_force_bias_cap_keeps_phase_and_clips_modulus(tiny):
    """The force-bias cap (a stabilisation outside the paper, off unless asked
    for): each capped component is the uncapped one times a positive factor
    <= 1, equal to it where |xbar_g| <= cap and of modulus exactly cap
    elsewhere; the local energy is untouched."""
    rng = np.random.default_rng(21)
    phi = ai.random_walkers(rng, tiny, 5, spread=1.5)
    y = ai.random_hidden(rng, tiny, 5, 6)
    phiT = O.trial_det(tiny, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(tiny, phiT, theta, ell)
    x0, e0 = O.walker_estimates(vb, ep, ell, 0.05)
    cap = float(np.median(np.abs(x0)))
    x1, e1 = O.walker_estimates(vb, ep, ell, 0.05, xbar_cap=cap)
    assert np.array_equal(e0, e1)
    big = np.abs(x0) > cap
    assert 0 < big.sum() < big.size
    assert np.array_equal(x1[~big], x0[~big])
    ratio = x1[big] / x0[big]
    assert np.abs(ratio.imag).max() <= 1e-15 and np.all((ratio.real > 0) & (ratio.real < 1))
    assert np.abs(np.abs(x1[big]) - cap).max() <= 1e-15 * cap


def test_local_energy_cap_clips_the_real_part_only(tiny):
    """The local-energy cap (a stabilisation outside the paper, off unless
    asked for): Re E_L inside [E_T - d, E_T + d] is unchanged bit for bit, a
    value outside becomes the nearest bound exactly, Im E_L and the force bias
    are untouched, the map is monotone, and an unbounded width is the identity.
    In the local-energy weight the cap bounds the per-step factor
    exp(-tau (Re E_L - E_T)) to [e^{-tau d}, e^{tau d}]."""
    rng = np.random.default_rng(23)
    phi = ai.random_walkers(rng, tiny, 9, spread=1.5)
    y = ai.random_hidden(rng, tiny, 9, 6)
    phiT = O.trial_det(tiny, y)
    ell, theta = O.green(phiT, phi)
    vb, ep = O.sample_contraction(tiny, phiT, theta, ell)
    x0, e0 = O.walker_estimates(vb, ep, ell, 0.05)
    et = float(np.median(e0.real))
    d = 0.5 * float(np.std(e0.real))
    x1, e1 = O.walker_estimates(vb, ep, ell, 0.05, eloc_cap=(et, d))
    assert np.array_equal(x0, x1) and np.array_equal(e0.imag, e1.imag)
    inside = np.abs(e0.real - et) <= d
    assert 0 < inside.sum() < inside.size
    assert np.array_equal(e1.real[inside], e0.real[inside])
    assert np.all(e1.real[(e0.real > et + d)] == et + d)
    assert np.all(e1.real[(e0.real < et - d)] == et - d)
    order = np.argsort(e0.real, kind="stable")
    assert np.all(np.diff(e1.real[order]) >= 0.0)
    _, e2 = O.walker_estimates(vb, ep, ell, 0.05, eloc_cap=(et, 1e300))
    assert np.array_equal(e2, e0)
    _, e3 = O.walker_estimates(vb, ep, ell, 0.05, eloc_cap=(et, 0.0))
    assert np.array_equal(e3, e0)
    # the weight factor of the local-energy formalism is then bounded
    tau, nw = 0.01, phi.shape[0]
    xi = np.random.default_rng(5).standard_normal((nw, tiny.n_chol))
    w = np.ones(nw)
    _, wn, _, _ = O.propagate(tiny, phi, xi, x1, phiT, ell, w, tau, 10, e_shift=et,
                              weight_mode=O.WEIGHT_LOCAL, eloc=e1)
    assert np.all(wn <= np.exp(tau * d) * (1 + 1e-15))
    live = wn > 0
    assert np.all(wn[live] <= np.exp(tau * d) * (1 + 1e-15))
    # with no cap the same walkers' factors leave that band
    _, wu, _, _ = O.propagate(tiny, phi, xi, x0, phiT, ell, w, tau, 10, e_shift=et,
                              weight_mode=O.WEIGHT_LOCAL, eloc=e0)
    mag_c = np.exp(-tau * (e1.real - et))
    mag_u = np.exp(-tau * (e0.real - et))
    assert mag_c.max() <= np.exp(tau * d) * (1 + 1e-15) < mag_u.max()
    assert np.allclose(wn / np.where(wu > 0, wu, 1.0), np.where(wu > 0, mag_c / mag_u, 1.0),
                       rtol=1e-12, atol=0)


def test_walker_chunks_step_like_the_whole_population(tiny):
    """A step of walkers w0 .. w0 + n - 1 taken alone, with w0 naming their
    place in the population, equals their rows of the whole population's step
    (without the comb, which couples walkers): the random streams belong to
    the walker index, so a population can be stepped in chunks."""
    nw, P, seed = 6, 4, 31
    st = O.init_state(tiny, nw, P, seed)
    kw = dict(dtau=0.01, weight_mode=O.WEIGHT_LOCAL, xbar_cap=1.0, eloc_cap=(-3.0, 2.0))
    for i in range(3):
        whole, rec = O.step(tiny, st, seed, i, **kw)
        parts = []
        for a, b in ((0, 2), (2, 6)):
            sub = O.State(st.phi[a:b], st.w[a:b], st.y[a:b], st.phiT[a:b], st.logov[a:b])
            parts.append(O.step(tiny, sub, seed, i, w0=a, **kw)[0])
        for name in ("phi", "w", "y", "phiT", "logov"):
            joined = np.concatenate([getattr(q, name) for q in parts])
            assert np.array_equal(joined, getattr(whole, name)), (i, name)
        st = whole
    # a wrong offset gives other streams
    sub = O.State(st.phi[2:6], st.w[2:6], st.y[2:6], st.phiT[2:6], st.logov[2:6])
    other = O.step(tiny, sub, seed, 3, w0=0, **kw)[0]
    ref = O.step(tiny, sub, seed, 3, w0=2, **kw)[0]
    assert not np.array_equal(other.y, ref.y)


def test_comb_population_control_properties():
    """The comb keeps the total weight, gives walker k either floor or ceil of
    nw W_k / sum W copies, none to zero-weight walkers, and with a cap first
    clips weights to cap x mean."""
    rng = np.random.default_rng(12)
    nw = 200
    w = rng.exponential(size=nw)
    w[::17] = 0.0
    for cap in (0.0, 3.0):
        parent, wn = O.comb(w, 9, 4, cap)
        wc = np.minimum(w, cap * w.mean()) if cap > 0 else w
        assert np.allclose(wn, wc.sum() / nw) and math.isclose(wn.sum(), wc.sum(), rel_tol=1e-13)
        counts = np.bincount(parent, minlength=nw)
        expect = nw * wc / wc.sum()
        assert np.all(counts >= np.floor(expect) - 1e-9) and np.all(counts <= np.ceil(expect) + 1e-9)
        assert np.all(counts[wc == 0] == 0)
        assert np.all(np.diff(parent) >= 0)
    p0, w0 = O.comb(np.zeros(5), 1, 1)
    assert np.array_equal(p0, np.arange(5))
    # normalize: the same parents, every weight 1
    pa, wa = O.comb(w, 9, 4, 3.0)
    pb, wb = O.comb(w, 9, 4, 3.0, normalize=True)
    assert np.array_equal(pa, pb) and np.all(wb == 1.0)
