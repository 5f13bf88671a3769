"""Pins of the oracle's initialisation from the trial and of its measurement
with extra paths (App. B, Initialization and Measurement; Sec. III.A, end of
the composite-walker part), against Fock-space brute force on the tiny Ising
system (2^K = 16 trial states, so every sum over hidden variables is exact).

The Fock-space trial states here are built with the exponential of the
second-quantised generator c sum_k y_k A_k acting on |Phi_0> (no determinant
code), and H is the Fock-space Hamiltonian of Eq. H_MC."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

import afqmc_inputs as ai
from oracle import afqmc_oracle as O
from oracle import fock as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ising_states(K):
    return np.array([[1.0 if (b >> k) & 1 else -1.0 for k in range(K)] for b in range(2 ** K)])


def _index(y):
    return ((y > 0) * (1 << np.arange(y.shape[-1]))).sum(-1).astype(int)


@pytest.fixture(scope="module")
def strong():
    """The tiny Ising system with coupling 0.5: the pair density of Eq.
    Metropolis then spans three decades, and E_var differs clearly from the
    mixed energy of the plain start Phi_0."""
    s = dataclasses.replace(ai.tiny_ising(), coupling=0.5)
    v0 = F.det_vector_sector(s.phi0)
    V = []
    for yk in _ising_states(s.K):
        v = expm(F.one_body_sector(s.coupling * np.einsum("k,kij->ij", yk, s.A), s.N)) @ v0
        V.append(np.kron(v, v))
    V = np.array(V)
    return s, V, F.hamiltonian(s), np.kron(v0, v0)


def test_pair_chain_samples_the_pair_density(strong):
    """After the pair chain the (walker field, path) pairs have the law
    pi(Y, Y') ~ |<Phi_T(Y')|Phi_T(Y)>| of Eq. Metropolis (uniform Ising prior):
    chi-square over the 256 cells, for the partner copy (no sweeps) and for
    a path after its own sweeps."""
    s, V, _, _ = strong
    Ov = V @ V.T
    pi = Ov / Ov.sum()
    nw = 2000
    st, yw = O.init_metropolis(s, nw, 2, 5, n_pair=10, n_burn=3)
    assert np.array_equal(st.w, np.full(nw, 2.0))
    bw = _index(yw)
    for p in range(2):
        cnt = np.zeros((16, 16))
        np.add.at(cnt, (bw, _index(st.y[:, p])), 1)
        exp_ = pi * nw
        cells = exp_ > 5
        chi2 = (((cnt - exp_) ** 2 / np.where(cells, exp_, 1.0))[cells]).sum()
        dof = cells.sum() - 1
        assert chi2 < dof + 5 * math.sqrt(2 * dof), (p, chi2, dof)
    # the plain prior law of the walker field is rejected by the same test
    m_prior = np.full(16, nw / 16.0)
    cw = np.bincount(bw, minlength=16)
    assert ((cw - m_prior) ** 2 / m_prior).sum() > 15 + 5 * math.sqrt(30)


def test_beta_zero_energy_is_the_variational_energy(strong):
    """At beta = 0 the mixed estimator over walkers initialised from the trial
    is the Metropolis estimate of <Psi_T|H|Psi_T>/<Psi_T|Psi_T> (App. B,
    Initialization), not the mixed energy of the plain start Phi_0."""
    s, V, H, v00 = strong
    psi = V.mean(0)
    e_var = psi @ H @ psi / (psi @ psi)
    e_mix0 = psi @ H @ v00 / (psi @ v00)
    nw, P = 2000, 6
    st, _ = O.init_metropolis(s, nw, P, 11, n_pair=10, n_burn=2)
    ell, theta = O.green(st.phiT, st.phi)
    vb, ep = O.sample_contraction(s, st.phiT, theta, ell)
    _, eloc = O.walker_estimates(vb, ep, ell, 0.01)
    num, den = O.estimator(st.w, eloc)
    e0 = num / den
    err = eloc.real.std(ddof=1) / math.sqrt(nw)      # walkers are independent
    assert abs(e0 - e_var) < 4 * err, (e0, e_var, err)
    assert abs(e_mix0 - e_var) > 10 * err


def test_beta_zero_energy_tiny_golden():
    """The same on the tiny workload itself against the stored E_var."""
    g = json.load(open(os.path.join(GOLDEN, "tiny_ising_ed.json")))
    s = ai.tiny_ising()
    nw = 1500
    st, _ = O.init_metropolis(s, nw, 4, 12, n_pair=8, n_burn=2)
    eloc, _, _, _, _ = O.local_energy(s, st.phi, st.phiT, 0.01)
    e0 = (st.w * eloc.real).sum() / st.w.sum()
    err = eloc.real.std(ddof=1) / math.sqrt(nw)
    assert abs(e0 - g["E_var"]) < 4 * err, (e0, g["E_var"], err)


def test_random_walk_init_matches_variational_energy_by_quadrature():
    """Gaussian hidden variables (K = 2) with the random-walk proposal: the
    beta = 0 energy equals <Psi_T|H|Psi_T>/<Psi_T|Psi_T> with the trial
    integral done by Gauss-Hermite quadrature in Fock space."""
    s = ai.gaussian_system(6, 2, 3, 2, seed=4, coupling=0.15, density=0.6)
    H = F.hamiltonian(s)
    v0 = F.det_vector_sector(s.phi0)
    x, wq = np.polynomial.hermite_e.hermegauss(24)
    wq = wq / wq.sum()
    psi = 0.0
    for i in range(len(x)):
        for j in range(len(x)):
            U = s.coupling * (x[i] * s.A[0] + x[j] * s.A[1])
            v = expm(F.one_body_sector(U, s.N)) @ v0
            psi = psi + wq[i] * wq[j] * np.kron(v, v)
    e_var = psi @ H @ psi / (psi @ psi)
    nw = 1500
    st, _ = O.init_metropolis(s, nw, 4, 13, n_pair=30, n_burn=4, proposal=O.PROPOSAL_RW,
                              rw_step=0.8)
    eloc, _, _, _, _ = O.local_energy(s, st.phi, st.phiT, 0.01)
    e0 = (st.w * eloc.real).sum() / st.w.sum()
    err = eloc.real.std(ddof=1) / math.sqrt(nw)
    assert abs(e0 - e_var) < 4 * err, (e0, e_var, err)


def _walkers_after_steps(s, nw, P, seed, n):
    """A population moved n steps, so walkers are complex and not trial states."""
    st = O.init_state(s, nw, P, seed)
    Eh, h1p = O.half_kinetic(s, 0.05), O.h1_eff(s)
    for i in range(n):
        st, _ = O.step(s, st, seed, i, 0.05, Eh=Eh, h1p=h1p, normalize=False)
    return st


def test_measurement_with_copied_paths_is_the_plain_estimator():
    """With P' = P or 3P copies and no sweeps, R = P'/P exactly and the
    corrected estimator is the plain one (Eq. mixed_estimator)."""
    s = ai.tiny_ising()
    st = _walkers_after_steps(s, 12, 4, 3, 5)
    eloc, _, _, _, _ = O.local_energy(s, st.phi, st.phiT, 0.05)
    num, den = O.estimator(st.w, eloc)
    for P2 in (4, 12):
        n2, d2, e2, R = O.measure_extra(s, st.phi, st.y, st.phiT, st.logov, st.w, 9,
                                        O.MEASURE_STEP, P2, 0, 0.05)
        alive = np.abs(O.phases(st.logov).sum(-1)) > 0
        assert np.allclose(R[alive], P2 / 4, rtol=1e-12, atol=0)
        assert np.allclose(e2[alive], eloc[alive], rtol=1e-12, atol=0)
        assert abs(n2 / d2 - num / den) <= 1e-12 * abs(num / den)


def test_measurement_paths_converge_to_exact_trial_ratios(strong):
    """Many fresh paths at a fixed walker: E'_L tends to the exact
    <Psi_T|H|phi>/<Psi_T|phi>, and the new sign sum per path,
    R sum_p S_p / P', to the exact <Psi_T|phi> / sum_y p(y)|<Phi_T(y)|phi>|
    (Eq. sign-path averaged over the path density of Eq. PDF-Y)."""
    s, V, H, _ = strong
    rng = np.random.default_rng(41)
    nw, P, P2 = 3, 4, 3000
    phi = ai.random_walkers(rng, s, nw, spread=1.0)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    w = np.ones(nw)
    _, _, e2, R = O.measure_extra(s, phi, y, phiT, logov, w, 21, O.MEASURE_STEP, P2, 40, 0.05)
    S = O.phases(logov).sum(-1)
    psi = V.mean(0)
    for k in range(nw):
        vw = F.det_vector(phi[k, 0], phi[k, 1])
        ov = V @ vw                                    # <Phi_T(y)|phi> for all 16 y
        e_exact = (psi @ H @ vw) / (psi @ vw)
        s_exact = ov.sum() / np.abs(ov).sum()
        s_est = R[k] * S[k] / P2
        assert abs(e2[k] - e_exact) < 0.02 * abs(e_exact), (k, e2[k], e_exact)
        assert abs(s_est - s_exact) < 0.05, (k, s_est, s_exact)
