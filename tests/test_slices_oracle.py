"""Pins of the oracle's multi-slice trial (Sec. II.C, Eqs. trial and
trial-AF; Sec. III.B: Psi_T = e^{-m tau_T H} Phi_0) against Fock-space brute
force on the tiny system:

* Thouless: the determinant F_m X_m ... X_1 F_0 Phi_0 (long Taylor series)
  equals the Fock-space product of the one-body exponentials on |Phi_0>;
* the Gaussian average over Y of the sampled trial, done by Gauss-Hermite
  quadrature with one generator per slice, equals the exact
  e^{-tau/2 H1} e^{-tau L^2 / 2} e^{-tau H1} ... e^{-tau/2 H1} |Phi_0 Phi_0>;
* m = 0 reduces to single-determinant phaseless AFQMC (the Jastrow trial at
  coupling 0), step for step;
* the path estimator of Eq. local-obs with the complex trial converges to the
  exact <Psi_T|H|phi>/<Psi_T|phi>."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.linalg import expm

import afqmc_inputs as ai
from oracle import afqmc_oracle as O
from oracle import fock as F


@pytest.fixture(scope="module")
def tiny():
    return ai.tiny_ising()


def test_thouless_multislice_trial(tiny):
    tau, m = 0.05, 3
    s = dataclasses.replace(ai.imaginary_time_trial(tiny, m, tau, n_gen=5), trial_taylor=40)
    rng = np.random.default_rng(3)
    y = rng.normal(size=(2, s.K))
    phiT = O.trial_det(s, y)
    assert phiT.dtype == np.complex128
    h = F.one_body_sector(tiny.h1, tiny.N)
    v0 = F.det_vector_sector(tiny.phi0)
    for w in range(2):
        v = expm(-0.5 * tau * h) @ v0
        for l in range(m):
            U = np.einsum("k,kij->ij", y[w, l * 5:(l + 1) * 5], tiny.L[:5])
            v = expm(1j * math.sqrt(tau) * F.one_body_sector(U, tiny.N)) @ v
            v = expm(-(0.5 if l == m - 1 else 1.0) * tau * h) @ v
        got = F.det_vector_sector(phiT[w])
        assert np.abs(got - v).max() <= 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("m", [1, 2])
def test_gaussian_average_of_the_trial_is_the_imaginary_time_state(tiny, m):
    tau = 0.1
    s = dataclasses.replace(ai.imaginary_time_trial(tiny, m, tau, n_gen=1), trial_taylor=40)
    x, wq = np.polynomial.hermite_e.hermegauss(40)
    wq = wq / wq.sum()
    grids = np.meshgrid(*([x] * m), indexing="ij")
    Y = np.stack([g.ravel() for g in grids], -1)
    Wt = np.prod(np.meshgrid(*([wq] * m), indexing="ij"), axis=0).ravel()
    phiT = O.trial_det(s, Y)
    avg = 0.0
    for q in range(len(Wt)):
        v = F.det_vector_sector(phiT[q])
        avg = avg + Wt[q] * np.kron(v, v)
    H1 = F.one_body_full(tiny.h1, tiny.N)
    L0 = F.one_body_full(tiny.L[0], tiny.N)
    ex = np.kron(F.det_vector_sector(tiny.phi0), F.det_vector_sector(tiny.phi0))
    ex = expm(-0.5 * tau * H1) @ ex
    for l in range(m):
        ex = expm(-0.5 * tau * (L0 @ L0)) @ ex
        ex = expm(-(0.5 if l == m - 1 else 1.0) * tau * H1) @ ex
    assert np.abs(avg - ex).max() <= 1e-10 * np.abs(ex).max()


def test_zero_slices_is_single_determinant_ph_afqmc():
    g = ai.small_gaussian(M=10, N=3, n_chol=6, K=4, seed=12)
    s0 = dataclasses.replace(ai.imaginary_time_trial(g, 0, 0.05), slice_F=np.eye(10)[None])
    sj = dataclasses.replace(g, coupling=0.0)
    nw, P, dtau = 5, 3, 0.02
    a = O.init_state(sj, nw, P, 4)
    b = O.State(a.phi.copy(), a.w.copy(), np.zeros((nw, P, 0)), O.trial_det(s0, np.zeros((nw, P, 0))),
                None)
    b.logov = O.log_overlap(b.phiT, b.phi)
    assert np.allclose(b.phiT, a.phiT, rtol=0, atol=1e-15)
    for i in range(3):
        a, ra = O.step(sj, a, 7, i, dtau, n_pc=1, w_cap=4.0)
        b, rb = O.step(s0, b, 7, i, dtau, n_pc=1, w_cap=4.0)
        assert abs(ra["e_num"] / ra["e_den"] - rb["e_num"] / rb["e_den"]) <= 1e-12
        assert np.abs(a.phi - b.phi).max() <= 1e-12
        assert np.abs(a.w - b.w).max() <= 1e-12


def test_path_estimator_with_complex_trial_converges(tiny):
    """m = 1, one generator: <Psi_T| by 60-point quadrature; 64 paths moved by
    the prior proposal at a fixed complex walker."""
    tau = 0.2
    s = dataclasses.replace(ai.imaginary_time_trial(tiny, 1, tau, n_gen=1), trial_taylor=40)
    x, wq = np.polynomial.hermite_e.hermegauss(60)
    wq = wq / wq.sum()
    pt = O.trial_det(s, x[:, None])
    psi = sum(wq[q] * F.det_vector(pt[q], pt[q]) for q in range(len(x)))
    rng = np.random.default_rng(9)
    phi = ai.random_walkers(rng, tiny, 1, spread=0.8)
    H = F.hamiltonian(tiny)
    vw = F.det_vector(phi[0, 0], phi[0, 1])
    e_exact = (psi @ H @ vw) / (psi @ vw)
    P = 64
    y = rng.normal(size=(1, P, 1))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    ests = []
    for st in range(240):
        y, phiT, logov, _, _ = O.metropolis(s, phi, y, phiT, logov, np.ones(1, complex),
                                            np.ones(1), 23, st, 1)
        if st >= 40:
            ell, theta = O.green(phiT, phi)
            vb, ep = O.sample_contraction(s, phiT, theta, ell)
            _, eloc = O.walker_estimates(vb, ep, ell, 0.01)
            ests.append(eloc[0])
    ests = np.array(ests)
    blocks = ests.reshape(20, -1).mean(1)
    err = np.abs(blocks.std(ddof=1)) / math.sqrt(len(blocks))
    assert abs(ests.mean() - e_exact) < 5 * err + 2e-3, (ests.mean(), e_exact, err)
