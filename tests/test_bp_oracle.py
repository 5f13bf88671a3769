"""Pins of the oracle's back-propagated one-body density matrix (App. B,
Measurement; Eqs. AFQMC_Metropolis_measure and AFQMC_Metropolis_measure2)
against Fock-space brute force on the tiny system: the restored projectors
are the Fock-space exponentials of the one-body operators (long Taylor
series on the determinant side), the operator c+_j c_i (both spins) sits
between them and the saved walker, and the sampled trial's paths are
weighted by <Phi_T(Y_p)|...|phi_mid> / |O_p(phi_end)|."""
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


def _fock_bp(s, phi_mid, xi, xbar, phiT, logov_end, tau):
    """Sum_p (<Phi_T,p| B_h..B_1 c+_j c_i |phi_mid>) / |O_p| over the same sum without the operator."""
    H1 = F.one_body_full(s.h1, s.N)
    ket = F.det_vector(phi_mid[0], phi_mid[1]).astype(complex)
    Bs = []
    for i in range(xi.shape[0]):
        V = O.field_matrix(s, xi[i][None], xbar[i][None], tau)[0]
        Bs.append(expm(-0.5 * tau * H1) @ expm(F.one_body_full(V, s.N)) @ expm(-0.5 * tau * H1))
    M = s.M
    num = np.zeros((M, M), dtype=complex)
    den = 0.0
    for p in range(phiT.shape[0]):
        bra = F.det_vector(phiT[p], phiT[p])
        for B in reversed(Bs):         # <bra| B_h ... B_1
            bra = bra @ B
        wgt = 1.0 / abs(np.exp(logov_end[p]))
        den = den + wgt * (bra @ ket)
        for i in range(M):
            for j in range(M):
                U = np.zeros((M, M))
                U[j, i] = 1.0
                num[i, j] += wgt * (bra @ F.one_body_full(U, s.N) @ ket)
    return num / den


@pytest.mark.parametrize("h", [0, 1, 3])
def test_back_propagated_density_against_fock_space(tiny, h):
    s, tau, P = tiny, 0.05, 3
    rng = np.random.default_rng(10 + h)
    phi_mid = ai.random_walkers(rng, s, 1, spread=0.5)
    xi = rng.normal(size=(1, h, s.n_chol))
    xbar = 0.2 * (rng.normal(size=(1, h, s.n_chol)) + 1j * rng.normal(size=(1, h, s.n_chol)))
    y = ai.random_hidden(rng, s, 1, P)
    phiT = O.trial_det(s, y)
    # the walker at the measurement step: phi_mid moved by the same projectors
    phi_end = phi_mid.copy()
    for i in range(h):
        phi_end = O.propagate_dets(s, phi_end, xi[:, i], xbar[:, i], tau, 40)
    logov = O.log_overlap(phiT, phi_end)
    num, den, Rk = O.back_propagated_density(s, phi_mid, xi, xbar, phiT, logov, np.ones(1), tau, 40)
    ref = _fock_bp(s, phi_mid[0], xi[0], xbar[0], phiT[0], logov[0], tau)
    assert np.abs(Rk[0] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert abs(np.trace(Rk[0]) - 2 * s.N) <= 1e-10
    assert den == 1.0 and np.allclose(num, Rk[0].real)


def test_no_restored_steps_is_the_mixed_density(tiny):
    """h = 0: the path-weighted mixed density with weights S_p (Eq. local-obs
    with the operator c+_j c_i in place of H)."""
    s = tiny
    rng = np.random.default_rng(4)
    nw, P = 3, 5
    phi = ai.random_walkers(rng, s, nw, spread=0.6)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    w = rng.uniform(0.5, 1.5, size=nw)
    num, den, Rk = O.back_propagated_density(s, phi, np.zeros((nw, 0, s.n_chol)),
                                             np.zeros((nw, 0, s.n_chol), complex), phiT, ell, w,
                                             0.01, 10)
    S = O.phases(ell)
    for k in range(nw):
        Rm = sum(S[k, p] * (theta[k, p, 0] + theta[k, p, 1]) @ phiT[k, p].T for p in range(P))
        Rm /= S[k].sum()
        assert np.abs(Rk[k] - Rm).max() <= 1e-12 * np.abs(Rm).max()
    assert abs(den - w.sum()) <= 1e-14 * den
    assert np.allclose(num, np.einsum("k,kij->ij", w, Rk.real), rtol=1e-13, atol=1e-13)
