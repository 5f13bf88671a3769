"""Fock-space brute force for tiny systems: exact references for the oracle.

TEST INFRASTRUCTURE ONLY (used by tests/ to pin the oracle).

Basis: for each spin, occupation sets {i_1 < ... < i_N} of M orbitals, the
state c+_{i_1} ... c+_{i_N} |0>; the two-spin space is the Kronecker product
(up-spin creators first).  A spin-conserving one-body operator
sum_ij U_ij c+_i c_j acts as U_up (x) 1 + 1 (x) U_dn, because moving a
creator/annihilator pair through the other spin's string costs no sign.
A Slater determinant with orbital matrix Phi [M, N] has the amplitude
det(Phi[S, :]) on occupation set S (the expansion of prod_k sum_i Phi_ik c+_i).
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def sector_basis(M: int, N: int):
    occs = list(itertools.combinations(range(M), N))
    index = {o: k for k, o in enumerate(occs)}
    return occs, index


def one_body_sector(U: np.ndarray, N: int) -> np.ndarray:
    """Matrix of sum_ij U_ij c+_i c_j in the N-particle sector of one spin."""
    M = U.shape[0]
    occs, index = sector_basis(M, N)
    D = len(occs)
    out = np.zeros((D, D), dtype=np.result_type(U.dtype, np.float64))
    for b, occ in enumerate(occs):
        occset = set(occ)
        for j in occ:
            nj = sum(1 for q in occ if q < j)
            rest = [q for q in occ if q != j]
            restset = set(rest)
            for i in range(M):
                if U[i, j] == 0 or i in restset:
                    continue
                ni = sum(1 for q in rest if q < i)
                new = tuple(sorted(rest + [i]))
                sign = -1.0 if (nj + ni) % 2 else 1.0
                out[index[new], b] += sign * U[i, j]
    return out


def one_body_full(U: np.ndarray, N: int) -> np.ndarray:
    """The two-spin operator U_up (x) 1 + 1 (x) U_dn (same U and N for both spins)."""
    Os = one_body_sector(U, N)
    I = np.eye(Os.shape[0])
    return np.kron(Os, I) + np.kron(I, Os)


def det_vector_sector(Phi: np.ndarray) -> np.ndarray:
    M, N = Phi.shape
    occs, _ = sector_basis(M, N)
    return np.array([np.linalg.det(Phi[list(o), :]) for o in occs])


def det_vector(Phi_up: np.ndarray, Phi_dn: np.ndarray) -> np.ndarray:
    return np.kron(det_vector_sector(Phi_up), det_vector_sector(Phi_dn))


def hamiltonian(sys) -> np.ndarray:
    """H = sum_s h1 + 1/2 sum_g Lhat_g^2 in the (N, N) sector (Eq. H_MC)."""
    H = one_body_full(sys.h1, sys.N).astype(np.float64)
    for g in range(sys.n_chol):
        Lg = one_body_full(sys.L[g], sys.N)
        H = H + 0.5 * (Lg @ Lg)
    return H


def ground_energy(sys) -> float:
    return float(np.linalg.eigvalsh(hamiltonian(sys))[0])


def expm_herm(H: np.ndarray, t: complex) -> np.ndarray:
    """exp(t H) for a real symmetric H by eigendecomposition."""
    lam, Q = np.linalg.eigh(H)
    return (Q * np.exp(t * lam)) @ Q.T
