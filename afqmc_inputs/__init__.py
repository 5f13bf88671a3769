"""Seeded synthetic inputs for phaseless AFQMC with a sampled correlated trial.

This module only *draws* inputs: one-body matrix h1, Cholesky-like vectors
L_gamma, the reference determinant Phi_0 and the trial generators A_k that
define Phi_T(y) = exp(c * sum_k y_k A_k) Phi_0 (Sec. II.C, Eqs. trial-AF and
trial_decomp; Sec. III.A, Eq. Metropolis_sampled_trial).  It holds none of the
method's arithmetic, so both the CPU oracle and the HIP path consume the very
same arrays.

The paper's own workloads (molecular integrals, VAFQMC-optimised trials) are
not available; these generators stand in for them with the shapes and value
distributions given below.  Draw order for one instance, all from
``numpy.random.default_rng(seed)``:

1. h1 off-diagonal: an (M, M) block of N(0, 0.1^2) normals, strict upper
   triangle kept and mirrored; diagonal = linspace(-2, 2, M).
2. L: for gamma = 0..n_chol-1, an (M, M) block of N(0,1) normals times
   0.3 sqrt(8/M)/sqrt(gamma+1), upper triangle (with diagonal) kept and
   mirrored.  The sqrt(8/M) keeps the per-orbital two-body scale
   sum_gamma sum_j L_ij^2 independent of M (dense random vectors would
   otherwise make it grow like M: E(Phi_0) ~ +380 at M = 64 with a mean path
   sign collapsing within ten steps); at M = 8 the factor is exactly 1.
3. Gaussian trial generators only: for k = 0..K-1, an (M, M) block of uniforms
   (mask: u < density) then an (M, M) block of N(0,1) values; the masked upper
   triangle (with diagonal) is mirrored.

Phi_0 is the N lowest eigenvectors of h1 (columns; sign fixed so that the
largest-magnitude entry of each column is positive).  This uses one
eigendecomposition of the input matrix; it is part of choosing the input
determinant, not a step of the method.

Multi-slice trials (Sec. II.C, Eqs. trial and trial-AF; Sec. III.B): the
trial determinant is Phi_T(Y) = F_m X_m ... F_1 X_1 F_0 Phi_0 with
X_l = T_n(i sqrt(s_l) sum_k y_{l,k} A_k) (the propagator's Taylor map) and
caller-given real one-body factors F_l.  imaginary_time_trial() fills them for
Psi_T = e^{-m tau_T H} Phi_0: generators A = the vectors L, s_l = tau_T,
F_0 = F_m = e^{-tau_T h1 / 2} and e^{-tau_T h1} in between (one
eigendecomposition of h1, again a choice of input, not a step of the method).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

HIDDEN_ISING = 0
HIDDEN_GAUSS = 1
TRIAL_JASTROW = 0    # Phi_T(y) = exp(c sum_k y_k A_k) Phi_0
TRIAL_SLICES = 1     # Phi_T(Y) = F_m X_m ... F_1 X_1 F_0 Phi_0 (complex)


@dataclasses.dataclass
class System:
    """One synthetic Hamiltonian plus trial definition (all float64, C order)."""

    M: int                 # one-particle basis size
    N: int                 # electrons per spin (n_up == n_dn)
    n_chol: int            # number of two-body vectors L_gamma
    K: int                 # number of hidden variables y
    hidden_kind: int       # HIDDEN_ISING (y in {-1,+1}) or HIDDEN_GAUSS (y ~ N(0,1))
    coupling: float        # c in Phi_T(y) = exp(c sum_k y_k A_k) Phi_0
    h1: np.ndarray         # [M, M]
    L: np.ndarray          # [n_chol, M, M]
    phi0: np.ndarray       # [M, N], orthonormal columns
    A: np.ndarray          # [K, M, M] symmetric trial generators ([K / m] for slices)
    name: str = ""
    trial_kind: int = TRIAL_JASTROW
    n_slices: int = 0                       # m (TRIAL_SLICES); K = m * len(A)
    slice_s: Optional[np.ndarray] = None    # [m] s_l in X_l = T_n(i sqrt(s_l) sum_k y A_k)
    slice_F: Optional[np.ndarray] = None    # [m + 1, M, M] one-body factors F_0 .. F_m
    trial_taylor: int = 10                  # order n of T_n in X_l


@dataclasses.dataclass
class RunConfig:
    """Run parameters that accompany a System (walkers, samples, time step)."""

    W: int                 # walkers
    P: int                 # hidden-variable samples (tethered paths) per walker
    dtau: float
    n_steps: int
    n_sweep: int = 1
    n_qr: int = 10
    n_taylor: int = 10     # Taylor order of exp(V) in the walker propagator
    proposal: int = 0      # 0 prior / Ising sweep, 1 random walk, 2 learned
    rw_step: float = 0.5
    weight_mode: int = 0   # 0 separate cosines, 1 combined angle, 2 half-plane


def _sym_from_upper(b: np.ndarray, keep_diag: bool = True) -> np.ndarray:
    k = 0 if keep_diag else 1
    u = np.triu(b, k)
    return u + np.triu(u, 1).T


def _phi0_from_h1(h1: np.ndarray, N: int) -> np.ndarray:
    evals, evecs = np.linalg.eigh(h1)
    phi0 = np.array(evecs[:, :N], dtype=np.float64, order="C")
    for j in range(N):
        i = int(np.argmax(np.abs(phi0[:, j])))
        if phi0[i, j] < 0:
            phi0[:, j] = -phi0[:, j]
    return np.ascontiguousarray(phi0)


def make_hamiltonian(rng: np.random.Generator, M: int, n_chol: int):
    """h1 and L in the documented draw order."""
    off = rng.normal(0.0, 0.1, size=(M, M))
    h1 = _sym_from_upper(off, keep_diag=False)
    h1[np.diag_indices(M)] = np.linspace(-2.0, 2.0, M)
    L = np.empty((n_chol, M, M), dtype=np.float64)
    for g in range(n_chol):
        b = rng.normal(0.0, 1.0, size=(M, M)) * (0.3 * math.sqrt(8.0 / M) / math.sqrt(g + 1.0))
        L[g] = _sym_from_upper(b, keep_diag=True)
    return np.ascontiguousarray(h1), np.ascontiguousarray(L)


def make_gauss_generators(rng: np.random.Generator, M: int, K: int,
                          density: float = 0.05) -> np.ndarray:
    A = np.empty((K, M, M), dtype=np.float64)
    for k in range(K):
        mask = rng.random(size=(M, M)) < density
        vals = rng.normal(0.0, 1.0, size=(M, M))
        A[k] = _sym_from_upper(np.where(mask, vals, 0.0), keep_diag=True)
    return np.ascontiguousarray(A)


def make_ising_pair_generators(M: int, K: int) -> np.ndarray:
    """A_k = number operator on orbital pair {2k, 2k+1} (diagonal 0/1)."""
    A = np.zeros((K, M, M), dtype=np.float64)
    for k in range(K):
        for j in (2 * k, 2 * k + 1):
            if j < M:
                A[k, j, j] = 1.0
    return A


def tiny_ising(seed: int = 1000) -> System:
    """M=8, N=2 per spin, 16 vectors, K=4 Ising spins on orbital pairs, c=0.2."""
    rng = np.random.default_rng(seed)
    M, N, n_chol, K = 8, 2, 16, 4
    h1, L = make_hamiltonian(rng, M, n_chol)
    return System(M=M, N=N, n_chol=n_chol, K=K, hidden_kind=HIDDEN_ISING,
                  coupling=0.2, h1=h1, L=L, phi0=_phi0_from_h1(h1, N),
                  A=make_ising_pair_generators(M, K), name="tiny-ising-M8")


def gaussian_system(M: int, N: int, n_chol: int, K: int, seed: int,
                    coupling: float = 0.1, density: float = 0.05,
                    name: str = "") -> System:
    rng = np.random.default_rng(seed)
    h1, L = make_hamiltonian(rng, M, n_chol)
    A = make_gauss_generators(rng, M, K, density)
    return System(M=M, N=N, n_chol=n_chol, K=K, hidden_kind=HIDDEN_GAUSS,
                  coupling=coupling, h1=h1, L=L, phi0=_phi0_from_h1(h1, N), A=A,
                  name=name or f"gauss-M{M}-N{N}-G{n_chol}-K{K}")


def exact_trial_system(M: int = 8, N: int = 2, n_chol: int = 8, K: int = 4,
                       seed: int = 77, hidden_kind: int = HIDDEN_GAUSS,
                       coupling: float = 0.1) -> System:
    """A Hamiltonian whose ground state is exactly the determinant Phi_0.

    L_gamma = P_v S_gamma P_v with P_v the projector on the virtual space of
    h1 (orbitals above the N lowest) so that every L_gamma annihilates the
    occupied orbitals, and trial generators block-diagonal in the occupied /
    virtual split so that exp(c sum y A) Phi_0 spans the same space as Phi_0.
    Then H2 = 1/2 sum L^2 >= 0 vanishes on Phi_0 and Phi_0 is an exact ground
    state (the occupied h1 levels are the lowest), E_0 = 2 * sum_{i<N} eps_i.
    """
    rng = np.random.default_rng(seed)
    h1, L0 = make_hamiltonian(rng, M, n_chol)
    evals, evecs = np.linalg.eigh(h1)
    phi0 = _phi0_from_h1(h1, N)
    virt = evecs[:, N:]
    Pv = virt @ virt.T
    L = np.ascontiguousarray(np.einsum("ij,gjk,kl->gil", Pv, L0, Pv))
    occ = phi0
    Po = occ @ occ.T
    A = np.empty((K, M, M))
    for k in range(K):
        B = _sym_from_upper(rng.normal(0.0, 1.0, size=(M, M)), keep_diag=True)
        A[k] = Po @ B @ Po + Pv @ B @ Pv
    return System(M=M, N=N, n_chol=n_chol, K=K, hidden_kind=hidden_kind,
                  coupling=coupling, h1=h1, L=L, phi0=phi0,
                  A=np.ascontiguousarray(A), name=f"exact-trial-M{M}")


# --------------------------------------------------------------------------
# Named workloads.  Instance seed = 1000 + index.

def workload(idx: int):
    """Return (System or list of Systems, RunConfig or list) for workload idx.

    0: tiny Ising Jastrow (M=8, N=2, 16 vectors, K=4), 64 walkers x 8 samples
    1: FP64 (M=64, N=16, 256 vectors, K=64 Gaussian), 512 walkers x 8 samples
    2: mixed precision (M=128, N=32, 512 vectors, K=128), 1024 walkers x 4
    3: 32 uneven systems (M in [24,160], N=M//4, 4M vectors, K=M//2)
    4: learned proposal (M=96, N=24, 384 vectors, K=128), 2048 walkers x 4
    5: multi-slice trial e^{-2 tau_T H} Phi_0 on the Hamiltonian of workload 1
       (m=2, tau_T=0.01, all 256 vectors as generators: K=512 Gaussian), 512 x 8
    """
    seed = 1000 + idx
    if idx == 0:
        return tiny_ising(seed), RunConfig(W=64, P=8, dtau=0.01, n_steps=200)
    if idx == 1:
        return (gaussian_system(64, 16, 256, 64, seed),
                RunConfig(W=512, P=8, dtau=0.005, n_steps=2000))
    if idx == 2:
        return (gaussian_system(128, 32, 512, 128, seed),
                RunConfig(W=1024, P=4, dtau=0.005, n_steps=2000))
    if idx == 3:
        rng = np.random.default_rng(seed)
        Ms = rng.integers(24, 161, size=32)
        Ws = np.rint(np.exp(rng.uniform(math.log(64), math.log(1024), size=32))).astype(int)
        systems, runs = [], []
        for s, (M, W) in enumerate(zip(Ms, Ws)):
            M = int(M)
            systems.append(gaussian_system(M, M // 4, 4 * M, M // 2, seed * 100 + s))
            runs.append(RunConfig(W=int(W), P=4, dtau=0.005, n_steps=200))
        return systems, runs
    if idx == 4:
        return (gaussian_system(96, 24, 384, 128, seed),
                RunConfig(W=2048, P=4, dtau=0.005, n_steps=2000, proposal=2))
    if idx == 5:
        base = gaussian_system(64, 16, 256, 64, 1001)
        return (imaginary_time_trial(base, 2, 0.01, name="itime-M64-N16-G256-m2"),
                RunConfig(W=512, P=8, dtau=0.005, n_steps=2000, proposal=1, rw_step=0.08))
    raise ValueError(f"no workload {idx}")


def imaginary_time_trial(sys: System, m: int, tau_T: float, n_gen: Optional[int] = None,
                         name: str = "") -> System:
    """The system with the trial Psi_T = e^{-m tau_T H} Phi_0 in multi-slice
    form (Sec. III.B with t_j = tau_T, H_T^j = H): generators A = the first
    n_gen vectors L (all by default), s_l = tau_T, F_0 = F_m = e^{-tau_T h1/2},
    F_l = e^{-tau_T h1} for 0 < l < m (F_0 = identity if m = 0: Psi_T = Phi_0).
    Hidden variables are Gaussian, K = m * n_gen."""
    n_gen = sys.n_chol if n_gen is None else n_gen
    lam, Q = np.linalg.eigh(sys.h1)
    half = (Q * np.exp(-0.5 * tau_T * lam)) @ Q.T
    full = (Q * np.exp(-tau_T * lam)) @ Q.T
    F = np.empty((m + 1, sys.M, sys.M))
    F[0] = half if m > 0 else np.eye(sys.M)
    for l in range(1, m + 1):
        F[l] = half if l == m else full
    return dataclasses.replace(
        sys, K=m * n_gen, hidden_kind=HIDDEN_GAUSS, coupling=0.0,
        A=np.ascontiguousarray(sys.L[:n_gen]), trial_kind=TRIAL_SLICES, n_slices=m,
        slice_s=np.full(m, float(tau_T)), slice_F=np.ascontiguousarray(F),
        name=name or f"{sys.name}-itime-m{m}")


def small_gaussian(M: int = 16, N: int = 4, n_chol: int = 24, K: int = 8,
                   seed: int = 5) -> System:
    """A small Gaussian-hidden system for fast parity tests."""
    return gaussian_system(M, N, n_chol, K, seed)


# --------------------------------------------------------------------------
# Walker-state generators (random but structured like a running simulation).

def random_walkers(rng: np.random.Generator, sys: System, nw: int,
                   spread: float = 0.3) -> np.ndarray:
    """phi[nw][2][M][N] complex128: Phi_0 plus a complex perturbation."""
    M, N = sys.M, sys.N
    base = np.broadcast_to(sys.phi0, (nw, 2, M, N))
    pert = rng.normal(size=(nw, 2, M, N)) + 1j * rng.normal(size=(nw, 2, M, N))
    return np.ascontiguousarray(base + spread * pert / math.sqrt(M))


def random_hidden(rng: np.random.Generator, sys: System, nw: int, P: int) -> np.ndarray:
    """y[nw][P][K] float64 drawn from the trial prior p_T."""
    if sys.hidden_kind == HIDDEN_ISING:
        return np.where(rng.random(size=(nw, P, sys.K)) < 0.5, -1.0, 1.0)
    return rng.normal(size=(nw, P, sys.K))


def random_fields(rng: np.random.Generator, sys: System, nw: int) -> np.ndarray:
    return rng.normal(size=(nw, sys.n_chol))


# --------------------------------------------------------------------------
# Learned-proposal network parameters.

MLP_HIDDEN = 256


def mlp_params(rng: np.random.Generator, M: int, K: int, H: int = MLP_HIDDEN,
               last_scale: float = 0.0) -> dict:
    """Initial weights of the proposal network, rounded to float32.

    W1 [M+K][H], W2 [H][H] ~ N(0, 1/fan_in), zero biases; the output layer
    W3 [H][2K] ~ N(0, last_scale^2 / H) and b3 = 0.  last_scale = 0 makes the
    network's first proposals the random walk of step sqrt(2).
    """
    D = M + K
    p = {
        "W1": rng.normal(size=(D, H)) / math.sqrt(D),
        "b1": np.zeros(H),
        "W2": rng.normal(size=(H, H)) / math.sqrt(H),
        "b2": np.zeros(H),
        "W3": rng.normal(size=(H, 2 * K)) * (last_scale / math.sqrt(H)),
        "b3": np.zeros(2 * K),
    }
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
