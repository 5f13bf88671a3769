"""Writes tests/golden/*.json from the oracle's Fock-space code only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import afqmc_inputs as ai  # noqa: E402
from oracle import fock as F  # noqa: E402

from scipy.linalg import expm  # noqa: E402

here = os.path.dirname(os.path.abspath(__file__))
s = ai.tiny_ising()
H = F.hamiltonian(s)
E = np.linalg.eigvalsh(H)
# the trial |Psi_T> = 2^-K sum_y exp(U-hat(y)) |Phi_0>_up |Phi_0>_dn over all 2^K
# Ising states (Eqs. trial_decomp and Metropolis_sampled_trial), built with the
# Fock-space exponential of U(y) = c sum_k y_k A_k (no determinant code)
v0 = F.det_vector_sector(s.phi0)
psi = 0.0
for b in range(2 ** s.K):
    yk = np.array([1.0 if (b >> k) & 1 else -1.0 for k in range(s.K)])
    U = s.coupling * np.einsum("k,kij->ij", yk, s.A)
    vs = expm(F.one_body_sector(U, s.N)) @ v0
    psi = psi + np.kron(vs, vs) / 2 ** s.K
phi0 = np.kron(v0, v0)
E_var = float(psi @ H @ psi / (psi @ psi))
E_mix0 = float(psi @ H @ phi0 / (psi @ phi0))
with open(os.path.join(here, "tiny_ising_ed.json"), "w") as f:
    json.dump({"workload": "tiny Ising Jastrow, M=8, N_up=N_dn=2, 16 vectors, seed 1000",
               "dim": int(H.shape[0]), "E0": float(E[0]), "E1": float(E[1]),
               "E_var": E_var, "E_mixed_phi0": E_mix0,
               "source": "exact diagonalisation of H = sum_s h1 + 1/2 sum_g L_g^2 (Eq. H_MC); "
                         "E_var = <Psi_T|H|Psi_T>/<Psi_T|Psi_T> and E_mixed_phi0 = "
                         "<Psi_T|H|Phi_0>/<Psi_T|Phi_0> of the 2^K-state trial"},
              f, indent=1)
print("E0", E[0], "E_var", E_var, "E_mixed_phi0", E_mix0)
