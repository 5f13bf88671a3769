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

here = os.path.dirname(os.path.abspath(__file__))
s = ai.tiny_ising()
H = F.hamiltonian(s)
E = np.linalg.eigvalsh(H)
with open(os.path.join(here, "tiny_ising_ed.json"), "w") as f:
    json.dump({"workload": "tiny Ising Jastrow, M=8, N_up=N_dn=2, 16 vectors, seed 1000",
               "dim": int(H.shape[0]), "E0": float(E[0]), "E1": float(E[1]),
               "source": "exact diagonalisation of H = sum_s h1 + 1/2 sum_g L_g^2 (Eq. H_MC)"},
              f, indent=1)
print("E0", E[0])
