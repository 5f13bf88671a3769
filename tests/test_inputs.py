"""The seeded synthetic inputs follow their stated recipe and are reproducible:
h1 with a linspace(-2, 2) diagonal and N(0, 0.1^2) off-diagonal entries,
symmetric Cholesky vectors of scale 0.3 sqrt(8/M) / sqrt(g+1), sparse symmetric
Gaussian trial generators (density 0.05) or orbital-pair number operators for
Ising fields, and Phi_0 the lowest N eigenvectors of h1."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import afqmc_inputs as ai  # noqa: E402


def test_workloads_are_reproducible():
    for idx in (0, 1, 5):
        a, ra = ai.workload(idx)
        b, rb = ai.workload(idx)
        for name in ("h1", "L", "phi0", "A"):
            assert np.array_equal(getattr(a, name), getattr(b, name)), (idx, name)
        assert ra == rb


@pytest.mark.parametrize("idx,shape", [(1, (64, 16, 256, 64)), (2, (128, 32, 512, 128)),
                                       (4, (96, 24, 384, 128))])
def test_gaussian_workload_recipe(idx, shape):
    s, run = ai.workload(idx)
    M, N, G, K = shape
    assert (s.M, s.N, s.n_chol, s.K) == shape
    assert s.hidden_kind == ai.HIDDEN_GAUSS and s.coupling == 0.1
    # h1: symmetric, prescribed diagonal, off-diagonal spread 0.1
    assert np.array_equal(s.h1, s.h1.T)
    assert np.array_equal(np.diag(s.h1), np.linspace(-2.0, 2.0, M))
    off = s.h1[np.triu_indices(M, 1)]
    assert abs(off.std() / 0.1 - 1.0) < 0.05 and abs(off.mean()) < 0.01
    # Cholesky vectors: symmetric, entry spread 0.3 sqrt(8/M) / sqrt(g + 1)
    assert np.array_equal(s.L, s.L.transpose(0, 2, 1))
    for g in (0, 3, G // 2, G - 1):
        spread = s.L[g][np.triu_indices(M)].std()
        assert abs(spread / (0.3 * math.sqrt(8.0 / M) / math.sqrt(g + 1.0)) - 1.0) < 0.08, g
    # trial generators: symmetric, upper triangle (with diagonal) 5 % dense
    assert np.array_equal(s.A, s.A.transpose(0, 2, 1))
    iu = np.triu_indices(M)
    density = np.count_nonzero(s.A[:, iu[0], iu[1]]) / (K * len(iu[0]))
    assert abs(density - 0.05) < 0.005
    # Phi_0: orthonormal, the lowest N eigenvectors of h1
    assert np.allclose(s.phi0.T @ s.phi0, np.eye(N), atol=1e-12)
    w = np.linalg.eigvalsh(s.h1)[:N]
    assert np.allclose(s.phi0.T @ s.h1 @ s.phi0, np.diag(w), atol=1e-12)
    assert run.dtau == 0.005


def test_tiny_ising_recipe():
    s, run = ai.workload(0)
    assert (s.M, s.N, s.n_chol, s.K) == (8, 2, 16, 4)
    assert s.hidden_kind == ai.HIDDEN_ISING and s.coupling == 0.2
    for k in range(s.K):  # number operator on the orbital pair {2k, 2k+1}
        expect = np.zeros((8, 8))
        expect[2 * k, 2 * k] = expect[2 * k + 1, 2 * k + 1] = 1.0
        assert np.array_equal(s.A[k], expect)
    assert (run.W, run.P, run.dtau) == (64, 8, 0.01)


def test_uneven_batch_recipe():
    systems, runs = ai.workload(3)
    assert len(systems) == len(runs) == 32
    for s, r in zip(systems, runs):
        assert 24 <= s.M <= 160 and s.N == s.M // 4
        assert s.n_chol == 4 * s.M and s.K == s.M // 2
        assert 64 <= r.W <= 1024 and r.P == 4
    # the draw spans the configured range: systems past M = 128 and N = 32 occur
    assert max(s.M for s in systems) > 150 and min(s.M for s in systems) < 30
    assert any(s.N > 32 for s in systems)
