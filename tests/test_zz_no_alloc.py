"""The entry point that allocates nothing, afqmc_local_energy_static, through
the C ABI: its local energies, per-path energies and force biases equal those
of afqmc_local_energy (the same kernels with workspace scratch) on two calls in
a row, the second with fewer walkers, in every contraction family; sizes past
its fixed scratch are refused on the host."""
import sys

import numpy as np
import pytest

import afqmc_inputs as ai
from oracle import afqmc_oracle as O

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


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    # name: (system factory, P, walkers of the first call, of the second, precision)
    "reg-M20-fp64": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 3, 9, 4, 0),
    "reg-M64-G256-fp64": (lambda: ai.workload(1)[0], 8, 6, 2, 0),
    "wg-M72-fp64": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 3, 5, 2, 0),
    "sh-M72-fp32": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 3, 5, 2, 1),
    "sh-M96-bf16x3": (lambda: ai.small_gaussian(M=96, N=24, n_chol=48, K=32, seed=8), 4, 4, 1, 3),
}


def _inputs(s, P, nw, seed):
    rng = np.random.default_rng(seed)
    phi = ai.random_walkers(rng, s, nw, spread=0.5)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    ell, theta = O.green(phiT, phi)
    return dev(phiT), dev(theta), dev(ell)


def _outputs(nw, P, G):
    z = dict(dtype=torch.complex128, device="cuda")
    return torch.zeros(nw, **z), torch.zeros(nw, P, **z), torch.zeros(nw, G, **z)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1.0)


@pytest.mark.parametrize("case", list(CASES))
def test_static_scratch_matches_workspace_entry_point(case):
    from paper_2505_18519_amd import afqmc as A
    fac, P, nw1, nw2, prec = CASES[case]
    s = fac()
    ctx = A.Context(s, P, 0.01, max_walkers=nw1, precision=prec)
    for call, (nw, seed) in enumerate(((nw1, 1), (nw2, 2))):
        _say("no-alloc", case, "call", call, "nw", nw)
        phiT, theta, ell = _inputs(s, P, nw, seed)
        el_ref, ep_ref, xb_ref = _outputs(nw, P, s.n_chol)
        A.afqmc_local_energy(ctx, nw, phiT, theta, ell, el_ref, ep_ref, xb_ref)
        el, ep, xb = _outputs(nw, P, s.n_chol)
        el2, _, xb2 = _outputs(nw, P, s.n_chol)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        # with the per-path energies taken by the caller, and with both kept in scratch
        A.afqmc_local_energy_static(ctx, nw, phiT, theta, ell, el, ep, xb)
        A.afqmc_local_energy_static(ctx, nw, phiT, theta, ell, el2, None, xb2)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        r_el, r_ep, r_xb = host(el_ref), host(ep_ref), host(xb_ref)
        assert _rel(host(el), r_el) <= TOL and _rel(host(el2), r_el) <= TOL
        assert _rel(host(ep), r_ep) <= TOL
        for w in range(nw):
            assert np.linalg.norm(host(xb)[w] - r_xb[w]) <= TOL * np.linalg.norm(r_xb[w])
            assert np.linalg.norm(host(xb2)[w] - r_xb[w]) <= TOL * np.linalg.norm(r_xb[w])


def test_static_scratch_refuses_sizes_past_its_maximum():
    _say("no-alloc: size limit")
    from paper_2505_18519_amd import afqmc as A
    s = ai.small_gaussian(M=8, N=2, n_chol=4096, K=4, seed=3)
    P = 64
    # 16 nw P G bytes of vb: 65 walkers need 16 * 65 * 64 * 4096 > 64 MiB
    nw = 65
    ctx = A.Context(s, P, 0.01, max_walkers=1)
    z = dict(device="cuda")
    phiT = torch.zeros(nw, P, s.M, s.N, dtype=torch.float64, **z)
    theta = torch.zeros(nw, P, 2, s.M, s.N, dtype=torch.complex128, **z)
    ell = torch.zeros(nw, P, dtype=torch.complex128, **z)
    el = torch.zeros(nw, dtype=torch.complex128, **z)
    with pytest.raises(A.AfqmcError) as ei:
        A.afqmc_local_energy_static(ctx, nw, phiT, theta, ell, el)
    assert ei.value.status == 2 and "scratch" in str(ei.value)
