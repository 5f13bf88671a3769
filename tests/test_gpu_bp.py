"""Back-propagated one-body density matrix (App. B, Measurement; Eqs.
AFQMC_Metropolis_measure and AFQMC_Metropolis_measure2) through the C ABI
against the FP64 oracle: direct calls on seeded inputs (real and complex
trials, h = 0 to 4, both kernel families' shapes), and a trajectory whose
field history and saved walkers follow the comb's parents on both sides."""
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
    # name: (system factory, P, nw, h)
    "tiny-ising-h3": (lambda: ai.tiny_ising(), 4, 6, 3),
    "tiny-ising-h0": (lambda: ai.tiny_ising(), 4, 3, 0),
    "gauss-M20-N5-ragged-h2": (lambda: ai.small_gaussian(M=20, N=5, n_chol=24, K=8, seed=5), 3, 4, 2),
    "cfg-M64-N16-G256-h2": (lambda: ai.workload(1)[0], 8, 2, 2),
    "gauss-M72-N20-h1": (lambda: ai.small_gaussian(M=72, N=20, n_chol=40, K=16, seed=7), 2, 2, 1),
    "itime-M8-m2-h4": (lambda: ai.imaginary_time_trial(ai.tiny_ising(), 2, 0.05), 5, 3, 4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_bp_density_matches_oracle(case):
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    mk, P, nw, h = CASES[case]
    s = mk()
    _say("case", case)
    dtau = 0.01
    rng = np.random.default_rng(8)
    phi_mid = ai.random_walkers(rng, s, nw, spread=0.5)
    hx = rng.normal(size=(nw, h, s.n_chol))
    hb = 0.1 * (rng.normal(size=(nw, h, s.n_chol)) + 1j * rng.normal(size=(nw, h, s.n_chol)))
    y = 0.7 * rng.normal(size=(nw, P, s.K)) if s.hidden_kind else ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    phi_end = phi_mid.copy()
    for i in range(h):
        phi_end = O.propagate_dets(s, phi_end, hx[:, i], hb[:, i], dtau, 10)
    logov = O.log_overlap(phiT, phi_end)
    w = rng.uniform(0.5, 1.5, size=nw)
    num, den, Rk = O.back_propagated_density(s, phi_mid, hx, hb, phiT, logov, w, dtau, 10)
    ctx = A.Context(s, P, dtau, max_walkers=nw)
    bp = D.BackProp(ctx, nw, max(h, 1))
    out = torch.zeros(s.M * s.M + 1, dtype=torch.float64, device="cuda")
    A.afqmc_bp_density(ctx, nw, h, dev(phi_mid), dev(hx) if h else None, dev(hb) if h else None,
                       dev(phiT), dev(logov), dev(w), bp.phit_bp, bp.theta_bp, bp.logov_bp, bp.rho,
                       out)
    torch.cuda.synchronize()
    g = host(out)
    assert np.abs(g[:-1].reshape(s.M, s.M) - num).max() <= TOL * np.abs(num).max()
    assert abs(g[-1] - den) <= 1e-14 * den
    assert np.abs(host(bp.rho) - Rk).max() <= TOL * np.abs(Rk).max()
    tr = np.trace(host(bp.rho), axis1=1, axis2=2)
    assert np.abs(tr - 2 * s.N).max() <= 1e-9


@pytest.mark.parametrize("sysname", ["tiny", "itime"])
def test_bp_trajectory_follows_the_comb(sysname):
    """Eight steps, comb every step, a window of h = 4 recorded steps 2..5:
    the density after step 5 equals the oracle's with the same history."""
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    if sysname == "tiny":
        s, kw, okw = ai.tiny_ising(), {}, {}
    else:
        s = ai.imaginary_time_trial(ai.tiny_ising(), 2, 0.05)
        kw = dict(proposal=A.PROPOSAL_RW, rw_step=0.3)
        okw = dict(proposal=O.PROPOSAL_RW, rw_step=0.3)
    nw, P, dtau, seed, h, start = 16, 6, 0.01, 77, 4, 2
    ctx = A.Context(s, P, dtau, max_walkers=nw, **kw)
    st = D.init_walkers(ctx, s.phi0, nw, seed)
    bp = D.BackProp(ctx, nw, h)
    ost = O.init_state(s, nw, P, seed)
    Eh, h1p = O.half_kinetic(s, dtau), O.h1_eff(s)
    est = torch.zeros(2, dtype=torch.float64, device="cuda")
    hx = np.zeros((nw, h, s.n_chol))
    hb = np.zeros((nw, h, s.n_chol), dtype=complex)
    phi_mid = None
    for i in range(start + h):
        if i == start:
            bp.start(st)
            phi_mid = ost.phi.copy()
        D.step(ctx, st, seed, i, est, n_sweep=1, n_qr=3, n_pc=1, w_cap=4.0, bp=bp)
        ost, rec = O.step(s, ost, seed, i, dtau, n_qr=3, Eh=Eh, h1p=h1p, n_pc=1, w_cap=4.0, **okw)
        if i >= start:
            hx[:, i - start] = rec["xi"]
            hb[:, i - start] = rec["xbar"]
            par = rec["parent"]
            hx, hb, phi_mid = hx[par], hb[par], phi_mid[par]
    assert bp.ready
    out = torch.zeros(s.M * s.M + 1, dtype=torch.float64, device="cuda")
    bp.density(st, out)
    torch.cuda.synchronize()
    num, den, Rk = O.back_propagated_density(s, phi_mid, hx, hb, ost.phiT, ost.logov, ost.w, dtau,
                                             10, Eh)
    g = host(out)
    _say(sysname, "BP occupations", np.round(np.diag(num) / den, 4))
    assert np.abs(host(bp.hist_xi) - hx).max() <= 4e-15 * np.abs(hx).max()
    assert np.abs(g[:-1].reshape(s.M, s.M) - num).max() <= 1e-9 * np.abs(num).max()
    assert abs(g[-1] - den) <= 1e-9 * den
    assert np.abs(host(bp.rho) - Rk).max() <= 1e-9 * np.abs(Rk).max()


def test_entry_points_reject_bad_arguments_and_accept_empty_calls():
    """Argument errors are reported (AfqmcError), never faults; nw = 0 is a no-op."""
    from paper_2505_18519_amd import afqmc as A
    from paper_2505_18519_amd import driver as D
    s = ai.tiny_ising()
    ctx = A.Context(s, 4, 0.01, max_walkers=4)
    bp = D.BackProp(ctx, 4, 3)
    xi = torch.zeros(4, s.n_chol, dtype=torch.float64, device="cuda")
    xb = torch.zeros(4, s.n_chol, dtype=torch.complex128, device="cuda")
    with pytest.raises(A.AfqmcError):           # slot outside [0, h)
        A.afqmc_bp_record(ctx, 4, 3, 3, xi, xb, bp.hist_xi, bp.hist_xbar)
    with pytest.raises(A.AfqmcError):           # h < 1
        A._check(ctx, A.load_library().afqmc_bp_record(ctx.handle, 4, 0, 0, None, None, None,
                                                        None), "bp_record")
    with pytest.raises(A.AfqmcError):           # negative history length
        A._check(ctx, A.load_library().afqmc_bp_density(ctx.handle, 4, -1, None, None, None, None,
                                                         None, None, None, None, None, None,
                                                         None), "bp_density")
    with pytest.raises(A.AfqmcError):           # p_src < 1
        A._check(ctx, A.load_library().afqmc_extend_paths(ctx.handle, 4, 0, None, None, None,
                                                           None, None, None), "extend_paths")
    with pytest.raises(A.AfqmcError):           # negative copy length
        A._check(ctx, A.load_library().afqmc_copy(ctx.handle, -1, None, None), "copy")
    # empty calls succeed without touching their (absent) arrays
    lib = A.load_library()
    assert lib.afqmc_bp_record(ctx.handle, 0, 3, 0, None, None, None, None) == 0
    assert lib.afqmc_bp_density(ctx.handle, 0, 2, None, None, None, None, None, None, None, None,
                                None, None, None) == 0
    assert lib.afqmc_gather_rows(ctx.handle, 0, None, 8, None, None) == 0
    assert lib.afqmc_gather_rows(ctx.handle, 4, None, 0, None, None) == 0
    assert lib.afqmc_copy(ctx.handle, 0, None, None) == 0
    assert lib.afqmc_init_metropolis(ctx.handle, 0, 1, 2, 2, None, None, None, None, None,
                                     None) == 0
    assert lib.afqmc_extend_paths(ctx.handle, 0, 1, None, None, None, None, None, None) == 0
    # the corrected estimator always writes its two sums, so it needs its arrays even at nw = 0
    assert lib.afqmc_estimator_corrected(ctx.handle, 0, None, None, None, 1, None, None,
                                         None) == 1
    one = torch.ones(8, dtype=torch.float64, device="cuda")
    onec = torch.ones(8, dtype=torch.complex128, device="cuda")
    out = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    A.afqmc_estimator_corrected(ctx, 0, one, onec, onec, 1, onec, out)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), [0.0, 0.0])
    # gather with a parent out of range copies nothing for that row
    src = torch.arange(12, dtype=torch.float64, device="cuda").reshape(4, 3)
    dst = torch.full((4, 3), -1.0, dtype=torch.float64, device="cuda")
    par = torch.tensor([3, 7, -2, 0], dtype=torch.int32, device="cuda")
    A.afqmc_gather_rows(ctx, 4, par, src, dst)
    torch.cuda.synchronize()
    ref = np.array([[9, 10, 11], [-1, -1, -1], [-1, -1, -1], [0, 1, 2]], dtype=float)
    assert np.array_equal(host(dst), ref)
