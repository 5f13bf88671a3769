"""Plain FP64 / complex128 CPU oracle of one AFQMC step with a sampled trial.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.  It
shares no code with the HIP library: the only common import is the seeded
input generator (afqmc_inputs), which holds none of the method's arithmetic.

Each function follows the paper's statement of the method, in its order and
notation, with numpy's matmul / slogdet / solve / eigh / qr as library steps:

* Sec. II.A, Eqs. H and H_MC: H = sum_s h1 + 1/2 sum_g L_g^2 (the Monte-Carlo
  form taken as the definition, not normal-ordered).
* Sec. II.A, Eqs. HS-V and HS: B(x) = e^{-tau T/2} exp(i sqrt(tau) sum_g x_g L_g)
  e^{-tau T/2}; the factor i is the sqrt(-tau) of Eq. HS-V with real L.
* Sec. II.B, Eqs. walker_prop, importance_function, shift1 and
  importance_function_CP: force-bias shift, hybrid weight, phaseless cosine.
* Sec. II.C, Eq. trial_decomp; Sec. III.A, Eq. Metropolis_sampled_trial: the
  sampled trial determinant Phi_T(y) = exp(c sum_k y_k A_k) Phi_0.
* Sec. III.A, Eqs. ratio-update-phi, sign-path, local-obs: overlap-ratio and
  local-observable estimators over the P tethered paths.
* Sec. III.A, Eqs. AFQMC_Metro_correction, AFQMC_Metro_constraint_cos and
  App. B (propagation pseudo-code): Metropolis update of the paths and the
  hand-off cosine projection.

Array conventions (C order): phi [nw, 2, M, N] complex, y [nw, P, K] float,
phiT [nw, P, M, N] float, logov [nw, P] complex (log-overlap, summed over the
two spins; -inf for a singular overlap), theta [nw, P, 2, M, N] complex.

Readings of points the paper leaves open (each is listed in the design notes):
the energy shift factor exp(tau E_T) in the weight; a fixed-order Taylor
series for exp(V) in the walker propagator (both sides compute that same
map); exact exp(U) by eigendecomposition for the trial determinant; the
frozen normaliser 1/|O_p(phi)| of Eq. Metropolis_sampled_trial taken at the
pre-move walker; only the phase of the hand-off ratio R applied to W.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import philox

WEIGHT_SEPARATE = 0   # App. B: cosine of Delta-theta, then cosine of Delta-theta_T
WEIGHT_COMBINED = 1   # one cosine of the summed angle (Sec. III.A, after Eq. AFQMC_Metro_constraint_cos)
WEIGHT_HALFPLANE = 2  # hand-off by the half-plane rule instead of the cosine
WEIGHT_LOCAL = 3      # local-energy formalism: |I| = exp(-tau (Re E_L - E_T)) (Sec. III.A)

PROPOSAL_PRIOR = 0    # independence sampler from p_T (App. B); Ising: single-spin-flip sweep
PROPOSAL_RW = 1       # Gaussian random walk y' = y + s eta


# ---------------------------------------------------------------------------
# Derived one-body matrices

def h1_eff(sys) -> np.ndarray:
    """h1' = h1 + 1/2 sum_g L_g L_g: the one-body part of <1/2 sum_g L_g^2>."""
    return sys.h1 + 0.5 * np.einsum("gij,gjk->ik", sys.L, sys.L)


def exp_sym(Msym: np.ndarray) -> np.ndarray:
    """exp of a real symmetric matrix by eigendecomposition."""
    lam, Q = np.linalg.eigh(Msym)
    return (Q * np.exp(lam)) @ Q.T


def half_kinetic(sys, dtau: float) -> np.ndarray:
    """e^{-tau h1 / 2}: the split one-body factor of B(x) (Eq. HS)."""
    return exp_sym(-0.5 * dtau * sys.h1)


# ---------------------------------------------------------------------------
# Sampled trial determinant (Eq. trial_decomp / Metropolis_sampled_trial)

TRIAL_JASTROW = 0
TRIAL_SLICES = 1


def trial_det(sys, y: np.ndarray) -> np.ndarray:
    """Phi_T(y) = exp(c sum_k y_k A_k) Phi_0 for y [..., K] -> [..., M, N] float,
    or the multi-slice determinant (trial_det_slices, complex)."""
    if getattr(sys, "trial_kind", TRIAL_JASTROW) == TRIAL_SLICES:
        return trial_det_slices(sys, y)
    y = np.asarray(y, dtype=np.float64)
    U = sys.coupling * np.einsum("...k,kij->...ij", y, sys.A)
    lam, Q = np.linalg.eigh(U)
    QtPhi = np.swapaxes(Q, -1, -2) @ sys.phi0
    return (Q * np.exp(lam)[..., None, :]) @ QtPhi


def trial_det_slices(sys, y: np.ndarray) -> np.ndarray:
    """Multi-slice trial determinant (Sec. II.C, Eqs. trial and trial-AF;
    Sec. III.B; the single-slice VAFQMC form of Eq. VAFQMC is m = 1):
    the bra <phi_T| prod_l B_T^l(y^l) overlaps a walker as det(Phi_T(Y)^T phi)
    with Phi_T(Y) = F_m X_m ... F_1 X_1 F_0 Phi_0, where
    X_l = T_n(i sqrt(s_l) sum_k y_{l,k} A_k) is the same n-term Taylor map as
    the walker propagator and F_l are the trial's real one-body factors.
    y [..., m * K_gen] -> [..., M, N] complex; m = 0 gives F_0 Phi_0."""
    y = np.asarray(y, dtype=np.float64)
    lead = y.shape[:-1]
    m = sys.n_slices
    kg = sys.A.shape[0]
    yy = y.reshape(-1, m, kg) if m > 0 else np.zeros((int(np.prod(lead)), 0, kg))
    n = yy.shape[0]
    X0 = (sys.slice_F[0] @ sys.phi0).astype(np.complex128)
    X = np.broadcast_to(X0, (n, sys.M, sys.N)).copy()
    for l in range(m):
        V = 1j * math.sqrt(sys.slice_s[l]) * np.einsum("nk,kij->nij", yy[:, l], sys.A)
        X = taylor_apply(V, X, sys.trial_taylor)
        X = np.einsum("ij,njk->nik", sys.slice_F[l + 1], X)
    return X.reshape(*lead, sys.M, sys.N)


# ---------------------------------------------------------------------------
# Overlap, log-overlap and Green's function (Eqs. ratio-update-phi, sign-path)

def overlap_matrices(phiT: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """A^s = Phi_T^T Phi^s: phiT [nw,P,M,N], phi [nw,2,M,N] -> [nw,P,2,N,N]."""
    return np.einsum("wpmi,wsmj->wpsij", phiT, phi)


def log_overlap(phiT: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """l_p = sum_s log det(Phi_T(y_p)^T Phi^s) [nw, P] complex; -inf if singular."""
    sign, logabs = np.linalg.slogdet(overlap_matrices(phiT, phi))
    sing = np.any(sign == 0, axis=-1)
    ell = logabs.sum(-1) + 1j * np.angle(sign).sum(-1)
    ell = np.where(sing, complex(-np.inf, 0.0), ell)
    return ell


def green(phiT: np.ndarray, phi: np.ndarray):
    """(l, Theta) with Theta^s = Phi^s (Phi_T^T Phi^s)^{-1}; Theta = 0 if singular."""
    A = overlap_matrices(phiT, phi)
    ell = log_overlap(phiT, phi)
    nw, P = ell.shape
    M, N = phi.shape[-2:]
    theta = np.zeros((nw, P, 2, M, N), dtype=np.complex128)
    for w in range(nw):
        for p in range(P):
            if not np.isfinite(ell[w, p].real):
                continue
            for s in range(2):
                # Theta A = Phi  <=>  A^T Theta^T = Phi^T
                theta[w, p, s] = np.linalg.solve(A[w, p, s].T, phi[w, s].T).T
    return ell, theta


def phases(ell: np.ndarray) -> np.ndarray:
    """S_p = O_p / |O_p| (Eq. sign-path); 0 for a singular sample (l = -inf).
    A NaN log-overlap (an overlap matrix with a non-finite entry) gives a NaN
    phase, so the walker's estimates and weight come out non-finite."""
    sing = np.isneginf(ell.real)
    with np.errstate(invalid="ignore"):
        return np.where(sing, 0.0, np.exp(1j * np.where(sing, 0.0, ell.imag)))


# ---------------------------------------------------------------------------
# Per-sample force bias and local energy (Wick's theorem on one determinant pair)

def sample_contraction(sys, phiT: np.ndarray, theta: np.ndarray, ell: np.ndarray,
                       h1p: Optional[np.ndarray] = None):
    """Per-sample vb [nw,P,G] and E_p [nw,P] complex.

    f_g^s = Phi_T^T L_g Theta^s;  vb_g = sum_s tr f_g^s = <L_g> (numerator of
    Eq. shift1 for one path);  E_p = sum_s tr(Phi_T^T h1' Theta^s)
    + 1/2 sum_g [ vb_g^2 - sum_s tr(f_g^s f_g^s) ].
    """
    if h1p is None:
        h1p = h1_eff(sys)
    nw, P = ell.shape
    G = sys.n_chol
    vb = np.zeros((nw, P, G), dtype=np.complex128)
    ep = np.zeros((nw, P), dtype=np.complex128)
    for w in range(nw):
        ok = ~np.isneginf(ell[w].real)
        # Phi_T^T L_g [P,G,N,M] and f = Y Theta^s [P,G,2,N,N], both as library
        # products (einsum's BLAS path, batched matmul)
        Y = np.einsum("pmi,gmn->pgin", phiT[w], sys.L, optimize=True)
        f = np.matmul(Y[:, :, None], theta[w][:, None])
        trf = np.einsum("pgsii->pgs", f)
        vbw = trf.sum(-1)
        ex = np.einsum("pgsij,pgsji->p", f, f)
        e1 = np.einsum("pmi,mn,psni->p", phiT[w], h1p, theta[w])
        epw = e1 + 0.5 * (vbw ** 2).sum(-1) - 0.5 * ex
        vb[w] = np.where(ok[:, None], vbw, 0.0)
        ep[w] = np.where(ok, epw, 0.0)
    return vb, ep


def walker_estimates(vb: np.ndarray, ep: np.ndarray, ell: np.ndarray, dtau: float,
                     xbar_cap: float = 0.0, eloc_cap=None):
    """Eq. local-obs over the P paths, then Eq. shift1.

    xbar_g = -i sqrt(tau) sum_p S_p vb_pg / sum_p S_p,  E_L = sum_p S_p E_p / sum_p S_p.
    The i comes from reading Eq. HS-V's sqrt(-tau) into the propagator with
    real L_g.  A walker whose phases sum to zero gets xbar = 0 and E_L = 0.
    With xbar_cap > 0 each component's modulus is clipped to xbar_cap (phase
    kept); with eloc_cap = (E_T, d), d > 0, a finite Re E_L is clipped to
    [E_T - d, E_T + d] (Im E_L kept).  Both are stabilisations outside the
    paper (the usual phaseless-AFQMC caps), off by default.
    """
    S = phases(ell)
    den = S.sum(-1)
    good = den != 0
    safe = np.where(good, den, 1.0)
    xbar = -1j * math.sqrt(dtau) * np.einsum("wp,wpg->wg", S, vb) / safe[:, None]
    eloc = np.einsum("wp,wp->w", S, ep) / safe
    xbar = np.where(good[:, None], xbar, 0.0)
    eloc = np.where(good, eloc, 0.0)
    if xbar_cap > 0.0:
        mag = np.abs(xbar)
        xbar = np.where(mag > xbar_cap, xbar * (xbar_cap / np.where(mag > 0, mag, 1.0)), xbar)
    if eloc_cap is not None and eloc_cap[1] > 0.0:
        lo, hi = eloc_cap[0] - eloc_cap[1], eloc_cap[0] + eloc_cap[1]
        fin = np.isfinite(eloc.real) & np.isfinite(eloc.imag)
        eloc = np.where(fin, np.minimum(np.maximum(eloc.real, lo), hi) + 1j * eloc.imag, eloc)
    return xbar, eloc


def local_energy(sys, phi, phiT, dtau):
    """(E_L [nw], xbar [nw,G], E_p [nw,P], vb [nw,P,G], logov [nw,P])."""
    ell, theta = green(phiT, phi)
    vb, ep = sample_contraction(sys, phiT, theta, ell)
    xbar, eloc = walker_estimates(vb, ep, ell, dtau)
    return eloc, xbar, ep, vb, ell


# ---------------------------------------------------------------------------
# Propagation (Eqs. HS, walker_prop) and hybrid phaseless weight

def taylor_apply(V: np.ndarray, X: np.ndarray, order: int) -> np.ndarray:
    """sum_{j=0}^{order} V^j X / j!  (V [nw,M,M], X [nw,...,M,N])."""
    out = X.copy()
    term = X.copy()
    for j in range(1, order + 1):
        term = np.einsum("wik,w...kn->w...in", V, term) / j
        out = out + term
    return out


def field_matrix(sys, xi: np.ndarray, xbar: np.ndarray, dtau: float) -> np.ndarray:
    """V = i sqrt(tau) sum_g (xi_g - xbar_g) L_g  -> [nw, M, M] complex."""
    c = xi.astype(np.complex128) - xbar
    return 1j * math.sqrt(dtau) * np.einsum("wg,gij->wij", c, sys.L)


def propagate_dets(sys, phi, xi, xbar, dtau, n_taylor, Eh=None):
    """phi' = e^{-tau h1/2} T_n(V) e^{-tau h1/2} phi (both spins)."""
    if Eh is None:
        Eh = half_kinetic(sys, dtau)
    V = field_matrix(sys, xi, xbar, dtau)
    X = np.einsum("ij,wsjn->wsin", Eh, phi)
    X = taylor_apply(V, X, n_taylor)
    return np.einsum("ij,wsjn->wsin", Eh, X)


def propagate(sys, phi, xi, xbar, phiT, logov, w, dtau, n_taylor,
              e_shift=0.0, weight_mode=WEIGHT_SEPARATE, Eh=None, eloc=None):
    """One walker move with the phaseless weight (App. B, step 1): the hybrid
    |I| = |exp(sum (xi xbar - xbar^2/2)) r| e^{tau E_T} (Eq. importance_function
    with the overlap ratio), or in the local-energy formalism (mode
    WEIGHT_LOCAL, Sec. III.A after Eq. importance_function_CP)
    |I| = exp(-tau (Re E_L - E_T)) with E_L = eloc at the pre-move walker;
    both times max(0, cos arg r).

    Returns (phi', w', ref, logov_new) where logov_new is l_p(phi') at the old
    paths, and ref is the phase reference the hand-off uses: the numerator
    num_r = sum_p exp(l'_p - Re l_p) of Eq. ratio-update-phi (separate and
    half-plane modes) or sum_p S_p (combined-angle mode).
    """
    phin = propagate_dets(sys, phi, xi, xbar, dtau, n_taylor, Eh)
    elln = log_overlap(phiT, phin)
    ok = ~np.isneginf(logov.real)
    okn = ~np.isneginf(elln.real) & ok
    with np.errstate(invalid="ignore"):
        diff = np.where(okn, elln, 0.0) - np.where(okn, logov.real, 0.0)
        num_r = np.where(okn, np.exp(diff), 0.0).sum(-1)
    S = phases(logov)
    den = S.sum(-1)
    alive = (den != 0) & (num_r != 0)
    r = np.where(alive, num_r / np.where(alive, den, 1.0), 1.0)
    if weight_mode == WEIGHT_LOCAL:
        mag = np.exp(-dtau * (np.asarray(eloc).real - e_shift))
    else:
        log_i = (xi * xbar - 0.5 * xbar * xbar).sum(-1) + np.log(r)
        mag = np.exp(log_i.real + dtau * e_shift)
    if weight_mode == WEIGHT_COMBINED:
        wn = w * mag
        ref = den
    else:
        wn = w * mag * np.maximum(0.0, np.cos(np.angle(r)))
        ref = num_r
    wn = np.where(alive & np.isfinite(wn), wn, 0.0)   # a non-finite weight kills the walker
    return phin, wn, ref, elln


# ---------------------------------------------------------------------------
# Metropolis update of the tethered paths (App. B, steps 2 and 3)

def metropolis(sys, phi, y, phiT, logov, ref, w, seed, step, n_sweep,
               proposal=PROPOSAL_PRIOR, rw_step=0.5, weight_mode=WEIGHT_SEPARATE, w0=0):
    """Move every path y_p towards P(y; phi) ~ p_T(y) |O(y; phi)| (Eq. PDF-Y).

    Gaussian prior proposal: y' ~ N(0, 1), alpha = |O(y')| / |O(y)|.
    Gaussian random walk: y' = y + s eta, alpha = |O(y')| N(y') / (|O(y)| N(y)).
    Ising: one sweep flips y_0 .. y_{K-1} in turn, alpha = |O(y')| / |O(y)|.
    Accept iff u < alpha.  Then the hand-off projection (Eq.
    AFQMC_Metro_constraint_cos) with Delta-theta_T = arg sum_p S'_p - arg ref.
    Returns (y', phiT', logov', w', n_accept [nw]).  w0: population index of
    the first walker (selects the walkers' random streams).
    """
    y = y.copy()
    phiT = phiT.copy()
    logov = logov.copy()
    nw, P, K = y.shape
    nacc = np.zeros(nw, dtype=np.int64)
    for s in range(n_sweep):
        if sys.hidden_kind == 0:
            u = philox.accept_uniforms(seed, step, nw, P, K, s, w0)
            for k in range(K):
                yp = y.copy()
                yp[:, :, k] = -yp[:, :, k]
                phiTp = trial_det(sys, yp)
                ellp = log_overlap(phiTp, phi)
                acc = _accept(u[:, :, k], ellp.real - logov.real)
                y = np.where(acc[..., None], yp, y)
                phiT = np.where(acc[..., None, None], phiTp, phiT)
                logov = np.where(acc, ellp, logov)
                nacc += acc.sum(-1)
        else:
            eta = philox.proposal_normals(seed, step, nw, P, K, s, w0)
            u = philox.accept_uniforms(seed, step, nw, P, 1, s, w0)[:, :, 0]
            if proposal == PROPOSAL_RW:
                yp = y + rw_step * eta
                extra = -0.5 * (yp * yp).sum(-1) + 0.5 * (y * y).sum(-1)
            else:
                yp = eta
                extra = 0.0
            phiTp = trial_det(sys, yp)
            ellp = log_overlap(phiTp, phi)
            acc = _accept(u, ellp.real - logov.real + extra)
            y = np.where(acc[..., None], yp, y)
            phiT = np.where(acc[..., None, None], phiTp, phiT)
            logov = np.where(acc, ellp, logov)
            nacc += acc.sum(-1)
    w = handoff(w, logov, ref, weight_mode)
    return y, phiT, logov, w, nacc


def _accept(u: np.ndarray, log_alpha: np.ndarray) -> np.ndarray:
    """u < alpha with alpha = exp(log_alpha); nan (both singular) rejects."""
    with np.errstate(invalid="ignore", over="ignore"):
        la = np.where(np.isnan(log_alpha), -np.inf, log_alpha)
        return (la >= 0.0) | (u < np.exp(np.minimum(la, 0.0)))


def handoff(w, logov_new, ref, weight_mode=WEIGHT_SEPARATE):
    """W <- W max(0, cos Delta-theta_T), Delta-theta_T = arg sum S' - arg ref.
    A non-finite reference or weight gives W = 0, as a non-finite weight
    update does in propagate."""
    Sn = phases(logov_new).sum(-1)
    with np.errstate(invalid="ignore"):
        dth = np.angle(Sn) - np.angle(ref)
        if weight_mode == WEIGHT_HALFPLANE:
            wrapped = np.angle(np.exp(1j * dth))
            fac = np.where(np.abs(wrapped) > 0.5 * np.pi, 0.0, 1.0)
        else:
            fac = np.maximum(0.0, np.cos(dth))
        wn = w * fac
    alive = (Sn != 0) & (ref != 0) & np.isfinite(Sn) & np.isfinite(ref) & np.isfinite(wn)
    return np.where(alive, wn, 0.0)


# ---------------------------------------------------------------------------
# Re-orthogonalisation and estimator

def reorthogonalize(phi: np.ndarray, logov: Optional[np.ndarray] = None):
    """Phi^s = Q R with real positive diag(R); Phi^s <- Q; l_p -= sum log R_ii."""
    nw = phi.shape[0]
    out = np.empty_like(phi)
    shift = np.zeros(nw)
    for w in range(nw):
        for s in range(2):
            Q, R = np.linalg.qr(phi[w, s])
            d = np.diag(R)
            ph = d / np.abs(d)
            out[w, s] = Q * ph[None, :]
            shift[w] += np.log(np.abs(d)).sum()
    if logov is None:
        return out, None
    return out, logov - shift[:, None]


def comb(w: np.ndarray, seed: int, step: int, w_cap: float = 0.0, normalize: bool = False):
    """Comb population control (a standard branching step; the paper is silent).

    With w_cap > 0 every weight is first clipped to w_cap times the mean
    weight.  Then, with u the COMB-stream uniform of this step and C the
    inclusive prefix sums of W, new walker j copies old walker
    parent[j] = min{k : C_k > (j + u) sum(W) / nw} and every new weight is
    sum(W) / nw, or 1 with normalize (a common factor, which cancels in the
    mixed estimator).  Returns (parent, new weights); an all-zero population
    is returned unchanged.
    """
    w = np.asarray(w, dtype=np.float64).copy()
    nw = len(w)
    if w_cap > 0.0:
        w = np.minimum(w, w_cap * w.sum() / nw)
    tot = w.sum()
    if not (tot > 0.0):
        return np.arange(nw), w
    u = philox.stream_uniforms(seed, step, [0], [philox.word3(philox.TAG_COMB)], 1)[0, 0, 0]
    C = np.cumsum(w)
    t = (np.arange(nw) + u) * (tot / nw)
    parent = np.minimum(np.searchsorted(C, t, side="right"), nw - 1)
    return parent, np.full(nw, 1.0 if normalize else tot / nw)


def estimator(w: np.ndarray, eloc: np.ndarray):
    """(sum_k W_k Re E_L,k, sum_k W_k) with exact summation (Eq. mixed_estimator).
    A walker whose Re E_L is not finite (a numerically singular overlap)
    contributes to neither sum; its move then gives it W = 0 (propagate)."""
    ok = np.isfinite(eloc.real)
    wk = np.where(ok, w, 0.0)
    return (math.fsum((wk * np.where(ok, eloc.real, 0.0)).tolist()), math.fsum(wk.tolist()))


# ---------------------------------------------------------------------------
# Initialisation from the trial and measurement with extra paths (App. B,
# Initialization and Measurement; Sec. III.A, end of the composite-walker part)

INIT_STEP = 1 << 63      # step indices INIT_STEP + j belong to the initialisation chains
MEASURE_STEP = 1 << 62   # step indices MEASURE_STEP + i belong to the measurement chains


def as_walker(phiT: np.ndarray) -> np.ndarray:
    """The determinant B_T(Y) phi_T of Eq. Metropolis_sampled_trial as a walker:
    the same real M x N orbitals for both spins, [n, M, N] -> [n, 2, M, N] complex."""
    return np.repeat(phiT[:, None], 2, axis=1).astype(np.complex128)


def init_metropolis(sys, nw, P, seed, n_pair, n_burn, proposal=PROPOSAL_PRIOR, rw_step=0.5):
    """Walkers sampled from the trial (App. B, Initialization; Eq. Metropolis).

    The variational Metropolis estimate of Eq. Metropolis samples pairs
    (Y_k, Y_k') from pi(Y, Y') ~ p_T(Y) p_T(Y') |<phi_T|B_T(Y') B_T(Y)|phi_T>|.
    pi is symmetric and each of its conditionals is the path density of Eq.
    PDF-Y with the other member's B_T(.) phi_T as the walker, so a chain of
    pairs alternates the two conditional Metropolis updates: the partner Y'
    given the walker B_T(Y_k) phi_T, then Y_k given the walker B_T(Y') phi_T.
    After n_pair rounds the walker is phi^0_k = B_T(Y_k) phi_T, each of its P
    paths starts as a copy of the partner (so every pair (Y_k, Y[p]) has the
    law pi whatever follows) and takes n_burn sweeps at that walker to
    decorrelate from the others, and W^0_k = Re sum_p S_p (the sum of the pair
    phases e^{i theta_{p,k}}).  For this trial family the overlaps are squares
    of real determinants, so W^0_k = P.

    Random streams: Y_k and Y' start from the INIT stream with sweeps 1 and 2;
    the chains use the Metropolis streams at steps INIT_STEP + 2j (partner)
    and INIT_STEP + 2j + 1 (walker field), and INIT_STEP + 2 n_pair for the
    paths' sweeps.  Returns (State, yw [nw, K])."""
    if getattr(sys, "trial_kind", TRIAL_JASTROW) != TRIAL_JASTROW:
        raise NotImplementedError("the walker B_T(Y) phi_T is built for the real symmetric "
                                  "trial family only")
    K, kind = sys.K, sys.hidden_kind
    ya = philox.init_hidden(seed, nw, 1, K, kind, sweep=1)
    yb = philox.init_hidden(seed, nw, 1, K, kind, sweep=2)
    pa, pb = trial_det(sys, ya), trial_det(sys, yb)
    one, ref = np.ones(nw), np.ones(nw, dtype=np.complex128)
    for j in range(n_pair):
        wa = as_walker(pa[:, 0])
        yb, pb, _, _, _ = metropolis(sys, wa, yb, pb, log_overlap(pb, wa), ref, one, seed,
                                     INIT_STEP + 2 * j, 1, proposal, rw_step)
        wb = as_walker(pb[:, 0])
        ya, pa, _, _, _ = metropolis(sys, wb, ya, pa, log_overlap(pa, wb), ref, one, seed,
                                     INIT_STEP + 2 * j + 1, 1, proposal, rw_step)
    phi = as_walker(pa[:, 0])
    y = np.repeat(yb, P, axis=1)
    phiT = np.repeat(pb, P, axis=1)
    y, phiT, logov, _, _ = metropolis(sys, phi, y, phiT, log_overlap(phiT, phi), ref, one, seed,
                                      INIT_STEP + 2 * n_pair, n_burn, proposal, rw_step)
    w = phases(logov).sum(-1).real
    return State(phi, w, y, phiT, logov), ya[:, 0]


def extend_paths(y, phiT, logov, P2):
    """The measurement's P2 paths start from the walker's own: path q copies path q mod P."""
    idx = np.arange(P2) % y.shape[1]
    return y[:, idx].copy(), phiT[:, idx].copy(), logov[:, idx].copy()


def measure_extra(sys, phi, y, phiT, logov, w, seed, step, P2, n_sweep, dtau,
                  proposal=PROPOSAL_PRIOR, rw_step=0.5, h1p=None, xbar_cap=0.0):
    """Mixed estimator with a freshly sampled measurement trial (Sec. III.A, end
    of the composite-walker part; App. B, Measurement).

    The walker's P paths are extended to P2 (extend_paths) and moved n_sweep
    sweeps towards p_T |O(.; phi)| at the fixed walker; E'_L is the local
    energy over the new paths (Eq. local-obs); the walker's weight enters
    numerator and denominator of Eq. mixed_estimator times the correction
    factor R_k = sum_q S'_q / sum_p S_p (sign ratios over the new and the
    current paths).  Returns (sum W Re(R E'_L), sum W Re R, E'_L [nw], R [nw]);
    a walker whose current sign sum is 0 has R = 0."""
    y2, phiT2, l2 = extend_paths(y, phiT, logov, P2)
    nw = phi.shape[0]
    y2, phiT2, l2, _, _ = metropolis(sys, phi, y2, phiT2, l2, np.ones(nw, dtype=np.complex128),
                                     np.ones(nw), seed, step, n_sweep, proposal, rw_step)
    ell2, theta2 = green(phiT2, phi)
    vb, ep = sample_contraction(sys, phiT2, theta2, ell2, h1p)
    _, eloc2 = walker_estimates(vb, ep, ell2, dtau, xbar_cap)
    S = phases(logov).sum(-1)
    S2 = phases(ell2).sum(-1)
    R = np.where(S != 0, S2 / np.where(S != 0, S, 1.0), 0.0)
    term = (R * eloc2).real
    ok = np.isfinite(term) & np.isfinite(R.real)   # as in estimator: non-finite walkers drop out
    num = math.fsum(np.where(ok, w * term, 0.0).tolist())
    den = math.fsum(np.where(ok, w * R.real, 0.0).tolist())
    return num, den, eloc2, R


# ---------------------------------------------------------------------------
# Back-propagated one-body density matrix (App. B, Measurement; Eqs.
# AFQMC_Metropolis_measure and AFQMC_Metropolis_measure2)

def back_propagated_density(sys, phi_mid, hist_xi, hist_xbar, phiT, logov, w, dtau, n_taylor,
                            Eh=None):
    """Density matrix with the last h projectors restored: the operator sits
    between the walker phi_mid saved h steps ago and the measurement step's
    trial propagated back through those h steps.

    hist_xi [nw, h, G], hist_xbar [nw, h, G]: the fields of the h steps
    (oldest first) of each walker's line of descent; phiT, logov: the paths
    and log-overlaps at the measurement step; w: the weights there.  With
    B_i = e^{-tau h1/2} T_n(V_i) e^{-tau h1/2} (symmetric), the bra
    <Phi_T(Y_p)| B_h ... B_1 is the determinant Phi~_p = B_1 ... B_h Phi_T(Y_p)
    (B_h applied first), and per path and spin
      R_p^s = phi_mid^s (Phi~_p^T phi_mid^s)^{-1} Phi~_p^T,
      R[i][j] = <Phi~_p| c+_j c_i |phi_mid> / <Phi~_p|phi_mid>;
    the sampled trial of Eq. Metropolis_sampled_trial weights path p by
    a_p = <Phi~_p|phi_mid> / |O_p(phi_end)|, so per walker
      R_k = sum_p a_p (R_p^up + R_p^dn) / sum_p a_p
    (a common factor of the a_p cancels; singular paths drop out).
    Returns (sum_k W_k Re R_k [M, M], sum_k W_k, R_k [nw, M, M])."""
    if Eh is None:
        Eh = half_kinetic(sys, dtau)
    nw, h = hist_xi.shape[:2]
    P = phiT.shape[1]
    X = phiT.astype(np.complex128).copy()                       # [nw, P, M, N]
    for i in range(h - 1, -1, -1):
        V = field_matrix(sys, hist_xi[:, i], hist_xbar[:, i], dtau)
        X = np.einsum("ij,wpjn->wpin", Eh, X)
        X = taylor_apply(V, X, n_taylor)
        X = np.einsum("ij,wpjn->wpin", Eh, X)
    lt, theta = green(X, phi_mid)                                # <Phi~_p|phi_mid>, Theta
    la = np.where(np.isfinite(lt.real) & np.isfinite(logov.real), lt - logov.real, -np.inf)
    shift = np.max(np.where(np.isfinite(la.real), la.real, -np.inf), axis=1, keepdims=True)
    shift = np.where(np.isfinite(shift), shift, 0.0)
    a = np.where(np.isfinite(la.real), np.exp(la - shift), 0.0)  # [nw, P]
    Rk = np.zeros((nw, sys.M, sys.M), dtype=np.complex128)
    for k in range(nw):
        den = a[k].sum()
        if den == 0:
            continue
        for p in range(P):
            if a[k, p] == 0:
                continue
            Rp = sum(theta[k, p, s] @ X[k, p].T for s in range(2))
            Rk[k] += a[k, p] * Rp
        Rk[k] /= den
    ok = np.array([np.all(np.isfinite(Rk[k])) for k in range(nw)]) & (np.abs(a).sum(1) > 0)
    wk = np.where(ok, w, 0.0)
    num = np.einsum("k,kij->ij", wk, np.where(ok[:, None, None], Rk.real, 0.0))
    return num, math.fsum(wk.tolist()), Rk


# ---------------------------------------------------------------------------
# One whole step (App. B order) for trajectory tests

class State:
    def __init__(self, phi, w, y, phiT, logov):
        self.phi, self.w, self.y, self.phiT, self.logov = phi, w, y, phiT, logov

    def copy(self):
        return State(self.phi.copy(), self.w.copy(), self.y.copy(), self.phiT.copy(),
                     self.logov.copy())


def init_state(sys, nw, P, seed):
    """phi = Phi_0 for both spins, W = 1, y ~ p_T (stream INIT)."""
    phi = np.broadcast_to(sys.phi0.astype(np.complex128), (nw, 2, sys.M, sys.N)).copy()
    y = philox.init_hidden(seed, nw, P, sys.K, sys.hidden_kind)
    phiT = trial_det(sys, y)
    logov = log_overlap(phiT, phi)
    return State(phi, np.ones(nw), y, phiT, logov)


def step(sys, st: State, seed, i, dtau, n_taylor=10, n_sweep=1, n_qr=10,
         e_shift=0.0, proposal=PROPOSAL_PRIOR, rw_step=0.5,
         weight_mode=WEIGHT_SEPARATE, Eh=None, h1p=None, xbar_cap=0.0, n_pc=0, w_cap=0.0,
         normalize=True, eloc_cap=None, w0=0):
    """Measure, propagate, move the paths, re-orthogonalise, and (every n_pc
    steps, if n_pc > 0) comb the population (weights reset to 1 with
    normalize).  w0: index of the first walker of st in the population (the
    random streams are per walker index).  Returns (state, record)."""
    ell, theta = green(st.phiT, st.phi)
    vb, ep = sample_contraction(sys, st.phiT, theta, ell, h1p)
    xbar, eloc = walker_estimates(vb, ep, ell, dtau, xbar_cap, eloc_cap)
    num, den = estimator(st.w, eloc)
    xi = philox.field_normals(seed, i, st.phi.shape[0], sys.n_chol, w0)
    phin, wn, ref, elln = propagate(sys, st.phi, xi, xbar, st.phiT, ell, st.w, dtau,
                                    n_taylor, e_shift, weight_mode, Eh, eloc)
    y, phiT, logov, w2, nacc = metropolis(sys, phin, st.y, st.phiT, elln, ref, wn, seed, i,
                                          n_sweep, proposal, rw_step, weight_mode, w0)
    if n_qr and (i + 1) % n_qr == 0:
        phin, logov = reorthogonalize(phin, logov)
    parent = np.arange(st.phi.shape[0])
    if n_pc and (i + 1) % n_pc == 0:
        parent, w2 = comb(w2, seed, i, w_cap, normalize)
        phin, y, phiT, logov = phin[parent], y[parent], phiT[parent], logov[parent]
    rec = dict(e_num=num, e_den=den, eloc=eloc, xbar=xbar, logov=ell, xi=xi,
               w_prop=wn, ref=ref, nacc=nacc, parent=parent)
    return State(phin, w2, y, phiT, logov), rec
