"""One AFQMC step with a sampled trial, in the order of App. B, through the C ABI.

Holds the composite-walker state (Sec. III.A, Fig. 2): walker determinants and
weights, the P tethered paths y with their trial determinants Phi_T(y) and
log-overlaps.  Every arithmetic step runs in libafqmc's kernels; this module
only allocates the state tensors and sequences the calls on one stream.
"""
from __future__ import annotations

import torch

from . import afqmc as A


class Walkers:
    """Device state of nw composite walkers plus per-step scratch outputs."""

    def __init__(self, ctx: A.Context, nw: int):
        c, dev = ctx, ctx.device
        self.nw = nw
        z = dict(device=dev)
        self.phi = torch.zeros(nw, 2, c.M, c.N, dtype=c.pdtype, **z)
        self.w = torch.ones(nw, dtype=torch.float64, **z)
        self.y = torch.zeros(nw, c.P, c.K, dtype=torch.float64, **z)
        self.phiT = torch.zeros(nw, c.P, c.M, c.N, dtype=c.tdtype, **z)
        self.logov = torch.zeros(nw, c.P, dtype=torch.complex128, **z)
        self.logov_new = torch.zeros(nw, c.P, dtype=torch.complex128, **z)
        self.theta = torch.zeros(nw, c.P, 2, c.M, c.N, dtype=torch.complex128, **z)
        self.xbar = torch.zeros(nw, c.G, dtype=torch.complex128, **z)
        self.eloc = torch.zeros(nw, dtype=torch.complex128, **z)
        self.xi = torch.zeros(nw, c.G, dtype=torch.float64, **z)
        self.ref = torch.zeros(nw, dtype=torch.complex128, **z)
        self.nacc = torch.zeros(nw, dtype=torch.int32, **z)
        ctx.reserve(nw)


def init_walkers(ctx: A.Context, phi0, nw: int, seed: int) -> Walkers:
    """phi = Phi_0 for both spins, W = 1, y ~ p_T, Phi_T(y) and l(y; phi)."""
    st = Walkers(ctx, nw)
    p0 = torch.as_tensor(phi0, dtype=ctx.pdtype, device=ctx.device)
    st.phi.copy_(p0.expand(nw, 2, ctx.M, ctx.N))
    A.afqmc_sample_prior(ctx, nw, seed, st.y)
    A.afqmc_trial_build(ctx, nw, st.y, st.phiT)
    A.afqmc_overlap(ctx, nw, st.phi, st.phiT, st.logov)
    return st


class BackProp:
    """Field history and saved walkers of a back-propagated measurement (App.
    B, Measurement): start() saves the walkers, the next h steps record their
    fields (step(..., bp=...)), and the history follows the walkers through
    every comb; after the h-th step, density() gives the back-propagated
    one-body density matrix."""

    def __init__(self, ctx: A.Context, nw: int, h: int):
        c, z = ctx, dict(device=ctx.device)
        self.ctx, self.nw, self.h = ctx, nw, h
        c128, f64 = torch.complex128, torch.float64
        self.hist_xi = torch.zeros(nw, h, c.G, dtype=f64, **z)
        self.hist_xbar = torch.zeros(nw, h, c.G, dtype=c128, **z)
        self.phi_mid = torch.zeros(nw, 2, c.M, c.N, dtype=c128, **z)
        self._spare = [torch.zeros_like(self.hist_xi), torch.zeros_like(self.hist_xbar),
                       torch.zeros_like(self.phi_mid)]
        self.phit_bp = torch.zeros(nw, c.P, c.M, c.N, dtype=c128, **z)
        self.theta_bp = torch.zeros(nw, c.P, 2, c.M, c.N, dtype=c128, **z)
        self.logov_bp = torch.zeros(nw, c.P, dtype=c128, **z)
        self.rho = torch.zeros(nw, c.M, c.M, dtype=c128, **z)
        self.parent = torch.zeros(nw, dtype=torch.int32, **z)
        self.slot = -1

    @property
    def recording(self) -> bool:
        return 0 <= self.slot < self.h

    @property
    def ready(self) -> bool:
        return self.slot == self.h

    def start(self, st: Walkers) -> None:
        A.afqmc_copy(self.ctx, st.phi, self.phi_mid)
        self.slot = 0

    def record(self, st: Walkers) -> None:
        A.afqmc_bp_record(self.ctx, st.nw, self.h, self.slot, st.xi, st.xbar, self.hist_xi,
                          self.hist_xbar)
        self.slot += 1

    def follow(self, nw: int) -> None:
        """Move the history and saved walkers with the comb's parents."""
        bufs = [self.hist_xi, self.hist_xbar, self.phi_mid]
        for src, dst in zip(bufs, self._spare):
            A.afqmc_gather_rows(self.ctx, nw, self.parent, src, dst)
        self.hist_xi, self.hist_xbar, self.phi_mid, self._spare = (
            self._spare[0], self._spare[1], self._spare[2], bufs)

    def density(self, st: Walkers, out: torch.Tensor) -> None:
        """out: device float64 [M*M + 1] = (sum W Re R_k (row-major), sum W)."""
        A.afqmc_bp_density(self.ctx, st.nw, self.h, self.phi_mid, self.hist_xi, self.hist_xbar,
                           st.phiT, st.logov, st.w, self.phit_bp, self.theta_bp, self.logov_bp,
                           self.rho, out)


def step(ctx: A.Context, st: Walkers, seed: int, i: int, est_out: torch.Tensor,
         e_shift: float = 0.0, n_sweep: int = 1, n_qr: int = 10, contract_events=None,
         n_pc: int = 0, w_cap: float = 0.0, normalize: bool = True,
         bp: "BackProp | None" = None) -> None:
    """Measure, propagate, move the paths, hand off, re-orthonormalise, and
    every n_pc steps (if n_pc > 0) comb the population (weights reset to 1
    with normalize, to their mean otherwise).  With bp recording, the step's
    fields join its history and the comb moves the history with the walkers.

    est_out: device float64 [2] receiving (sum W Re E_L, sum W) at the
    pre-move state (Eq. mixed_estimator).  contract_events, if given, is a
    pair of torch.cuda.Event recorded on the current stream around the
    Cholesky contraction (afqmc_local_energy).
    """
    nw = st.nw
    A.afqmc_green(ctx, nw, st.phi, st.phiT, st.logov, st.theta)
    if contract_events is not None:
        contract_events[0].record()
    A.afqmc_local_energy(ctx, nw, st.phiT, st.theta, st.logov, st.eloc, None, st.xbar)
    if contract_events is not None:
        contract_events[1].record()
    A.afqmc_estimator(ctx, nw, st.w, st.eloc, est_out)
    A.afqmc_philox_normal(ctx, seed, i, A.TAG_FIELD, nw, ctx.G, st.xi)
    A.afqmc_propagate(ctx, nw, st.phi, st.xi, st.xbar, st.phiT, st.logov, e_shift, st.w,
                      st.ref, st.logov_new, st.eloc)
    following = bp is not None and bp.recording
    if following:
        bp.record(st)
    A.afqmc_metropolis_x(ctx, nw, st.phi, st.y, st.phiT, st.logov_new, st.ref, st.w, seed, i,
                         n_sweep, st.nacc)
    st.logov, st.logov_new = st.logov_new, st.logov
    if n_qr and (i + 1) % n_qr == 0:
        A.afqmc_reorthogonalize(ctx, nw, st.phi, st.logov)
    if n_pc and (i + 1) % n_pc == 0:
        A.afqmc_population_control(ctx, nw, st.phi, st.w, st.y, st.phiT, st.logov, seed, i, w_cap,
                                   parent=bp.parent if following else None, normalize=normalize)
        if following:
            bp.follow(nw)


def init_walkers_metropolis(ctx: A.Context, nw: int, seed: int, n_pair: int = 10,
                            n_burn: int = 4) -> Walkers:
    """Walkers sampled from the trial (App. B, Initialization): phi^0_k =
    B_T(Y_k) phi_T with P paths each and W^0_k = sum_p S_p, so that the mixed
    estimate at beta = 0 is the Metropolis estimate of the trial's variational
    energy.  st.yw holds the walker fields Y_k."""
    st = Walkers(ctx, nw)
    st.yw = torch.zeros(nw, ctx.K, dtype=torch.float64, device=ctx.device)
    A.afqmc_init_metropolis(ctx, nw, seed, n_pair, n_burn, st.yw, st.phi, st.y, st.phiT,
                            st.logov, st.w)
    return st


class Measurement:
    """Device buffers of a measurement trial with mctx.P paths per walker
    (Sec. III.A, end of the composite-walker part; App. B, Measurement).
    mctx is a context of the same system with the measurement's path count."""

    def __init__(self, mctx: A.Context, nw: int):
        c, z = mctx, dict(device=mctx.device)
        self.ctx, self.nw = mctx, nw
        self.y = torch.zeros(nw, c.P, c.K, dtype=torch.float64, **z)
        self.phiT = torch.zeros(nw, c.P, c.M, c.N, dtype=c.tdtype, **z)
        self.logov = torch.zeros(nw, c.P, dtype=torch.complex128, **z)
        self.theta = torch.zeros(nw, c.P, 2, c.M, c.N, dtype=torch.complex128, **z)
        self.eloc = torch.zeros(nw, dtype=torch.complex128, **z)
        self.R = torch.zeros(nw, dtype=torch.complex128, **z)
        mctx.reserve(nw)


def measure_extra(m: Measurement, st: Walkers, seed: int, i: int, out: torch.Tensor,
                  n_sweep: int = 4) -> None:
    """Mixed estimate at step i with a freshly sampled measurement trial: the
    walkers' paths extended to m.ctx.P, moved n_sweep sweeps at the current
    walkers (Metropolis streams at step MEASURE_STEP + i), the local energy
    over the new paths, and each weight times R_k = sum S' / sum S in both
    sums.  out: device float64 [2] = (sum W Re(R E'_L), sum W Re R).  Leaves
    the walkers' own paths untouched."""
    c, nw, P = m.ctx, st.nw, st.y.shape[1]
    A.afqmc_extend_paths(c, nw, P, st.y, st.phiT, st.logov, m.y, m.phiT, m.logov)
    A.afqmc_metropolis_x(c, nw, st.phi, m.y, m.phiT, m.logov, None, None, seed,
                         A.MEASURE_STEP + i, n_sweep)
    A.afqmc_green(c, nw, st.phi, m.phiT, m.logov, m.theta)
    A.afqmc_local_energy(c, nw, m.phiT, m.theta, m.logov, m.eloc, None, None)
    A.afqmc_estimator_corrected(c, nw, st.w, m.eloc, m.logov, P, st.logov, out, m.R)


class EnergyReference:
    """Trial energy E_T of a long run and the local-energy cap around it.

    Steps 0..19 run without the cap and with E_T = 0.  After step 19, and
    after every step i with (i + 1) % 100 == 0 from step 99 on, E_T becomes
    the mixed estimate over the last (at most) 100 steps, sum num / sum den
    of est[max(0, i - 99) .. i]; from then on the context clips Re E_L to
    E_T +- width (afqmc_set_eloc_cap; width = sqrt(2 / tau) by default, the
    usual phaseless-AFQMC cap) and e_shift = E_T enters the weights.  The
    schedule reads the estimator sums back to the host only at those steps.
    """

    def __init__(self, ctx: A.Context, width: "float | None" = None):
        import math
        self.ctx = ctx
        self.width = math.sqrt(2.0 / ctx.dtau) if width is None else float(width)
        self.e_t = None

    @property
    def e_shift(self) -> float:
        return 0.0 if self.e_t is None else self.e_t

    def attach(self, ctx: A.Context) -> None:
        """Carry E_T and the cap over to another context of the same run."""
        self.ctx = ctx
        if self.e_t is not None:
            A.afqmc_set_eloc_cap(ctx, self.e_t, self.width)

    def update(self, i: int, est: torch.Tensor) -> None:
        """After step i; est: device float64 [>= i + 1, 2] of the run's sums."""
        if not (i == 19 or (i >= 99 and (i + 1) % 100 == 0)):
            return
        seg = est[max(0, i - 99):i + 1].sum(0).cpu()
        num, den = float(seg[0]), float(seg[1])
        if den > 0.0 and num == num:
            self.e_t = num / den
            A.afqmc_set_eloc_cap(self.ctx, self.e_t, self.width)
