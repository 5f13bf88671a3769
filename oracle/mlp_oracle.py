"""FP64 oracle of the learned Metropolis proposal for the hidden variables.

TEST INFRASTRUCTURE ONLY (tests/, the smoke check, the benchmark's CPU leg).

Sec. III.A (leapfrog step 2) and App. B move the hidden variables with
Metropolis proposals drawn from the prior and leave the proposal open to other
schemes.  This extension (not in the paper) learns a local proposal: a
multilayer perceptron maps the features
z = [Re diag(G_up + G_dn) (M values), y (K values)] of a path at the current
walker to a mean and a log-variance,
  h1 = tanh(z W1 + b1), h2 = tanh(h1 W2 + b2), o = h2 W3 + b3,
  mu = y + o[:K]  (a displacement from the current state),
  lv = LV_MAX tanh(o[K:] / LV_MAX),
and proposes from the diagonal Gaussian q(y' | z) = N(mu, 2 diag exp(lv)).
Acceptance is exact Metropolis-Hastings with the reverse density evaluated at
the proposal's own features:
  log alpha = Re l(y') - Re l(y) - |y'|^2/2 + |y|^2/2 + log q(y | z') - log q(y' | z).
Training is denoising score matching on the random-walk moves the chains
already make: for a state y and its proposal y~ = y + s eta, Adam (lr 1e-3,
betas 0.9 / 0.999, eps 1e-8) lowers -log q(y | z(y~)), whose minimiser has
mu(y~) = E[y | y~] = y~ + s^2 grad log p_s(y~) (Tweedie's formula, p_s the
path density smoothed by N(0, s^2)) and exp(lv) = Var[y | y~] ~ s^2.  The
proposal N(mu(y), 2 exp(lv)) is then the Langevin step y + (h/2) grad log p +
sqrt(h) eta with h = 2 s^2: the factor 2 pairs the denoiser's drift with the
noise that belongs to it.  With a zero output layer (W3 = b3 = 0) the
proposal is the random walk of step sqrt(2).

Parameters are a dict of float64 arrays W1 [D,H], b1 [H], W2 [H,H], b2 [H],
W3 [H,2K], b3 [2K]; flattened in that order for the C ABI.
"""
from __future__ import annotations

import math

import numpy as np

from . import afqmc_oracle as O
from . import philox

LV_MAX = 4.0
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(p):
    return np.concatenate([p[k].ravel() for k in PARAM_ORDER])


def unflatten(v, D, H, K):
    shapes = {"W1": (D, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, 2 * K), "b3": (2 * K,)}
    out, off = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.array(v[off:off + n]).reshape(shapes[k])
        off += n
    return out


def forward(p, z):
    """(mu, lv, cache) for features z [B, D]."""
    a1 = z @ p["W1"] + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.tanh(a2)
    o = h2 @ p["W3"] + p["b3"]
    K = o.shape[1] // 2
    mu = z[:, -K:] + o[:, :K]
    t = np.tanh(o[:, K:] / LV_MAX)
    lv = LV_MAX * t
    return mu, lv, (z, h1, h2, t)


LOG2 = math.log(2.0)


def log_q(mu, lv, yp):
    """log N(yp; mu, diag exp(lv)) per row."""
    d = yp - mu
    return (-0.5 * lv - 0.5 * d * d * np.exp(-lv) - 0.5 * math.log(2 * math.pi)).sum(-1)


def loss_and_grad(p, z, yp, mask):
    """Mean over masked rows of -log q(yp | z) and its gradient w.r.t. p
    (mu depends on the parameters through o[:K] only)."""
    mu, lv, (z, h1, h2, t) = forward(p, z)
    m = np.asarray(mask, dtype=np.float64)
    n = m.sum()
    if n == 0:
        return 0.0, {k: np.zeros_like(v) for k, v in p.items()}
    lq = log_q(mu, lv, yp)
    loss = -(m * lq).sum() / n
    d = yp - mu
    e = np.exp(-lv)
    g_mu = -(d * e)                       # d(-log q)/d mu
    g_lv = 0.5 - 0.5 * d * d * e          # d(-log q)/d lv
    g_olv = g_lv * (1.0 - t * t)          # through lv = LV_MAX tanh(o / LV_MAX)
    dO = np.concatenate([g_mu, g_olv], axis=1) * (m / n)[:, None]
    g = {}
    g["W3"] = h2.T @ dO
    g["b3"] = dO.sum(0)
    dh2 = (dO @ p["W3"].T) * (1.0 - h2 * h2)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"].T) * (1.0 - h1 * h1)
    g["W1"] = z.T @ dh1
    g["b1"] = dh1.sum(0)
    return loss, g


class Adam:
    def __init__(self, p, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in p.items()}
        self.v = {k: np.zeros_like(v) for k, v in p.items()}
        self.t = 0

    def step(self, p, g):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in p:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g[k] * g[k]
            p[k] = p[k] - self.lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps)


def green_diag(phiT, phi):
    """(l, Re diag(G_up + G_dn)) per path: G^s = Theta^s Phi_T^T, so
    G^s_mm = sum_n Theta^s_mn Phi_T,mn; a singular path gives zeros.  [nw, P, M]."""
    ell, theta = O.green(phiT, phi)
    gd = np.einsum("wpsmn,wpmn->wpm", theta, phiT.astype(np.complex128))
    return ell, gd.real


def features(gdiag, y):
    return np.concatenate([gdiag, y], axis=-1)


def metropolis_learned(sys, phi, y, phiT, logov, ref, w, seed, step, n_sweep, params,
                       weight_mode=O.WEIGHT_SEPARATE, adam=None, trace=None, rw_step=0.0):
    """Learned-proposal Metropolis update of the paths, then the hand-off.

    One network move per path: z = features at (phi, y); draw
    y' = mu + sqrt(2 exp(lv)) eta with eta from the PROPOSAL stream; Phi_T(y'),
    l(y') and z' = features at (phi, y'); accept iff u < alpha (ACCEPT stream).
    With rw_step > 0 each sweep s is a random-walk move y~ = y + rw_step eta
    (stream sweep index 2s; accepted with |O(y~)| N(y~) / (|O(y)| N(y)))
    followed by the network move (index 2s + 1), a cycle of two exact
    kernels; otherwise the network move uses index s.

    Training (an Adam optimiser given; needs rw_step > 0): in every sweep,
    between the random-walk proposal and its accept test, one Adam step on the
    mean over all paths of -log q(y | z(y~)) (denoising score matching).

    Returns (y', phiT', logov', w', n_accept (both kinds of move), last loss).
    A list passed as `trace` receives (log alpha, u) of every network move.
    """
    y = y.copy()
    phiT = phiT.copy()
    logov = logov.copy()
    nw, P, K = y.shape
    if adam is not None and not rw_step > 0.0:
        raise ValueError("training uses the random-walk moves: needs rw_step > 0")
    nacc = np.zeros(nw, dtype=np.int64)
    loss = 0.0
    for s in range(n_sweep):
        sl = s
        if rw_step > 0.0:
            eta = philox.proposal_normals(seed, step, nw, P, K, 2 * s)
            u = philox.accept_uniforms(seed, step, nw, P, 1, 2 * s)[:, :, 0]
            yt = y + rw_step * eta
            phiTt = O.trial_det(sys, yt)
            ellt, gdt = green_diag(phiTt, phi)
            if adam is not None:
                zt = features(gdt, yt).reshape(nw * P, -1)
                loss, g = loss_and_grad(params, zt, y.reshape(nw * P, K), np.ones(nw * P, bool))
                adam.step(params, g)
            acc = O._accept(u, ellt.real - logov.real - 0.5 * (yt * yt).sum(-1)
                            + 0.5 * (y * y).sum(-1))
            y = np.where(acc[..., None], yt, y)
            phiT = np.where(acc[..., None, None], phiTt, phiT)
            logov = np.where(acc, ellt, logov)
            nacc += acc.sum(-1)
            sl = 2 * s + 1
        _, gd = green_diag(phiT, phi)
        z = features(gd, y).reshape(nw * P, -1)
        mu, lv, _ = forward(params, z)
        lvq = lv + LOG2                                  # proposal variance 2 exp(lv)
        eta = philox.proposal_normals(seed, step, nw, P, K, sl).reshape(nw * P, K)
        yp = mu + np.exp(0.5 * lvq) * eta
        lq_f = log_q(mu, lvq, yp)
        ypr = yp.reshape(nw, P, K)
        phiTp = O.trial_det(sys, ypr)
        ellp, gdp = green_diag(phiTp, phi)
        zp = features(gdp, ypr).reshape(nw * P, -1)
        mup, lvp, _ = forward(params, zp)
        lq_r = log_q(mup, lvp + LOG2, y.reshape(nw * P, K))
        u = philox.accept_uniforms(seed, step, nw, P, 1, sl)[:, :, 0]
        la = (ellp.real - logov.real - 0.5 * (ypr * ypr).sum(-1) + 0.5 * (y * y).sum(-1)
              + (lq_r - lq_f).reshape(nw, P))
        acc = O._accept(u, la)
        if trace is not None:
            trace.append((la.copy(), u.copy()))
        y = np.where(acc[..., None], ypr, y)
        phiT = np.where(acc[..., None, None], phiTp, phiT)
        logov = np.where(acc, ellp, logov)
        nacc += acc.sum(-1)
    w = O.handoff(w, logov, ref, weight_mode)
    return y, phiT, logov, w, nacc, loss
