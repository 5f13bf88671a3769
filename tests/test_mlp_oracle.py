"""Pins of the oracle's learned Metropolis proposal (an extension beside the
paper's prior proposal of Sec. III.A / App. B).

Each check ties the oracle to something other than itself: central finite
differences for the backward pass, scipy's normal density and a sampled
histogram for the proposal density, closed-form Adam steps, the exact
reduction to the prior proposal when the output layer is zero, and a
detailed-balance check of the chain against 2-D quadrature of p_T |O|.
"""
import math

import numpy as np
import pytest
from scipy import stats

import afqmc_inputs as ai
from oracle import afqmc_oracle as O
from oracle import mlp_oracle as ML


def _tiny_net(rng, D=5, H=8, K=3, scale=0.7):
    p = {
        "W1": rng.normal(size=(D, H)) * scale,
        "b1": rng.normal(size=H) * 0.1,
        "W2": rng.normal(size=(H, H)) * scale,
        "b2": rng.normal(size=H) * 0.1,
        "W3": rng.normal(size=(H, 2 * K)) * scale,
        "b3": rng.normal(size=2 * K) * 0.3,
    }
    return p


def test_backward_matches_central_differences():
    """Every parameter's gradient of the masked mean of -log q against
    central differences (step 1e-5), relative 1e-7 of the gradient's scale."""
    rng = np.random.default_rng(3)
    D, H, K, B = 5, 8, 3, 11
    p = _tiny_net(rng, D, H, K)
    z = rng.normal(size=(B, D))
    yp = rng.normal(size=(B, K)) * 1.5
    mask = rng.random(B) < 0.6
    mask[0] = True
    loss, g = ML.loss_and_grad(p, z, yp, mask)
    v0 = ML.flatten(p)
    ga = ML.flatten(g)
    h = 1e-5
    gn = np.zeros_like(v0)
    for i in range(v0.size):
        vp = v0.copy()
        vp[i] += h
        vm = v0.copy()
        vm[i] -= h
        lp, _ = ML.loss_and_grad(ML.unflatten(vp, D, H, K), z, yp, mask)
        lm, _ = ML.loss_and_grad(ML.unflatten(vm, D, H, K), z, yp, mask)
        gn[i] = (lp - lm) / (2 * h)
    assert np.abs(ga - gn).max() < 1e-7 * np.abs(gn).max(), np.abs(ga - gn).max()
    # the loss is the masked mean of -log q
    mu, lv, _ = ML.forward(p, z)
    ref = -np.mean([stats.norm.logpdf(yp[b], mu[b], np.exp(0.5 * lv[b])).sum()
                    for b in range(B) if mask[b]])
    assert abs(loss - ref) < 1e-12 * abs(ref)


def test_log_q_is_the_density_of_the_sampler():
    """log q equals scipy's normal log-density with sd exp(lv/2), and draws
    mu + exp(lv/2) eta follow it (KS test against the same normal)."""
    rng = np.random.default_rng(4)
    mu = rng.normal(size=(6, 2))
    lv = rng.uniform(-3.9, 3.9, size=(6, 2))
    yp = rng.normal(size=(6, 2)) * 2
    ref = stats.norm.logpdf(yp, mu, np.exp(0.5 * lv)).sum(-1)
    assert np.allclose(ML.log_q(mu, lv, yp), ref, rtol=1e-13, atol=1e-13)
    # the oracle's sampler: y' = mu + exp(lv / 2) eta
    eta = rng.normal(size=20000)
    draws = 0.3 + math.exp(0.5 * -1.2) * eta
    lq = ML.log_q(np.full((1, 1), 0.3), np.full((1, 1), -1.2), np.zeros((1, 1)))
    assert abs(lq[0] - stats.norm.logpdf(0.0, 0.3, math.exp(-0.6))) < 1e-13
    assert stats.kstest(draws, stats.norm(0.3, math.exp(-0.6)).cdf).pvalue > 1e-3


def test_output_transform_bounds_and_zero_layer():
    rng = np.random.default_rng(5)
    p = _tiny_net(rng, scale=5.0)
    z = rng.normal(size=(50, 5)) * 3
    mu, lv, _ = ML.forward(p, z)
    assert np.all(np.abs(lv) < ML.LV_MAX)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    mu, lv, _ = ML.forward(p, z)
    assert np.all(mu == z[:, -3:]) and np.all(lv == 0.0)     # mu = y: a random walk


def test_adam_closed_forms():
    """First step moves every coordinate by -lr sign(g) (bias correction);
    a constant gradient keeps moving by -lr g / (|g| + eps) at every step."""
    rng = np.random.default_rng(6)
    p = {"a": rng.normal(size=20)}
    g = {"a": rng.normal(size=20)}
    opt = ML.Adam(p, lr=1e-3)
    p0 = p["a"].copy()
    opt.step(p, g)
    assert np.allclose(p["a"] - p0, -1e-3 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-9, atol=0)
    for _ in range(30):
        p1 = p["a"].copy()
        opt.step(p, g)
        assert np.allclose(p["a"] - p1, -1e-3 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-7, atol=0)


def test_adam_training_fits_a_gaussian():
    """Online training on draws from N(0.7, 0.5^2) drives mu to 0.7 and lv to
    log 0.25 (the minimiser of the expected -log q)."""
    rng = np.random.default_rng(7)
    D, H, K = 3, 16, 1
    p = _tiny_net(rng, D, H, K, scale=0.3)
    opt = ML.Adam(p, lr=3e-3)
    z = np.zeros((256, D))
    for it in range(1500):
        yp = 0.7 + 0.5 * rng.normal(size=(256, 1))
        _, g = ML.loss_and_grad(p, z, yp, np.ones(256, bool))
        opt.step(p, g)
    mu, lv, _ = ML.forward(p, z[:1])
    assert abs(mu[0, 0] - 0.7) < 0.05 and abs(lv[0, 0] - math.log(0.25)) < 0.1, (mu, lv)


def _paths(s, nw, P, seed):
    rng = np.random.default_rng(seed)
    phi = ai.random_walkers(rng, s, nw, spread=0.8)
    y = ai.random_hidden(rng, s, nw, P)
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    ref = np.exp(1j * rng.uniform(-0.3, 0.3, size=nw))
    return phi, y, phiT, logov, ref


def test_zero_output_layer_is_the_random_walk():
    """With W3 = b3 = 0 the network proposes y + sqrt(2) eta: its q ratio is
    1 and the learned step makes the decisions of the oracle's random walk of
    step sqrt(2), over three sweeps."""
    s = ai.small_gaussian(M=10, N=3, n_chol=6, K=5, seed=8)
    phi, y, phiT, logov, ref = _paths(s, 3, 6, 9)
    p = ai.mlp_params(np.random.default_rng(1), s.M, s.K, H=16, last_scale=0.0)
    w = np.ones(3)
    a = O.metropolis(s, phi, y, phiT, logov, ref, w, 11, 4, 3, proposal=O.PROPOSAL_RW,
                     rw_step=math.exp(0.5 * math.log(2.0)))
    b = ML.metropolis_learned(s, phi, y, phiT, logov, ref, w, 11, 4, 3, p)
    assert np.array_equal(a[4], b[4])
    assert a[4].sum() > 0 and a[4].sum() < 3 * 6 * 3
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-15)
    assert np.allclose(a[2], b[2], rtol=0, atol=1e-12)
    assert np.array_equal(a[3], b[3])


def _toy():
    """K = 2 Gaussian-hidden toy whose path density p_T |O| is clearly shifted
    from the prior (E y_2 = 0.85, E y_2^2 = 1.8 by quadrature)."""
    return ai.gaussian_system(6, 2, 3, 2, seed=4, coupling=0.15, density=0.6)


@pytest.mark.parametrize("rw_step", [0.0, 0.5])
def test_learned_chain_samples_the_path_density(rw_step):
    """Detailed balance of the learned proposal on a K = 2 Gaussian toy with a
    state-dependent network (alone, or cycled with random-walk moves): the
    chains' mean and second moments of y match quadrature of
    p_T(y) |O(y; phi)| (Eq. PDF-Y)."""
    s = _toy()
    rng = np.random.default_rng(2)
    phi = ai.random_walkers(rng, s, 1, spread=0.8)
    P = 160
    p = ai.mlp_params(np.random.default_rng(3), s.M, s.K, H=12, last_scale=1.5)
    p["b3"][2:] = 0.4          # proposals wider than the prior
    y = rng.normal(size=(1, P, 2))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    acc, nacc = [], 0
    for st in range(260):
        y, phiT, logov, _, na, _ = ML.metropolis_learned(s, phi, y, phiT, logov, np.ones(1, complex),
                                                         np.ones(1), 5, st, 1, p, rw_step=rw_step)
        if st >= 20:
            acc.append(y[0].copy())
            nacc += na[0]
    assert 0.1 < nacc / (240 * P * (2 if rw_step else 1)) < 0.95
    samp = np.stack(acc)                         # [T, P, 2]
    g = np.linspace(-7, 7, 141)
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    lo = O.log_overlap(O.trial_det(s, Y[None]), phi)[0]
    dens = np.exp(lo.real - lo.real.max() - 0.5 * (Y * Y).sum(-1))
    dens /= dens.sum()
    feats = lambda v: np.concatenate([v, v * v, v[..., :1] * v[..., 1:]], -1)
    ref = (dens[:, None] * feats(Y)).sum(0)
    per_chain = feats(samp).mean(0)              # chains are independent
    err = per_chain.std(0, ddof=1) / math.sqrt(P)
    z = (per_chain.mean(0) - ref) / err
    assert np.abs(z).max() < 5.0, z


def test_learned_chain_with_the_reverse_density_at_the_wrong_state_is_biased():
    """The detailed-balance check above has the power to see a wrong q ratio:
    evaluating the reverse density with the current state's features instead
    of the proposal's biases the sampled moments well beyond 5 sigma."""
    s = _toy()
    rng = np.random.default_rng(2)
    phi = ai.random_walkers(rng, s, 1, spread=0.8)
    P = 160
    p = ai.mlp_params(np.random.default_rng(3), s.M, s.K, H=12, last_scale=1.5)
    p["b3"][2:] = 0.4
    y = rng.normal(size=(1, P, 2))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    from oracle import philox
    samples = []
    for st in range(260):
        _, gd = ML.green_diag(phiT, phi)
        z = ML.features(gd, y).reshape(P, -1)
        mu, lv, _ = ML.forward(p, z)
        eta = philox.proposal_normals(5, st, 1, P, 2, 0).reshape(P, 2)
        yp = mu + np.exp(0.5 * lv) * eta
        lq_f = ML.log_q(mu, lv, yp)
        lq_r = ML.log_q(mu, lv, y.reshape(P, 2))        # planted mistake: z instead of z'
        ypr = yp.reshape(1, P, 2)
        phiTp = O.trial_det(s, ypr)
        ellp = O.log_overlap(phiTp, phi)
        u = philox.accept_uniforms(5, st, 1, P, 1, 0)[:, :, 0]
        la = (ellp.real - logov.real - 0.5 * (ypr * ypr).sum(-1) + 0.5 * (y * y).sum(-1)
              + (lq_r - lq_f).reshape(1, P))
        a = O._accept(u, la)
        y = np.where(a[..., None], ypr, y)
        phiT = np.where(a[..., None, None], phiTp, phiT)
        logov = np.where(a, ellp, logov)
        if st >= 20:
            samples.append(y[0].copy())
    samp = np.stack(samples)
    g = np.linspace(-7, 7, 141)
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    lo = O.log_overlap(O.trial_det(s, Y[None]), phi)[0]
    dens = np.exp(lo.real - lo.real.max() - 0.5 * (Y * Y).sum(-1))
    dens /= dens.sum()
    feats = lambda v: np.concatenate([v, v * v, v[..., :1] * v[..., 1:]], -1)
    ref = (dens[:, None] * feats(Y)).sum(0)
    per_chain = feats(samp).mean(0)
    err = per_chain.std(0, ddof=1) / math.sqrt(P)
    z = (per_chain.mean(0) - ref) / err
    assert np.abs(z).max() > 5.0, z


def test_training_learns_the_denoiser_of_the_path_density():
    """Denoising score matching on the random-walk moves at a fixed walker:
    the trained network's mean at a noisy point y~ approaches E[y | y~] and
    exp(lv) approaches Var[y | y~] of p_T(y) |O(y; phi)| smoothed by
    N(0, s^2) (both by 2-D quadrature) -- Tweedie's formula, the learned
    Langevin drift."""
    s = _toy()
    rng = np.random.default_rng(12)
    phi = ai.random_walkers(rng, s, 1, spread=0.8)
    P, sig = 64, 0.8
    p = ai.mlp_params(np.random.default_rng(13), s.M, s.K, H=16, last_scale=0.0)
    p["b3"][2:] = 4 * math.atanh(math.log(sig * sig) / 4)      # start as the walk of step sig
    opt = ML.Adam(p, lr=1e-2)
    y = rng.normal(size=(1, P, 2))
    phiT = O.trial_det(s, y)
    logov = O.log_overlap(phiT, phi)
    for st in range(400):
        if st == 250:
            opt.lr = 2e-3
        y, phiT, logov, _, _, loss = ML.metropolis_learned(
            s, phi, y, phiT, logov, np.ones(1, complex), np.ones(1), 21, st, 1, p, adam=opt,
            rw_step=sig)
    # probe points from the smoothed density: chain states plus N(0, sig^2)
    yt = y + sig * rng.normal(size=y.shape)
    _, gd = ML.green_diag(O.trial_det(s, yt), phi)
    mu, lv, _ = ML.forward(p, ML.features(gd, yt).reshape(P, -1))
    g = np.linspace(-7, 7, 141)
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    lo = O.log_overlap(O.trial_det(s, Y[None]), phi)[0]
    dens = np.exp(lo.real - lo.real.max() - 0.5 * (Y * Y).sum(-1))
    ker = np.exp(-0.5 * ((yt[0][:, None, :] - Y[None]) ** 2).sum(-1) / sig**2) * dens[None]
    ker /= ker.sum(1, keepdims=True)
    m_ref = ker @ Y                                              # E[y | y~]
    v_ref = ker @ (Y * Y) - m_ref**2                             # Var[y | y~]
    drift = np.abs(m_ref - yt[0]).mean()
    err = np.abs(mu - m_ref).mean()
    assert err < 0.2 * drift, (err, drift)
    assert np.abs(np.exp(lv).mean(0) / v_ref.mean(0) - 1).max() < 0.2, (np.exp(lv).mean(0),
                                                                      v_ref.mean(0))
