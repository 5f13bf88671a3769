"""Philox4x64-10 counter-based generator and the stream layout of the method.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product path.

Generator: Philox4x64 with 10 rounds as published by Salmon, Moraes, Dror and
Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11).  One call maps a
256-bit counter (four uint64) and a 128-bit key (two uint64) to four uint64.
Each round multiplies words 0 and 2 by the two Philox multipliers, forms the
new words from the high/low halves of the 128-bit products XORed with words
1, 3 and the round key, and bumps the key by the two Weyl constants.

Stream layout shared with the HIP path (each side implements it on its own):
  key     = (seed, 0)
  counter = (block, walker, step, tag << 48 | sweep << 24 | sample)
  word i of a stream is word i % 4 of block i // 4
  uniform u = (word >> 11) * 2^-53                       in [0, 1)
  normals come in Box-Muller pairs from the two uniforms (u_a, u_b) of words
  (2j, 2j+1) of a block: r = sqrt(-2 log(1 - u_a)), t = 2 pi u_b,
  z_{2j} = r cos t, z_{2j+1} = r sin t; normal i is z_{i % 4} of block i // 4.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15   # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1

TAG_FIELD = 1
TAG_PROPOSAL = 2
TAG_ACCEPT = 3
TAG_COMB = 4
TAG_INIT = 5
TAG_MLP = 6


def philox4x64_scalar(ctr, key):
    """Reference single-block Philox4x64-10 in Python integers."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for _ in range(10):
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return (x0, x1, x2, x3)


def _mulhilo64(a: np.ndarray, b: int):
    """Full 64x64 -> 128-bit product of uint64 arrays by a constant."""
    a = a.astype(np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64(ctr: np.ndarray, key0: int, key1: int = 0) -> np.ndarray:
    """Vectorised Philox4x64-10: ctr [..., 4] uint64 -> [..., 4] uint64."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = int(key0) & MASK64, int(key1) & MASK64
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo64(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo64(x2, PHILOX_M1)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                              hi0 ^ x3 ^ np.uint64(k1), lo0)
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
    return np.stack([x0, x1, x2, x3], axis=-1)


def word3(tag: int, sweep: int = 0, sample: int = 0) -> int:
    return (int(tag) << 48) | (int(sweep) << 24) | int(sample)


def _counters(n_blocks: int, walkers: np.ndarray, step: int, w3: np.ndarray) -> np.ndarray:
    """Counter array [len(walkers), len(w3), n_blocks, 4]."""
    nwk, n3 = len(walkers), len(w3)
    c = np.zeros((nwk, n3, n_blocks, 4), dtype=np.uint64)
    c[..., 0] = np.arange(n_blocks, dtype=np.uint64)[None, None, :]
    c[..., 1] = np.asarray(walkers, dtype=np.uint64)[:, None, None]
    c[..., 2] = np.uint64(step)
    c[..., 3] = np.asarray(w3, dtype=np.uint64)[None, :, None]
    return c


def uniforms_from_words(words: np.ndarray) -> np.ndarray:
    return (words >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normals_from_words(words: np.ndarray) -> np.ndarray:
    """words [..., nb, 4] -> normals [..., 4 nb] (Box-Muller pairs)."""
    u = uniforms_from_words(words)
    ua = u[..., 0::2]
    ub = u[..., 1::2]
    r = np.sqrt(-2.0 * np.log(1.0 - ua))
    t = 2.0 * np.pi * ub
    z = np.empty(u.shape, dtype=np.float64)
    z[..., 0::2] = r * np.cos(t)
    z[..., 1::2] = r * np.sin(t)
    return z.reshape(*u.shape[:-2], -1)


def stream_words(seed: int, step: int, walkers, w3s, n_words: int) -> np.ndarray:
    """Raw uint64 words [n_walkers, n_w3, n_words]."""
    nb = (n_words + 3) // 4
    c = _counters(nb, np.asarray(walkers), step, np.asarray(w3s, dtype=np.uint64))
    w = philox4x64(c, seed, 0)
    return w.reshape(len(walkers), len(w3s), nb * 4)[..., :n_words]


def stream_normals(seed: int, step: int, walkers, w3s, n: int) -> np.ndarray:
    nb = (n + 3) // 4
    c = _counters(nb, np.asarray(walkers), step, np.asarray(w3s, dtype=np.uint64))
    w = philox4x64(c, seed, 0)
    return normals_from_words(w)[..., :n]


def stream_uniforms(seed: int, step: int, walkers, w3s, n: int) -> np.ndarray:
    return uniforms_from_words(stream_words(seed, step, walkers, w3s, n))


# Named streams --------------------------------------------------------------

def field_normals(seed: int, step: int, nw: int, n_chol: int, w0: int = 0) -> np.ndarray:
    """Auxiliary fields xi [nw, n_chol] of walkers w0 .. w0 + nw - 1 for one
    propagation step."""
    return stream_normals(seed, step, np.arange(w0, w0 + nw), [word3(TAG_FIELD)], n_chol)[:, 0, :]


def proposal_normals(seed: int, step: int, nw: int, P: int, n: int, sweep: int,
                     w0: int = 0) -> np.ndarray:
    """Normals [nw, P, n] for the hidden-variable proposal of one sweep
    (walkers w0 .. w0 + nw - 1)."""
    w3 = [word3(TAG_PROPOSAL, sweep, p) for p in range(P)]
    return stream_normals(seed, step, np.arange(w0, w0 + nw), w3, n)


def accept_uniforms(seed: int, step: int, nw: int, P: int, n: int, sweep: int,
                    w0: int = 0) -> np.ndarray:
    """Uniforms [nw, P, n] for the Metropolis accept tests of one sweep
    (walkers w0 .. w0 + nw - 1)."""
    w3 = [word3(TAG_ACCEPT, sweep, p) for p in range(P)]
    return stream_uniforms(seed, step, np.arange(w0, w0 + nw), w3, n)


def init_hidden(seed: int, nw: int, P: int, K: int, hidden_kind: int, sweep: int = 0) -> np.ndarray:
    """Initial hidden variables drawn from the trial prior p_T, [nw, P, K].
    sweep 0: the tethered paths; sweeps 1 and 2: the walker field Y_k and its
    partner Y' of the initialisation from the trial (one each per walker, P = 1)."""
    w3 = [word3(TAG_INIT, sweep, p) for p in range(P)]
    if hidden_kind == 0:
        u = stream_uniforms(seed, 0, np.arange(nw), w3, K)
        return np.where(u < 0.5, -1.0, 1.0)
    return stream_normals(seed, 0, np.arange(nw), w3, K)
