"""Counter-based random numbers for the oracle (test infrastructure only).

The paper asks for an independent pseudo-random stream per parallel worker so
that intra-chain loops over univariate draws can run in parallel (Sec.
"Comments on parallelization").  A counter-based generator gives every draw
its own address instead, so any worker -- a CPU core or a GPU lane -- can
produce the draw for (chain, sweep, phase, element) without shared state.

Generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11).  One call maps a 128-bit counter
(w0, w1, w2, w3) and a 64-bit key (k0, k1) to four 32-bit words.  A round
multiplies counter words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57
(full 64-bit products), and outputs (hi(w2*M1) ^ w1 ^ k0, lo(w2*M1),
hi(w0*M0) ^ w3 ^ k1, lo(w0*M0)); the key is bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85) between rounds.

Derived draws (the contract shared with the GPU path):
  U23(x)   = (floor(x / 2^9) + 1/2) * 2^-23, in (0, 1), exact in FP32 and FP64
  normals  Box-Muller on a word pair (xa, xb): r = sqrt(-2 ln U23(xa)),
           theta = 2 pi U23(xb); the pair is (r cos theta, r sin theta)
  gamma    Marsaglia & Tsang, "A simple method for generating gamma
           variables", ACM TOMS 26(3), 2000, without the squeeze test

Pins: philox4x32_10 against rocRAND's philox4x32_10 engine (a library
implementation compiled on the host), U23 / Box-Muller / gamma against their
distributions (KS tests against scipy.stats) -- see tests/test_oracle_rng.py.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_S32 = np.uint64(32)

# Phase word w2 of the counter: which step of the sweep a draw belongs to.
PHASE_MESSENGER = 0
PHASE_SIGNAL = 1
PHASE_GAMMA = 2
GAMMA_ATTEMPTS = 1 << 16   # counter word 0 of a gamma draw is bin * 2^16 + attempt


def key_words(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def philox4x32_10(w0, w1, w2, w3, k0, k1):
    """Four uint32 output arrays for counters (w0..w3) and key (k0, k1)."""
    c0, c1, c2, c3 = (np.asarray(w, dtype=np.uint64) & _MASK for w in (w0, w1, w2, w3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    ka = np.uint64(k0) & _MASK
    kb = np.uint64(k1) & _MASK
    for _ in range(10):
        p0 = _M0 * c0          # < 2^64: exact in uint64
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ ka, p1 & _MASK,
                          (p0 >> _S32) ^ c3 ^ kb, p0 & _MASK)
        ka = (ka + _W0) & _MASK
        kb = (kb + _W1) & _MASK
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def u23(x) -> np.ndarray:
    """Uniform on (0, 1) from the top 23 bits of a 32-bit word."""
    x = np.asarray(x, dtype=np.uint32)
    return ((x >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(xa, xb):
    """A pair of independent unit normals from two 32-bit words."""
    r = np.sqrt(-2.0 * np.log(u23(xa)))
    theta = 2.0 * np.pi * u23(xb)
    return r * np.cos(theta), r * np.sin(theta)


def normals4(w0, w1, w2, w3, seed):
    """The four unit normals of one Philox call: (cos A, sin A, cos B, sin B)."""
    k0, k1 = key_words(seed)
    x0, x1, x2, x3 = philox4x32_10(w0, w1, w2, w3, k0, k1)
    ga, gb = box_muller(x0, x1)
    gc, gd = box_muller(x2, x3)
    return ga, gb, gc, gd


def gamma_mt(shape: float, seed: int, chain: int, sweep: int, bin_index: int) -> float:
    """One Gamma(shape, 1) draw by Marsaglia & Tsang (2000).

    Attempt j of bin b in sweep n of chain c reads the Philox words of counter
    (b * 2^16 + j, n, PHASE_GAMMA, c).  z is the cosine normal of the word pair
    (x0, x1) and u = U23(x2).  With d = shape - 1/3 and c' = 1/sqrt(9 d), the
    candidate v = (1 + c' z)^3 is accepted when v > 0 and
    ln u < z^2 / 2 + d - d v + d ln v; the draw is then d v.  For shape < 1 the
    draw is Gamma(shape + 1) * U^(1/shape) with U = U23(x3) of attempt 0.
    """
    k0, k1 = key_words(seed)
    a = float(shape)
    boost = a < 1.0
    if boost:
        a += 1.0
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    u_boost = None
    for j in range(GAMMA_ATTEMPTS):
        x0, x1, x2, x3 = philox4x32_10(bin_index * GAMMA_ATTEMPTS + j, sweep, PHASE_GAMMA,
                                       chain, k0, k1)
        if j == 0:
            u_boost = float(u23(x3))
        z = float(box_muller(x0, x1)[0])
        u = float(u23(x2))
        v = (1.0 + c * z) ** 3
        if v > 0.0 and np.log(u) < 0.5 * z * z + d - d * v + d * np.log(v):
            g = d * v
            return g * u_boost ** (1.0 / shape) if boost else g
    raise RuntimeError("Marsaglia-Tsang: no acceptance within 2^16 attempts")
