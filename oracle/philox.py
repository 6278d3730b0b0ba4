"""Counter-based random streams: Philox4x64-10 and Box-Muller normals.

The paper draws its normals with cuRAND (Section "Efficient generation of model
errors"); any stream of independent N(0,1) draws satisfies the method.  Both the oracle
and the HIP library implement the same published counter-based generator (Salmon,
Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3", SC'11), so the two
paths draw identical numbers without sharing code.

Philox4x64-R: a 4x64-bit counter and a 2x64-bit key.  Each round multiplies counter
words 0 and 2 by two fixed odd constants, and rebuilds the counter from the high and low
product halves xor-ed with the other two words and the key; the key is advanced by two
Weyl constants between rounds.  Ten rounds.

Stream layout (shared convention, documented in the library header as well):
  key     = (seed, 0)
  counter = (block, step_or_analysis_index, (tag << 32) | ensemble_id, particle)
One block yields four 64-bit words -> two Box-Muller pairs -> four normals; normal n of
a field is lane n % 4 of block n // 4.  Box-Muller in float64:
  u1 = ((x >> 11) + 1) * 2^-53  in (0, 1],  u2 = (y >> 11) * 2^-53  in [0, 1)
  (r cos(2 pi u2), r sin(2 pi u2)),  r = sqrt(-2 ln u1).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1

TAG_MODEL_ERROR = 1
TAG_XI = 2
TAG_NU = 3
TAG_OBS = 4
TAG_INIT = 5
TAG_RESAMPLE = 6

TWO_PI = 6.283185307179586
TWO_M53 = 2.0 ** -53


def philox4x64_int(ctr, key, rounds: int = 10):
    """Reference Philox4x64 on Python integers (one counter)."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """64x64 -> 128-bit product of a constant a and uint64 array b, as (hi, lo)."""
    a = np.uint64(a)
    aL, aH = a & _M32, a >> _S32
    bL, bH = b & _M32, b >> _S32
    ll = aL * bL
    lh = aL * bH
    hl = aH * bL
    hh = aH * bH
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps mod 2^64
    return hi, lo


def philox4x64(c0: np.ndarray, c1, c2, c3, key0: int, key1: int = 0, rounds: int = 10):
    """Vectorised Philox4x64 over an array of counter word 0 (other words broadcast)."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        shape = c0.shape
        c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), shape).copy()
        c2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), shape).copy()
        c3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), shape).copy()
        c0 = c0.copy()
        k0 = int(key0) & MASK64
        k1 = int(key1) & MASK64
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo(PHILOX_M0, c0)
            hi1, lo1 = _mulhilo(PHILOX_M1, c2)
            c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def counter_words(step: int, tag: int, ensemble_id: int, particle: int):
    """Counter words 1..3 of the stream layout."""
    return (int(step) & MASK64, ((int(tag) << 32) | (int(ensemble_id) & 0xFFFFFFFF)) & MASK64,
            int(particle) & MASK64)


def box_muller(x: np.ndarray, y: np.ndarray):
    """Two uint64 words -> two float64 N(0,1) draws."""
    u1 = ((x >> np.uint64(11)).astype(np.float64) + 1.0) * TWO_M53
    u2 = (y >> np.uint64(11)).astype(np.float64) * TWO_M53
    r = np.sqrt(-2.0 * np.log(u1))
    ang = TWO_PI * u2
    return r * np.cos(ang), r * np.sin(ang)


def normals(n: int, seed: int, step: int, tag: int, ensemble_id: int, particle: int) -> np.ndarray:
    """First n normals of the stream (seed; step, tag, ensemble, particle), float64."""
    nblk = (n + 3) // 4
    w1, w2, w3 = counter_words(step, tag, ensemble_id, particle)
    x0, x1, x2, x3 = philox4x64(np.arange(nblk, dtype=np.uint64), w1, w2, w3, seed, 0)
    a0, a1 = box_muller(x0, x1)
    a2, a3 = box_muller(x2, x3)
    out = np.stack([a0, a1, a2, a3], axis=1).reshape(-1)
    return out[:n]


def uniforms(n: int, seed: int, step: int, tag: int, ensemble_id: int, particle: int) -> np.ndarray:
    """First n uniforms in [0,1) of the stream: word w of block b is draw 4b+w, u=(x>>11) 2^-53."""
    nblk = (n + 3) // 4
    w1, w2, w3 = counter_words(step, tag, ensemble_id, particle)
    xs = philox4x64(np.arange(nblk, dtype=np.uint64), w1, w2, w3, seed, 0)
    words = np.stack(xs, axis=1).reshape(-1)[:n]
    return (words >> np.uint64(11)).astype(np.float64) * TWO_M53
