"""Philox4x64-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): ten rounds of two 64x64->128-bit multiplies with the
multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157, a word permutation,
and a Weyl key schedule with increments 0x9E3779B97F4A7C15 and
0xBB67AE8584CAA73B.  Plain Python integers.

Pinned against numpy.random.Philox (an independent implementation of the
same generator) in tests/test_oracle_philox.py.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B


def philox4x64(counter, key, rounds: int = 10):
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(rounds):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
        if r + 1 < rounds:
            k0 = (k0 + _W0) & MASK64
            k1 = (k1 + _W1) & MASK64
    return c0, c1, c2, c3


def proposal_draw(seed: int, walker: int, step: int, n_elec: int):
    """One Metropolis proposal's random numbers.

    key = (seed, 0), counter = (walker, step, 0, 0):
      e = floor(w0 * n_elec / 2^64)      electron index in [0, n_elec)
      d = w1 >> 62                        nearest-neighbour direction 0..3
      u = (w2 >> 11) * 2^-53              uniform in [0, 1)
    """
    w0, w1, w2, _ = philox4x64((walker, step, 0, 0), (seed, 0))
    e = (w0 * n_elec) >> 64
    d = w1 >> 62
    u = (w2 >> 11) * (2.0 ** -53)
    return e, d, u
