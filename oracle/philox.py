"""Philox4x32-10 counter-based generator and the uniform / normal transforms.

Test infrastructure (CPU oracle); never part of the product path.

The paper draws its random numbers with a per-thread stateful generator that is
kept between kernel launches (Sec. "Kernel Design").  This build replaces it by
a stateless counter-based generator so that every random number is a pure
function of (seed, MPC step, SMC iteration, purpose, element index).  The
generator is Philox4x32 with 10 rounds as defined by Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):

  * state: counter (c0, c1, c2, c3) and key (k0, k1), 32-bit words;
  * one round: multiply c0 by 0xD2511F53 and c2 by 0xCD9E8D57 as 32x32->64
    products (hi, lo); the new counter is
    (hi(c2 product) ^ c1 ^ k0, lo(c2 product), hi(c0 product) ^ c3 ^ k1,
    lo(c0 product));
  * between rounds the key is bumped by the Weyl constants
    (0x9E3779B9, 0xBB67AE85);
  * the four output words are the counter after 10 rounds.

Counter layout used throughout: (element index, SMC iteration J,
purpose | scenario << 8, MPC step), key = (seed low word, seed high word).

Parity note: no published known-answer vectors are available here; the
generator is pinned by statistical properties and bijectivity (tests), and the
GPU words are compared bit-exactly with these.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint32(0x9E3779B9)
PHILOX_W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

# purposes of random draws (third counter word, low byte)
INIT, WIND, RESAMPLE, MOVE, ACCEPT, MALA = 1, 2, 3, 4, 5, 6


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit counters; returns 4 uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32).astype(np.uint64)
    c1 = np.asarray(c1, dtype=np.uint32).astype(np.uint64)
    c2 = np.asarray(c2, dtype=np.uint32).astype(np.uint64)
    c3 = np.asarray(c3, dtype=np.uint32).astype(np.uint64)
    k0 = np.uint64(np.uint32(k0))
    k1 = np.uint64(np.uint32(k1))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & MASK32
        p0 = PHILOX_M0 * c0            # < 2^64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def words(seed: int, mpc_step: int, J: int, purpose: int, elem, scenario: int = 0):
    """The 4 Philox words for element indices ``elem`` of one stream."""
    elem = np.asarray(elem, dtype=np.int64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    c1 = np.uint32(int(J) & 0xFFFFFFFF)
    c2 = np.uint32(((int(scenario) << 8) | int(purpose)) & 0xFFFFFFFF)
    c3 = np.uint32(int(mpc_step) & 0xFFFFFFFF)
    return philox4x32_10(elem.astype(np.uint32), c1, c2, c3, k0, k1)


def uniform_from(wa, wb):
    """u = ((wa >> 6) * 2^26 + (wb >> 6) + 1/2) * 2^-52, strictly inside (0, 1).

    52 random bits; the sum is < 2^52 so adding 1/2 and scaling are exact."""
    a = (np.asarray(wa, np.uint32) >> np.uint32(6)).astype(np.float64)
    b = (np.asarray(wb, np.uint32) >> np.uint32(6)).astype(np.float64)
    return (a * 67108864.0 + b + 0.5) * 2.0 ** -52


def uniforms(seed, mpc_step, J, purpose, elem, scenario=0):
    w = words(seed, mpc_step, J, purpose, elem, scenario)
    return uniform_from(w[0], w[1])


def normals_pair(seed, mpc_step, J, purpose, elem, scenario=0):
    """Box-Muller pair (z0, z1) from one counter: u1 from words (0, 1),
    u2 from words (2, 3); z0 = r cos(2 pi u2), z1 = r sin(2 pi u2) with
    r = sqrt(-2 ln u1)."""
    w = words(seed, mpc_step, J, purpose, elem, scenario)
    u1 = uniform_from(w[0], w[1])
    u2 = uniform_from(w[2], w[3])
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def normals(seed, mpc_step, J, purpose, elem, scenario=0):
    """One standard normal per element (the first of the Box-Muller pair)."""
    return normals_pair(seed, mpc_step, J, purpose, elem, scenario)[0]
