"""Philox4x64-10 and the draw maps of Alg. 1 (oracle side; test infrastructure only).

Alg. 1 draws a reduced normal vector xi_r ~ N(0, I_r) for the proposal, a uniform
xi_1 for the first-stage decision, and the splitting proposition of Sec. 5.3 draws a prior sample M ~ mu for
the complement move. Both the oracle and the device path generate these from one
counter-based generator so that chains can be compared draw for draw.

Generator: Philox4x64 with 10 rounds, as defined by Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11). A 4x64-bit counter and a
2x64-bit key map to four 64-bit outputs:

    round:  (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2      (128-bit products)
            c' = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)
    key schedule between rounds: k0 += W0, k1 += W1   (mod 2^64)

with M0 = 0xD2E7470EE14C6C93, M1 = 0xCA5A826395121157 and the Weyl increments
W0 = 0x9E3779B97F4A7C15 (golden ratio), W1 = 0xBB67AE8584CAA73B (sqrt(3) - 1).

Stream layout used by both sides:
    key     = (seed, request_id)
    counter = (block, stream, step, chain)
    stream  = 0 proposal normals xi_r, 1 complement normals, 2 MH uniform,
              3 initial reduced state, 4 initial complement state.

Maps from a 64-bit word w:
    uniform  u = ((w >> 12) + 0.5) * 2^-52, exact in double and strictly inside (0, 1)
             (from 2^-53 to 1 - 2^-53);
    normals  Box-Muller on the pairs (u0, u1) and (u2, u3) of one block:
             n0 = R(u0) cos(2 pi u1), n1 = R(u0) sin(2 pi u1),
             n2 = R(u2) cos(2 pi u3), n3 = R(u2) sin(2 pi u3), R(u) = sqrt(-2 log u).
Normal number i of a stream comes from block i // 4, slot i % 4.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1

STREAM_XI = 0
STREAM_COMPLEMENT = 1
STREAM_UNIFORM = 2
STREAM_INIT_X = 3
STREAM_INIT_Z = 4


def philox4x64_scalar(counter, key, rounds: int = 10):
    """Reference Philox4x64 on Python integers (one block)."""
    c = [int(v) & MASK64 for v in counter]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for i in range(rounds):
        if i > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """128-bit product of the constant a with each uint64 in b, split into 32-bit limbs."""
    a0 = np.uint64(a & 0xFFFFFFFF)
    a1 = np.uint64(a >> 32)
    b0 = b & _M32
    b1 = b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = np.uint64(a) * b  # wraps mod 2^64
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Vectorised Philox4x64 over broadcastable uint64 arrays; returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for i in range(rounds):
            if i > 0:
                k0 = np.uint64((int(k0) + W0) & MASK64)
                k1 = np.uint64((int(k1) + W1) & MASK64)
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def to_uniform(w: np.ndarray) -> np.ndarray:
    """Map 64-bit words to doubles strictly inside (0, 1): ((w >> 12) + 0.5) 2^-52."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def normals(seed: int, request_id: int, stream: int, step, chain, count: int) -> np.ndarray:
    """Normals 0..count-1 of one stream for each (step, chain) pair.

    ``step`` and ``chain`` broadcast against each other; the result has shape
    broadcast(step, chain).shape + (count,).
    """
    step = np.asarray(step, dtype=np.uint64)
    chain = np.asarray(chain, dtype=np.uint64)
    step, chain = np.broadcast_arrays(step, chain)
    nblk = (count + 3) // 4
    blk = np.arange(nblk, dtype=np.uint64)
    shape = step.shape + (nblk,)
    o = philox4x64(np.broadcast_to(blk, shape), np.full(shape, stream, dtype=np.uint64),
                   np.broadcast_to(step[..., None], shape), np.broadcast_to(chain[..., None], shape),
                   seed, request_id)
    u = [to_uniform(v) for v in o]
    r01 = np.sqrt(-2.0 * np.log(u[0]))
    r23 = np.sqrt(-2.0 * np.log(u[2]))
    t1 = 2.0 * np.pi * u[1]
    t3 = 2.0 * np.pi * u[3]
    out = np.empty(shape + (4,), dtype=np.float64)
    out[..., 0] = r01 * np.cos(t1)
    out[..., 1] = r01 * np.sin(t1)
    out[..., 2] = r23 * np.cos(t3)
    out[..., 3] = r23 * np.sin(t3)
    return out.reshape(step.shape + (nblk * 4,))[..., :count]


def uniforms(seed: int, request_id: int, step, chain) -> np.ndarray:
    """The MH uniform xi_1 of Alg. 1 for each (step, chain): word 0 of block 0, stream 2."""
    step = np.asarray(step, dtype=np.uint64)
    chain = np.asarray(chain, dtype=np.uint64)
    step, chain = np.broadcast_arrays(step, chain)
    o = philox4x64(np.zeros(step.shape, dtype=np.uint64),
                   np.full(step.shape, STREAM_UNIFORM, dtype=np.uint64), step, chain,
                   seed, request_id)
    return to_uniform(o[0])
