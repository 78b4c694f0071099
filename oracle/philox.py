"""Philox4x64-10 and the standard Gaussian test matrix Omega -- oracle side.

Algorithm 1 draws ``Omega = randn(m, n)`` (Section 3.1; the sketch width
becomes d in the truncated form).  The paper does not name a generator, so
this project fixes one that both sides implement independently from its
published definition:

* Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11): a 4x64-bit counter and a 2x64-bit key;
  each round multiplies counter words 0 and 2 by two fixed odd constants,
  xors the high halves into words 1 and 3 together with the key, and the key
  advances by two Weyl increments between rounds.
* Element Omega[i, j] of an m-row matrix has the column-major index
  l = i + j*m.  Its Philox block is counter (l // 4, 0, 0, 0), key
  (seed, stream); it takes lane l % 4 of that block's four normals.  Hence
  the leading columns of Omega do not depend on d (the prefix property).
* Uniforms: u = ((w >> 12) + 0.5) * 2**-52, exact in fp64 and strictly
  inside (0, 1).
* Normals: Box-Muller on the word pairs (w0, w1) and (w2, w3):
  r = sqrt(-2 ln u_a), z_a = r cos(2 pi u_b), z_b = r sin(2 pi u_b).

Pure numpy uint64 arithmetic; the 64x64->128 multiply is split into 32-bit
halves.
"""
import numpy as np

# Philox4x64 round multipliers and key (Weyl) increments, SC'11 Table 2.
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays: returns (high word, low word)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2**64
    return hi, lo


def philox4x64_10(counters, key):
    """Philox4x64-10 of an (N, 4) uint64 counter array under a 2-word key.

    Returns the (N, 4) uint64 output words, word order as in the counter.
    """
    with np.errstate(over="ignore"):
        c = np.array(counters, dtype=np.uint64, copy=True).reshape(-1, 4)
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        x0, x1, x2, x3 = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
        for r in range(ROUNDS):
            if r > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo(PHILOX_M0, x0)
            hi1, lo1 = _mulhilo(PHILOX_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return np.stack([x0, x1, x2, x3], axis=1)


def uniforms_from_words(w):
    """Map uint64 words to fp64 uniforms ((w >> 12) + 0.5) * 2**-52 in (0, 1)."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def gaussian_words(nblocks, seed, stream=0, first_block=0):
    """Philox output words for blocks first_block .. first_block+nblocks-1."""
    ctr = np.zeros((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(first_block, first_block + nblocks, dtype=np.uint64)
    return philox4x64_10(ctr, (np.uint64(seed), np.uint64(stream)))


def normals_from_block_words(words):
    """Box-Muller on one (N, 4) array of Philox words -> (N, 4) normals."""
    u = uniforms_from_words(words)
    out = np.empty(u.shape, dtype=np.float64)
    for pair in (0, 1):
        ua, ub = u[:, 2 * pair], u[:, 2 * pair + 1]
        r = np.sqrt(-2.0 * np.log(ua))
        t = 2.0 * np.pi * ub
        out[:, 2 * pair] = r * np.cos(t)
        out[:, 2 * pair + 1] = r * np.sin(t)
    return out


def gaussian_matrix(m, d, seed, stream=0):
    """Omega (m x d, fp64): element (i, j) from column-major index i + j*m."""
    total = m * d
    if total == 0:
        return np.zeros((m, d), dtype=np.float64)
    nblocks = (total + 3) // 4
    z = normals_from_block_words(gaussian_words(nblocks, seed, stream))
    flat = z.reshape(-1)[:total]
    return flat.reshape(d, m).T.copy()
