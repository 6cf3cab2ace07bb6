"""Gaussian random test matrices from a counter-based generator (oracle).

The paper draws the columns of the test matrix Omega_n from a Gaussian
distribution (Section 3.1, first step of the randomized tensor algorithm;
Algorithm 1 draws its test matrix as ``rand(J, l)``; the remark after Algorithm 1 notes
that Gaussian matrices are what the theory assumes).  Here Omega_n is a
pure function of (seed, mode, batch, row, column), so any row block of it
can be regenerated anywhere without being stored.

Generator: Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11): a 4x32-bit counter,
a 2x32-bit key, ten rounds; each round multiplies counter words 0 and 2 by
0xD2511F53 and 0xCD9E8D57, and the key advances by the Weyl constants
0x9E3779B9 / 0xBB67AE85 between rounds.

Mapping (reading adopted for this implementation; the paper does not fix
one):
  key      = (seed mod 2^32, seed >> 32)
  counter  = (j mod 2^32, j >> 32, c // 4, (batch << 8) | mode)
  u_i      = ((x_i >> 8) + 1) * 2^-24  in (0, 1]          (exact in fp32)
  Box-Muller (Box & Muller 1958) on the pairs (u0, u1) and (u2, u3):
     z_{4m}   = sqrt(-2 ln u0) cos(2 pi u1)
     z_{4m+1} = sqrt(-2 ln u0) sin(2 pi u1)
     z_{4m+2} = sqrt(-2 ln u2) cos(2 pi u3)
     z_{4m+3} = sqrt(-2 ln u2) sin(2 pi u3)
  Omega_n[j, c] = z_c of counter group m = c // 4; columns >= l are unused.

Row index j is the C-order position of an element among all elements that
share its mode-n index: for the (L, I_n, Rr) view of a C-order tensor,
j = a * Rr + b.  The oracle evaluates log/sqrt/cos/sin in float64.

Parity: pinned by the published known-answer vectors of Philox4x32-10 and
by an independent implementation (rocRAND's open-source header) compiled
into a host test; the Gaussian transform is pinned statistically.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox rounds on arrays of counters (values < 2^32, any shape).

    Returns the four 32-bit output words as uint64 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0                      # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def omega_bits(seed: int, mode: int, batch: int, row0: int, nrows: int, ngroups: int):
    """Raw Philox words for rows [row0, row0+nrows) and counter groups
    0..ngroups-1: uint64 array (nrows, 4*ngroups), column 4m+i = word i."""
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    j = np.arange(row0, row0 + nrows, dtype=np.uint64)
    lo = j & _MASK
    hi = j >> np.uint64(32)
    tag = np.uint64(((int(batch) << 8) | int(mode)) & 0xFFFFFFFF)
    out = np.empty((nrows, 4 * ngroups), dtype=np.uint64)
    for m in range(ngroups):
        x = philox4x32_10(lo, hi, np.uint64(m), tag, k0, k1)
        for i in range(4):
            out[:, 4 * m + i] = x[i]
    return out


def uniforms(bits):
    """u = ((x >> 8) + 1) / 2^24, in (0, 1]."""
    return ((np.asarray(bits, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 1.0) * (2.0 ** -24)


def omega(seed: int, mode: int, batch: int, row0: int, nrows: int, l: int):
    """Rows [row0, row0+nrows) of the Gaussian test matrix Omega (nrows x l), float64."""
    ngroups = (int(l) + 3) // 4
    u = uniforms(omega_bits(seed, mode, batch, row0, nrows, ngroups))
    z = np.empty_like(u)
    for m in range(ngroups):
        ra = np.sqrt(-2.0 * np.log(u[:, 4 * m + 0]))
        rb = np.sqrt(-2.0 * np.log(u[:, 4 * m + 2]))
        ta = 2.0 * np.pi * u[:, 4 * m + 1]
        tb = 2.0 * np.pi * u[:, 4 * m + 3]
        z[:, 4 * m + 0] = ra * np.cos(ta)
        z[:, 4 * m + 1] = ra * np.sin(ta)
        z[:, 4 * m + 2] = rb * np.cos(tb)
        z[:, 4 * m + 3] = rb * np.sin(tb)
    return z[:, :l]


def omega_uniform(seed: int, mode: int, batch: int, row0: int, nrows: int, l: int):
    """Rows [row0, row0+nrows) of the uniform test matrix (Algorithm 1's test-matrix draw
    writes rand(J, l); the remark after Algorithm 1 notes that a uniform test
    matrix is sufficient in practice): entry (j, c) is the uniform u of word
    c mod 4 of counter group c // 4 of row j, in (0, 1]; float64."""
    ngroups = (int(l) + 3) // 4
    return uniforms(omega_bits(seed, mode, batch, row0, nrows, ngroups))[:, :l]


# the first 64 primes: the Halton bases of columns 0..63
PRIMES = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71, 73,
          79, 83, 89, 97, 101, 103, 107, 109, 113, 127, 131, 137, 139, 149, 151, 157, 163,
          167, 173, 179, 181, 191, 193, 197, 199, 211, 223, 227, 229, 233, 239, 241, 251,
          257, 263, 269, 271, 277, 281, 283, 293, 307, 311]


def radical_inverse(i: int, base: int) -> float:
    """The base-b radical inverse of the integer i >= 1: its digits mirrored
    about the radix point, as the exact ratio of two integers."""
    num, den = 0, 1
    while i > 0:
        i, d = divmod(i, base)
        num = num * base + d
        den *= base
    return num / den


def omega_halton(row0: int, nrows: int, l: int):
    """Rows [row0, row0+nrows) of the quasi-random test matrix (the note in
    Section 3.1 on drawing the entries from a Halton sequence): row j is the
    Halton point j + 1, entry (j, c) the radical inverse of j + 1 in the c-th
    prime base; deterministic, in (0, 1); float64."""
    out = np.empty((nrows, l))
    for c in range(l):
        b = PRIMES[c]
        out[:, c] = [radical_inverse(j + 1, b) for j in range(row0, row0 + nrows)]
    return out


def select_columns(seed: int, mode: int, batch: int, J: int, l: int):
    """l distinct column indices out of J (the remark after Algorithm 1:
    randomly selected columns in place of the sketch's product), by Floyd's
    sampling without replacement: for i = J - l, ..., J - 1 draw t uniform on
    {0, ..., i}; keep t unless already chosen, else keep i.  Draw number s
    takes the Philox words of counter (s mod 2^32, s >> 32, 2^31,
    (batch << 8) | mode): t = floor(x * (i + 1) / 2^64) with
    x = (word1 << 32) | word0.  Returned sorted ascending."""
    if l > J:
        raise ValueError("cannot select more columns than the unfolding has")
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    tag = ((int(batch) << 8) | int(mode)) & 0xFFFFFFFF
    chosen = set()
    for s, i in enumerate(range(J - l, J)):
        w = philox4x32_10(np.uint64(s & 0xFFFFFFFF), np.uint64(s >> 32), np.uint64(1 << 31),
                          np.uint64(tag), k0, k1)
        x = (int(w[1]) << 32) | int(w[0])
        t = (x * (i + 1)) >> 64
        chosen.add(i if t in chosen else t)
    return np.array(sorted(chosen), dtype=np.int64)

