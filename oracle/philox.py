"""Counter-based Gaussian numbers for the sampling matrix G and the probes.

The paper draws G from a Gaussian law (Section 4.2.3, the hybrid sampling
matrix Phi).  To let two independent implementations draw the same G, the
entries are a pure function of their coordinates: Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11)
turns a 128-bit counter and a 64-bit key into four 32-bit words, and the
Box-Muller transform turns two 53-bit uniforms into two normals.

Entry coordinates (the convention both implementations follow):
  key  = (seed, 2*level + stream)     stream 0: sketch rows, 1: error probes
  ctr  = (i >> 1, v, segment, half)   i: row of G, v: vertex id of the far
                                      DOF, segment: index within the level,
                                      half: 0 for A[n, sigma] rows, 1 for
                                      A[sigma, n]^T rows
  u1   = ((x1 << 32 | x0) >> 11) * 2^-53 + 2^-54
  u2   = ((x3 << 32 | x2) >> 11) * 2^-53 + 2^-54
  g    = sqrt(-2 ln u1) * (cos(2 pi u2) if i even else sin(2 pi u2))
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on Python integers (one block)."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & np.uint64(MASK) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & np.uint64(MASK)
    k1 = np.asarray(k1, dtype=np.uint64) & np.uint64(MASK)
    m = np.uint64(MASK)
    for _ in range(10):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = (p0 >> np.uint64(32)) & m, p0 & m
        hi1, lo1 = (p1 >> np.uint64(32)) & m, p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & m
        k1 = (k1 + np.uint64(W1)) & m
    return c0, c1, c2, c3


def uniform53(hi, lo):
    """The uniform number in (0, 1] of two 32-bit words: the top 53 bits of
    hi:lo scaled by 2^-53, shifted by half a step (2^-54) so that 0 is never
    reached and the logarithm of Box-Muller stays finite (the largest word
    rounds to exactly 1, which gives a radius of 0)."""
    hi = np.asarray(hi, dtype=np.uint64)
    lo = np.asarray(lo, dtype=np.uint64)
    w = ((hi << np.uint64(32)) | lo) >> np.uint64(11)
    return w.astype(np.float64) * 2.0 ** -53 + 2.0 ** -54


def gaussian(seed, level, stream, rows, verts, segment, halves):
    """Matrix of normals g[i, j] for row indices ``rows`` (length h) and
    columns given by (verts[j], halves[j]) of one segment."""
    rows = np.asarray(rows, dtype=np.uint64)
    verts = np.asarray(verts, dtype=np.uint64)
    halves = np.asarray(halves, dtype=np.uint64)
    R, V = np.meshgrid(rows, verts, indexing="ij")
    _, H = np.meshgrid(rows, halves, indexing="ij")
    x0, x1, x2, x3 = philox4x32_10_np(R >> np.uint64(1), V, np.uint64(segment), H,
                                      np.uint64(seed), np.uint64(2 * level + stream))
    u1 = uniform53(x1, x0)
    u2 = uniform53(x3, x2)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    even = (R & np.uint64(1)) == 0
    return np.where(even, rad * np.cos(ang), rad * np.sin(ang))
