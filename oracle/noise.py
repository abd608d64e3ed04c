"""Poisson noise on projection data (the paper's simulated data, Sec. 3.3), float64.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU baseline, never by the library.

Model (reading of the paper's noise statement): a ray with line integral p and
attenuation mu per unit density carries lambda = I0 exp(-mu p) expected photons;
the count is N ~ Poisson(lambda), and the noisy line integral is
p~ = -ln(max(N, 1) / I0) / mu.

Random numbers come from the counter-based generator Philox4x64-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011):
element e draws the blocks philox((e, j, 0, 0), (seed, 0)), j = 0, 1, ..., each
block giving four 64-bit words, and a word x becomes the uniform
((x >> 11) + 1/2) 2^-53 in (0, 1).

The count is drawn
  - for lambda < 10 by inversion: the smallest k with u <= sum_{i<=k} e^-lambda lambda^i / i!,
    accumulated term by term from the first uniform;
  - for lambda >= 10 by Hoermann's transformed rejection with squeeze (PTRS;
    W. Hoermann, "The transformed rejection method for generating Poisson random
    variables", Insurance: Mathematics and Economics 12, 1993), two uniforms per
    trial, trials taking the uniforms of the blocks in order; after 256 rejected
    trials (never reached in practice) the count is lambda rounded to nearest even.
Every decision is taken in float64.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
SMALL_LAMBDA = 10.0
MAX_TRIALS = 256     # rejection trials; acceptance exceeds 0.8 per trial, so never reached


def philox4x64(ctr, key, rounds=10):
    """One Philox4x64 block: counter (4 words), key (2 words) -> 4 words (Python ints)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W[0]) & MASK64
            k1 = (k1 + PHILOX_W[1]) & MASK64
        p0 = PHILOX_M[0] * x0
        p1 = PHILOX_M[1] * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0) & MASK64, p1 & MASK64, ((p0 >> 64) ^ x3 ^ k1) & MASK64, p0 & MASK64
    return [x0, x1, x2, x3]


def to_uniform(x):
    return ((int(x) >> 11) + 0.5) * 2.0 ** -53


class Stream:
    """The uniforms of element e, in order."""

    def __init__(self, seed, e):
        self.seed, self.e, self.j, self.buf = int(seed), int(e), 0, []

    def next(self):
        if not self.buf:
            self.buf = [to_uniform(w) for w in philox4x64((self.e, self.j, 0, 0), (self.seed, 0))]
            self.j += 1
        return self.buf.pop(0)


def poisson_inversion(lam, u):
    """Smallest k with u <= P(N <= k), for lambda < 10 (at most 1000 terms)."""
    p = math.exp(-lam)
    F = p
    k = 0
    while u > F and k < 1000:
        k += 1
        p = p * lam / k
        F = F + p
    return k


def poisson_ptrs(lam, stream):
    """Transformed rejection with squeeze, lambda >= 10."""
    slam = math.sqrt(lam)
    loglam = math.log(lam)
    b = 0.931 + 2.53 * slam
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    v_r = 0.9277 - 3.6224 / (b - 2.0)
    for _ in range(MAX_TRIALS):
        U = stream.next() - 0.5
        V = stream.next()
        us = 0.5 - abs(U)
        k = math.floor((2.0 * a / us + b) * U + lam + 0.43)
        if us >= 0.07 and V <= v_r:
            return k
        if k < 0 or (us < 0.013 and V > us):
            continue
        if math.log(V) + math.log(inv_alpha) - math.log(a / (us * us) + b) <= -lam + k * loglam - math.lgamma(k + 1.0):
            return k
    return round(lam)


def poisson_count(lam, seed, e):
    if not lam > 0.0:
        return 0
    s = Stream(seed, e)
    if lam < SMALL_LAMBDA:
        return poisson_inversion(lam, s.next())
    return poisson_ptrs(lam, s)


def poisson_noise(p, photons, mu, seed):
    """Noisy line integrals and counts for the array p (element index = flat index).
    Pure Python per element: for parity inputs of up to ~1e5 elements."""
    flat = np.asarray(p, np.float64).ravel()
    counts = np.empty(flat.size, np.int64)
    out = np.empty(flat.size, np.float64)
    for e, pe in enumerate(flat):
        lam = photons * math.exp(-mu * pe)
        n = poisson_count(lam, seed, e)
        counts[e] = n
        out[e] = -math.log(max(n, 1) / photons) / mu
    return out.reshape(np.shape(p)), counts.reshape(np.shape(p))
