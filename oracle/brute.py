"""Brute-force k-space sums for tiny grids (N <= 16).

TEST INFRASTRUCTURE ONLY (see ``oracle/polyspec.py``).

These evaluate the bispectrum numerator and the triangle count straight
from their Fourier-space definitions -- the triple integral over
k1 + k2 + k3 = 0 of eq. (ideal-bk) and eq. (N-ell-def) at ell = 0, with the
Dirac delta discretised as closure modulo N -- by looping over every mode
pair (n1, n2) and setting n3 = -(n1 + n2) mod N.  They share no arithmetic
with the separable real-space form and so pin it (eq. beta-def).
"""

from __future__ import annotations

import numpy as np

from .polyspec import bin_of_modes, dft

__all__ = ["brute_sums"]


def brute_sums(delta: np.ndarray, edges, trips):
    """Return (sum over closed triangles of D1 D2 D3, triangle count) per triplet.

    Pure Python loops over modes: keep N <= 16.
    """
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if n > 16:
        raise ValueError("brute force is for N <= 16")
    D = dft(d)
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    modes = [[] for _ in range(nb)]
    for i in range(n):
        for j in range(n):
            for k in range(n):
                b = int(idx[i, j, k])
                if b >= 0:
                    modes[b].append((i, j, k))
    sums = np.zeros(len(trips), dtype=np.complex128)
    cnt = np.zeros(len(trips), dtype=np.int64)
    for t, (a, b, c) in enumerate(trips):
        acc = 0.0 + 0.0j
        m = 0
        for (i1, j1, k1) in modes[a]:
            for (i2, j2, k2) in modes[b]:
                i3 = (-i1 - i2) % n
                j3 = (-j1 - j2) % n
                k3 = (-k1 - k2) % n
                if idx[i3, j3, k3] == c:
                    acc += D[i1, j1, k1] * D[i2, j2, k2] * D[i3, j3, k3]
                    m += 1
        sums[t] = acc
        cnt[t] = m
    return sums, cnt
