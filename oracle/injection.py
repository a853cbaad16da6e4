"""FP64 expectation of the binned bispectrum of a field with an injected
bispectrum (validation set-up of Sec. VI.B.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Injection: D -> D + (eps/6) beta(k) DFT[phi^2], phi = IDFT[(beta/P) D] for a
Gaussian D with <|D|^2> = (N_pix^2/V) P.  To first order in eps (the eps^2
terms have an odd number of Gaussian factors; the next term is eps^3),
<D1 D2 D3> = eps beta1 beta2 beta3 N_pix^3/V^2 on every closed triangle
n1 + n2 + n3 = 0 (mod N), the lattice closure the estimator uses.  The
expectation of the ideal estimator is therefore the bin average over closed
triangles,

    E[B_abc,l] = eps (2l+1) sum_closed beta1 beta2 beta3 L_l(mu_3) / T_abc
               = eps (2l+1) N_pix^2 sum_x Bt_a Bt_b Bt_c,l / T_abc,

with Bt_b = IDFT[Theta_b beta], Bt_c,l = IDFT[Theta_c beta L_l(mu)] (the
separable form of Sec. IV.D.1).
"""

from __future__ import annotations

import numpy as np

from .multipoles import legendre, mu_grid
from .polyspec import bin_of_modes, idft, kmag2, triangle_counts, triangle_triplets


def _beta_grid(n: int, box: float, beta) -> np.ndarray:
    if not callable(beta):  # given on the full DFT grid
        return np.asarray(beta, dtype=np.float64).reshape(n, n, n)
    kf = 2.0 * np.pi / box
    return np.asarray(beta(kf * np.sqrt(kmag2(n).astype(np.float64))), dtype=np.float64)


def expected_bispectrum(n: int, box: float, edges, beta, eps: float = 1.0, lmax: int = 0):
    """(triplets with T > 0, E[B] of shape (lmax/2 + 1, n_trip)); ``beta`` is
    a callable of k in h/Mpc or an array on the full DFT grid (symmetric
    under n -> -n)."""
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(n, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep]
    bg = _beta_grid(n, box, beta)
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    npix = float(n) ** 3
    Bt = np.stack([idft(np.where(idx == b, bg, 0.0)).real for b in range(nb)])
    mu = mu_grid(n)
    out = []
    for ell in range(0, lmax + 1, 2):
        Bl = Bt if ell == 0 else np.stack(
            [idft(np.where(idx == b, bg * legendre(ell, mu), 0.0)).real for b in range(nb)])
        s = np.array([np.sum(Bt[a] * Bt[b] * Bl[c]) for a, b, c in trips])
        out.append(eps * (2 * ell + 1) * npix**2 * s / T)
    return trips, np.array(out)


def brute_expected(n: int, box: float, edges, trips, beta, ell: int = 0) -> np.ndarray:
    """The same bin average by explicit loops over closed mode triangles (N <= 12)."""
    if n > 12:
        raise ValueError("brute force is for N <= 12")
    bg = _beta_grid(n, box, beta)
    idx = bin_of_modes(n, edges)
    Lmu = legendre(ell, mu_grid(n))
    out = np.zeros(len(trips))
    for t, (a, b, c) in enumerate(trips):
        tot, cnt = 0.0, 0
        for i1 in np.argwhere(idx == a):
            for i2 in np.argwhere(idx == b):
                i3 = tuple((-i1 - i2) % n)
                if idx[i3] == c:
                    tot += bg[tuple(i1)] * bg[tuple(i2)] * bg[i3] * Lmu[i3]
                    cnt += 1
        out[t] = (2 * ell + 1) * tot / cnt if cnt else np.nan
    return out
