"""FP64 oracle for power spectrum and bispectrum multipoles with a global
line of sight (the z axis of the grid).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Power multipoles, ideal limit of eq. (pk-limit) with P_fid = m = 1:
  numerator  p_{b,l} = (1/2) (V/N_pix^2) sum_{n in b} L_l(mu_n) |D(n)|^2 and
  the discrete Fisher matrix F_{b; l l'} = (1/2) sum_{n in b} L_l L_l'
  (eq. pk-limit keeps the l-l' couplings that a finite Fourier grid
  induces; it becomes diag(N_b / (2l+1)) / 2 only in the continuum), so
  P_{b,l} = sum_{l'} (F_b^-1)_{l l'} p_{b,l'}.  Here mu_n = n_z / |n|.
* Bispectrum multipoles by the definition eq. (ideal-bk): the Legendre
  weight sits on k_3 (the mode in the largest bin c), normalised by
  (2l+1) / N_0 with N_0 = T_abc, evaluated through the separable form of
  Sec. IV.D.1 with the weighted field g_{c,l} = IDFT[Theta_c L_l(mu) D]:
  B_{abc,l} = (2l+1) (V^2/N_pix) sum_x G_a G_b g_{c,l} / T_abc.
"""

from __future__ import annotations

import numpy as np

from .polyspec import bin_of_modes, dft, freqs, idft, kmag2, triangle_counts, triangle_triplets


def legendre(ell: int, mu: np.ndarray) -> np.ndarray:
    """Legendre polynomial L_ell for ell in {0, 2, 4}."""
    mu = np.asarray(mu, dtype=np.float64)
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu * mu - 1.0)
    if ell == 4:
        m2 = mu * mu
        return (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0
    raise ValueError("ell must be 0, 2 or 4")


def mu_grid(n: int) -> np.ndarray:
    """mu = n_z / |n| on the full DFT grid (0 at n = 0)."""
    f = freqs(n)
    k2 = kmag2(n).astype(np.float64)
    kz = np.broadcast_to(f[None, None, :].astype(np.float64), k2.shape)
    out = np.zeros_like(k2)
    nz = k2 > 0
    out[nz] = kz[nz] / np.sqrt(k2[nz])
    return out


def power_multipoles(delta: np.ndarray, box: float, edges, lmax: int = 4) -> np.ndarray:
    """P_{b,l} for l = 0, 2, ..., lmax, shape (lmax/2 + 1, n_bins)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    npix = float(n) ** 3
    vol = float(box) ** 3
    D = dft(d)
    p2 = D.real * D.real + D.imag * D.imag
    idx = bin_of_modes(n, edges)
    mu = mu_grid(n)
    ells = list(range(0, lmax + 1, 2))
    L = np.stack([legendre(l, mu) for l in ells])
    nb = len(edges) - 1
    out = np.zeros((len(ells), nb))
    for b in range(nb):
        m = idx == b
        Lb = L[:, m]
        F = 0.5 * Lb @ Lb.T
        p = 0.5 * vol / npix**2 * (Lb * p2[m][None, :]).sum(axis=1)
        out[:, b] = np.linalg.solve(F, p)
    return out


def weighted_fields(delta: np.ndarray, edges, ell: int) -> np.ndarray:
    """g_{b,l} = Re IDFT[Theta_b L_l(mu) D] for every bin."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    D = dft(d)
    idx = bin_of_modes(n, edges)
    w = legendre(ell, mu_grid(n))
    return np.stack([idft(np.where(idx == b, w * D, 0.0)).real for b in range(len(edges) - 1)])


def bispectrum_multipoles(delta: np.ndarray, box: float, edges, lmax: int = 2):
    """(triplets, B) with B of shape (lmax/2 + 1, n_trip) for the triangle-valid
    triplets with T_abc > 0."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(n, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep]
    npix = float(n) ** 3
    vol = float(box) ** 3
    G0 = weighted_fields(d, edges, 0)
    out = []
    for ell in range(0, lmax + 1, 2):
        Gl = G0 if ell == 0 else weighted_fields(d, edges, ell)
        s = np.array([np.sum(G0[a] * G0[b] * Gl[c]) for a, b, c in trips])
        out.append((2 * ell + 1) * vol * vol / npix * s / T)
    return trips, np.array(out)


def brute_multipole_sums(delta: np.ndarray, edges, trips, ell: int):
    """sum over closed triangles (n1 in a, n2 in b, n3 in c, n1+n2+n3 = 0 mod N)
    of L_l(mu_3) D1 D2 D3, by explicit mode loops (N <= 12)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if n > 12:
        raise ValueError("brute force is for N <= 12")
    D = dft(d)
    idx = bin_of_modes(n, edges)
    mu = mu_grid(n)
    nb = len(edges) - 1
    modes = [np.argwhere(idx == b) for b in range(nb)]
    out = np.zeros(len(trips), dtype=np.complex128)
    for t, (a, b, c) in enumerate(trips):
        acc = 0.0 + 0.0j
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = (-i1 - i2) % n
                if idx[tuple(i3)] == c:
                    acc += legendre(ell, mu[tuple(i3)]) * D[tuple(i1)] * D[tuple(i2)] * D[tuple(i3)]
        out[t] = acc
    return out
