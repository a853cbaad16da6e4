"""FP64 oracle for the weighted ideal estimators: fiducial-power weights,
pixel-window deconvolution and Poisson shot noise.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (ideal limits of Sec. III.D.1, eq. pk-limit, and Sec. IV.D.1,
with the data d = nbar delta so that the 1/nbar factors cancel):

* window      m(n) = prod_i sinc(pi n_i / N)^order  (order 1 NGP, 2 CIC, 3 TSC);
* power       P_b = (V/N_pix^2) sum_{n in b} |D/m|^2 / P_fid^2 / sum_{n in b} 1/P_fid^2 - 1/nbar
              (the Fisher matrix is the P_fid^-2 weighted bin volume; the bias
              term contributes 1/nbar);
* bispectrum  B_abc = (V^2/N_pix^3) sum_closed D1 D2 D3 / (m1 m2 m3 P1 P2 P3) / N_0 - B_shot,
              N_0 = sum_closed 1/(P1 P2 P3),
              B_shot = 1/nbar^2 + <P1 + P2 + P3>/nbar with the N_0 weights and the
              power model P = P_fid - 1/nbar (P_fid includes the shot noise).
  Separable form (eq. beta-def): with G~_b = IDFT[Theta_b D/(m P_fid)],
  H~_b = IDFT[Theta_b / P_fid] and H_b = IDFT[Theta_b],
  B = (V^2/N_pix) sum_x G~G~G~ / N_0,  N_0 = N_pix^2 sum_x H~H~H~,
  <P1+P2+P3> = N_pix^2 sum_x (H_a H~_b H~_c + H~_a H_b H~_c + H~_a H~_b H_c) / N_0 - 3/nbar.
* multipoles (global line of sight along z, eq. pk-limit and eq. bk-num-ideal
  with their ideal normalisations):
  P_{b,l} = sum_l' (F_b^-1)_{l l'} p_{b,l'} - delta_l0 / nbar with
  p_{b,l} = (V/N_pix^2) sum_{n in b} L_l |D/m|^2 / P_fid^2 and
  F_b[l][l'] = sum_{n in b} L_l L_l' / P_fid^2 (the discrete Fisher matrix);
  B_{abc,l} = (2l+1) (V^2/N_pix) sum_x G~_a G~_b g~_{c,l} / N_0 - delta_l0 B_shot,
  g~_{c,l} = IDFT[Theta_c L_l(mu) D/(m P_fid)].  With an isotropic P_fid the
  Poisson terms load only the monopole (Sec. IV.D.1, and for P the discrete
  Fisher matrix maps a constant 1/nbar exactly onto l = 0).
"""

from __future__ import annotations

import numpy as np

from . import noncubic as _nc
from .multipoles import legendre, mu_grid
from .polyspec import bin_of_modes, dft, freqs, idft, triangle_counts, triangle_triplets


def _shape(n) -> tuple:
    return tuple(int(v) for v in np.broadcast_to(np.asarray(n), (3,)))


def window(n, order: int) -> np.ndarray:
    """m(n) = prod_i sinc(pi n_i / N_i)^order on the full DFT grid of side n
    (or shape (Nx, Ny, Nz))."""
    w = [np.sinc(freqs(N).astype(np.float64) / N) ** order for N in _shape(n)]  # sinc(x) = sin(pi x)/(pi x)
    return w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]


def _kmag2(shape) -> np.ndarray:
    fx, fy, fz = (freqs(N) for N in shape)
    return fx[:, None, None] ** 2 + fy[None, :, None] ** 2 + fz[None, None, :] ** 2


def _pfid_grid(n, pfid) -> np.ndarray:
    k2 = _kmag2(_shape(n))
    if pfid is None:
        return np.ones(k2.shape)
    tab = np.asarray(pfid, dtype=np.float64)
    out = np.ones(k2.shape)
    inside = k2 < tab.size
    out[inside] = tab[k2[inside]]
    return out


def weighted_power(delta, box: float, edges, order: int = 0, pfid=None, nbar: float = 0.0) -> np.ndarray:
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape  # any grid shape; a box with equal sides (P_fid over integer |n|^2)
    npix, vol = float(d.size), float(box) ** 3
    D = dft(d) / window(n, order)
    P = _pfid_grid(n, pfid)
    idx = _nc.bin_of_modes(n, box, edges)
    nb = len(edges) - 1
    out = np.zeros(nb)
    for b in range(nb):
        m = idx == b
        w = 1.0 / P[m] ** 2
        out[b] = vol / npix**2 * np.sum(w * np.abs(D[m]) ** 2) / np.sum(w)
    return out - (1.0 / nbar if nbar > 0 else 0.0)


def weighted_bispectrum(delta, box: float, edges, order: int = 0, pfid=None, nbar: float = 0.0):
    """(triplets, B, N_0, A) for the triangle-valid triplets with closed triangles;
    A is the same normalisation of sum_x |G~ G~ G~| (for tolerances)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape
    npix, vol = float(d.size), float(box) ** 3
    trips = triangle_triplets(edges)
    T, _ = _nc.triangle_counts(n, box, edges, trips)
    trips = trips[T > 0]
    P = _pfid_grid(n, pfid)
    D = dft(d) / (window(n, order) * P)
    idx = _nc.bin_of_modes(n, box, edges)
    nb = len(edges) - 1
    G = np.stack([idft(np.where(idx == b, D, 0.0)).real for b in range(nb)])
    Hw = np.stack([idft(np.where(idx == b, 1.0 / P, 0.0)).real for b in range(nb)])
    s = np.array([np.sum(G[a] * G[b] * G[c]) for a, b, c in trips])
    sa = np.array([np.sum(np.abs(G[a] * G[b] * G[c])) for a, b, c in trips])
    n0 = npix**2 * np.array([np.sum(Hw[a] * Hw[b] * Hw[c]) for a, b, c in trips])
    B = vol * vol / npix * s / n0
    A = vol * vol / npix * sa / n0
    if nbar > 0:
        H = np.stack([idft((idx == b).astype(np.float64)).real for b in range(nb)])
        q = npix**2 * np.array([np.sum(H[a] * Hw[b] * Hw[c] + Hw[a] * H[b] * Hw[c] + Hw[a] * Hw[b] * H[c])
                                for a, b, c in trips])
        B = B - (1.0 / nbar**2 + (q / n0 - 3.0 / nbar) / nbar)
    return trips, B, n0, A


def weighted_power_multipoles(delta, box: float, edges, lmax: int = 4, order: int = 0, pfid=None,
                              nbar: float = 0.0) -> np.ndarray:
    """P_{b,l} for l = 0, 2, ..., lmax, shape (lmax/2 + 1, n_bins)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    npix, vol = float(n) ** 3, float(box) ** 3
    D = dft(d) / window(n, order)
    p2 = D.real * D.real + D.imag * D.imag
    P = _pfid_grid(n, pfid)
    idx = bin_of_modes(n, edges)
    mu = mu_grid(n)
    ells = list(range(0, lmax + 1, 2))
    L = np.stack([legendre(l, mu) for l in ells])
    out = np.zeros((len(ells), len(edges) - 1))
    for b in range(len(edges) - 1):
        m = idx == b
        w = 1.0 / P[m] ** 2
        Lb = L[:, m]
        F = (Lb * w[None, :]) @ Lb.T
        p = vol / npix**2 * (Lb * (w * p2[m])[None, :]).sum(axis=1)
        out[:, b] = np.linalg.solve(F, p)
    if nbar > 0:
        out[0] -= 1.0 / nbar
    return out


def weighted_bispectrum_multipoles(delta, box: float, edges, lmax: int = 2, order: int = 0, pfid=None,
                                   nbar: float = 0.0):
    """(triplets, B) with B of shape (lmax/2 + 1, n_trip) for the triangle-valid
    triplets with closed triangles."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    npix, vol = float(n) ** 3, float(box) ** 3
    trips, B0, n0, _ = weighted_bispectrum(d, box, edges, order, pfid, nbar)
    P = _pfid_grid(n, pfid)
    D = dft(d) / (window(n, order) * P)
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    G = np.stack([idft(np.where(idx == b, D, 0.0)).real for b in range(nb)])
    out = [B0]
    mu = mu_grid(n)
    for ell in range(2, lmax + 1, 2):
        Dl = legendre(ell, mu) * D
        Gl = np.stack([idft(np.where(idx == b, Dl, 0.0)).real for b in range(nb)])
        s = np.array([np.sum(G[a] * G[b] * Gl[c]) for a, b, c in trips])
        out.append((2 * ell + 1) * vol * vol / npix * s / n0)
    return trips, np.array(out)


def brute_weighted_sums(delta, edges, trips, order: int = 0, pfid=None, ell: int = 0):
    """By explicit loops over closed mode triangles (N <= 8): the weighted
    numerator sum L_l(mu_3) D1 D2 D3 / (m1 m2 m3 P1 P2 P3), N_0 = sum 1/(P1 P2 P3)
    and sum (P1 + P2 + P3)/(P1 P2 P3)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if n > 8:
        raise ValueError("brute force is for N <= 8")
    D = dft(d) / window(n, order)
    P = _pfid_grid(n, pfid)
    idx = bin_of_modes(n, edges)
    Lmu = legendre(ell, mu_grid(n))
    modes = [np.argwhere(idx == b) for b in range(len(edges) - 1)]
    num = np.zeros(len(trips), dtype=np.complex128)
    n0 = np.zeros(len(trips))
    q = np.zeros(len(trips))
    for t, (a, b, c) in enumerate(trips):
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = (-i1 - i2) % n
                if idx[tuple(i3)] != c:
                    continue
                p1, p2, p3 = P[tuple(i1)], P[tuple(i2)], P[tuple(i3)]
                wt = 1.0 / (p1 * p2 * p3)
                num[t] += wt * Lmu[tuple(i3)] * D[tuple(i1)] * D[tuple(i2)] * D[tuple(i3)]
                n0[t] += wt
                q[t] += wt * (p1 + p2 + p3)
    return num, n0, q
