"""FP64 oracle of the bispectrum multipoles with the discrete ideal Fisher
matrix: eq. (bk-num-ideal) and eq. (bk-fish-ideal) of Sec. IV.D.1 with the
degeneracy factors of eq. (Delta-alpha-def) and N_l of eq. (N-ell-def),
global line of sight along z, P_fid = m = nbar = 1, cubic grid and box.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a kept triplet t = (a, b, c), a <= b <= c, and l, l' in {0, 2, ..,
lmax}, the sums run over the closed triangles n1 + n2 + n3 = 0 (mod N)
with n1 in bin a, n2 in b, n3 in c; mu_i = n_i,z / |n_i| and u_i = n_i / |n_i|:

* numerator (eq. bk-num-ideal without its 1/Delta):
      nt_l = (V^2 / N_pix^3) sum L_l(mu_3) D1 D2 D3;
* Fisher block (eq. bk-fish-ideal without its 1/(Delta_l Delta_l')): the
  six permutations of the k's that keep every k_i in its bin leave
      Ft_{l l'} = sum L_l(mu_3) P_l'
      P_l' = L_l'(mu_3)                              a < b < c
             2 L_l'(mu_3)                            a = b < c
             L_l'(mu_3) + L_l'(mu_2)                 a < b = c
             2 [L_l'(mu_1) + L_l'(mu_2) + L_l'(mu_3)]  a = b = c
  (blocks of different bin triplets do not couple);
* degeneracy (eq. Delta-alpha-def): Delta_l = 1, 2, 1 + N_l/N_0,
  2 (1 + 2 N_l/N_0) in the same four cases, with N_l = sum L_l(u_2 . u_3)
  (eq. N-ell-def on the grid) and N_0 = T;
* estimator: F = Delta^-1 Ft Delta^-1 and b^num = Delta^-1 nt, so
      b = F^-1 b^num = Delta Ft^+ nt,
  Ft^+ the pseudo-inverse of the symmetric block (eigenvalues below 1e-12
  of the largest are dropped).

In the continuum Ft -> diag(Delta_l T / (2l+1)) (eq. bk-fish-ideal2) and b
reduces to eq. (ideal-bk), (2l+1) nt_l / T, which is what
``oracle.multipoles.bispectrum_multipoles`` returns.

Separable forms (Sec. IV.D.1): for even weights f, g, h,
sum f(n1) g(n2) h(n3) over closed triangles = N_pix^2 sum_x F G H with
F = IDFT[Theta_a f] etc.; N_l goes through the tensor expansion
(u . v)^p = sum_{|alpha| = p} p!/alpha! u^alpha v^alpha.

Reading (the paper is silent on it): a mode with a Nyquist component
(|n_i| = N/2) has two representatives, +N/2 and -N/2, whose directions
differ; in N_l such a mode takes the average over its representatives, so
odd powers of a Nyquist component vanish.  (mu^2 and the Legendre weights
do not depend on the choice.)
"""

from __future__ import annotations

import itertools
import math

import numpy as np

from .multipoles import legendre, mu_grid, weighted_fields
from .polyspec import bin_of_modes, dft, freqs, idft, kmag2, triangle_counts, triangle_triplets


def _case(a: int, b: int, c: int) -> int:
    """0: a < b < c, 1: a = b < c, 2: a < b = c, 3: a = b = c."""
    if a == b == c:
        return 3
    if a == b:
        return 1
    if b == c:
        return 2
    return 0


def _unit_grid(n: int) -> np.ndarray:
    """u = n / |n| on the full grid, shape (3, n, n, n) (0 at n = 0)."""
    f = freqs(n).astype(np.float64)
    k = np.stack(np.broadcast_arrays(f[:, None, None], f[None, :, None], f[None, None, :]))
    r = np.sqrt(kmag2(n).astype(np.float64))
    out = np.zeros_like(k)
    nz = r > 0
    out[:, nz] = k[:, nz] / r[nz]
    return out


def _weighted_unit_fields(n: int, edges, w: np.ndarray) -> np.ndarray:
    idx = bin_of_modes(n, edges)
    return np.stack([idft(np.where(idx == b, w, 0.0)).real for b in range(len(edges) - 1)])


def _multi_indices(p: int):
    return [a for a in itertools.product(range(p + 1), repeat=3) if sum(a) == p]


def fisher_blocks(n: int, edges, lmax: int):
    """(triplets, Ft [nt, ne, ne], Delta [nt, ne], T [nt], Nl [nt, ne]) for
    the triangle-valid triplets with closed triangles, by the separable
    sums (FP64)."""
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(n, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep].astype(np.float64)
    ells = list(range(0, lmax + 1, 2))
    ne = len(ells)
    npix2 = float(n) ** 6
    mu = mu_grid(n)
    L = {l: legendre(l, mu) for l in ells}
    H = _weighted_unit_fields(n, edges, np.ones((n, n, n)))
    HL = {l: _weighted_unit_fields(n, edges, L[l]) for l in ells}

    def tri(Fa, Fb, Fc):
        return npix2 * np.array([np.sum(Fa[a] * Fb[b] * Fc[c]) for a, b, c in trips])

    d33, x32, x31 = {}, {}, {}
    for i, l in enumerate(ells):
        for j, lp in enumerate(ells):
            d33[i, j] = tri(H, H, _weighted_unit_fields(n, edges, L[l] * L[lp]))
            x32[i, j] = tri(H, HL[lp], HL[l])
            x31[i, j] = tri(HL[lp], H, HL[l])
    # N_l = sum L_l(u2 . u3) through the tensor expansion of (u2 . u3)^p
    u = _unit_grid(n)
    cpow = {0: T.copy()}
    for p in (2, 4):
        if p > 2 * (lmax // 2) and p > 2:
            break
        acc = np.zeros(len(trips))
        nyq = np.abs(np.stack(np.broadcast_arrays(*(freqs(n)[ix] for ix in (
            np.s_[:, None, None], np.s_[None, :, None], np.s_[None, None, :]))))) == n // 2
        for al in _multi_indices(p):
            w = u[0] ** al[0] * u[1] ** al[1] * u[2] ** al[2]
            for ax in range(3):  # odd power of a Nyquist component: average of +-N/2 is zero
                if al[ax] % 2:
                    w = np.where(nyq[ax], 0.0, w)
            Hw = _weighted_unit_fields(n, edges, w)
            coef = math.factorial(p) / (math.factorial(al[0]) * math.factorial(al[1]) * math.factorial(al[2]))
            acc += coef * tri(H, Hw, Hw)
        cpow[p] = acc
    Nl = np.zeros((len(trips), ne))
    for i, l in enumerate(ells):
        if l == 0:
            Nl[:, i] = T
        elif l == 2:
            Nl[:, i] = 1.5 * cpow[2] - 0.5 * T
        else:
            Nl[:, i] = (35.0 * cpow[4] - 30.0 * cpow[2] + 3.0 * T) / 8.0
    Ft = np.zeros((len(trips), ne, ne))
    Delta = np.zeros((len(trips), ne))
    for t, (a, b, c) in enumerate(trips):
        case = _case(a, b, c)
        for i in range(ne):
            r = Nl[t, i] / T[t]
            Delta[t, i] = (1.0, 2.0, 1.0 + r, 2.0 * (1.0 + 2.0 * r))[case]
            for j in range(ne):
                if case == 0:
                    Ft[t, i, j] = d33[i, j][t]
                elif case == 1:
                    Ft[t, i, j] = 2.0 * d33[i, j][t]
                elif case == 2:
                    Ft[t, i, j] = d33[i, j][t] + x32[i, j][t]
                else:
                    Ft[t, i, j] = 2.0 * (d33[i, j][t] + x32[i, j][t] + x31[i, j][t])
    return trips, Ft, Delta, T, Nl


def numerators(delta: np.ndarray, box: float, edges, trips, lmax: int) -> np.ndarray:
    """nt [ne, nt] = (V^2/N_pix) sum_x G_a G_b g_{c,l} (eq. bk-num-ideal,
    separable form, without 1/Delta)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    npix, vol = float(n) ** 3, float(box) ** 3
    G0 = weighted_fields(d, edges, 0)
    out = []
    for l in range(0, lmax + 1, 2):
        Gl = G0 if l == 0 else weighted_fields(d, edges, l)
        out.append(vol * vol / npix * np.array([np.sum(G0[a] * G0[b] * Gl[c]) for a, b, c in trips]))
    return np.array(out)


def pinv_sym(F: np.ndarray, rcond: float = 1e-12) -> np.ndarray:
    """Pseudo-inverse of a symmetric matrix from its eigen-decomposition."""
    w, V = np.linalg.eigh(0.5 * (F + F.T))
    big = np.max(np.abs(w)) if w.size else 0.0
    inv = np.array([1.0 / x if abs(x) > rcond * big else 0.0 for x in w])
    return (V * inv[None, :]) @ V.T


def mixing(Ft: np.ndarray, Delta: np.ndarray, T: np.ndarray, lmax: int) -> np.ndarray:
    """R [nt, ne, ne] with b = R y, y_l = (2l+1) nt_l / T the eq. (ideal-bk)
    multipoles: R = Delta Ft^+ diag(T / (2l'+1))."""
    ells = np.arange(0, lmax + 1, 2)
    R = np.zeros_like(Ft)
    for t in range(Ft.shape[0]):
        R[t] = (Delta[t][:, None] * pinv_sym(Ft[t])) * (T[t] / (2 * ells + 1))[None, :]
    return R


def bispectrum_multipoles_fisher(delta: np.ndarray, box: float, edges, lmax: int = 2):
    """(triplets, b [ne, nt]) with the discrete ideal Fisher matrix."""
    d = np.asarray(delta, dtype=np.float64)
    trips, Ft, Delta, T, _ = fisher_blocks(d.shape[0], edges, lmax)
    nt = numerators(d, box, edges, trips, lmax)
    b = np.zeros_like(nt)
    for t in range(len(trips)):
        b[:, t] = Delta[t] * (pinv_sym(Ft[t]) @ nt[:, t])
    return trips, b


def _representatives(k: np.ndarray, n: int):
    """The integer vectors that represent mode k: each Nyquist component
    (|k_i| = N/2) as +N/2 and as -N/2."""
    opts = [(c, -c) if abs(c) == n // 2 else (c,) for c in k]
    return [np.array(v, dtype=np.float64) for v in itertools.product(*opts)]


def brute_blocks(n: int, edges, trips, lmax: int):
    """Ft, Delta-free N_l and T by explicit loops over closed triangles
    (small grids only): (Ft [nt, ne, ne], Nl [nt, ne], T [nt])."""
    if n > 10:
        raise ValueError("brute force is for N <= 10")
    idx = bin_of_modes(n, edges)
    f = freqs(n)
    ells = list(range(0, lmax + 1, 2))
    ne = len(ells)
    modes = [np.argwhere(idx == b) for b in range(len(edges) - 1)]

    def vec(i):
        return np.array([f[i[0]], f[i[1]], f[i[2]]], dtype=np.float64)

    Ft = np.zeros((len(trips), ne, ne))
    Nl = np.zeros((len(trips), ne))
    T = np.zeros(len(trips))
    for t, (a, b, c) in enumerate(trips):
        case = _case(a, b, c)
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = (-i1 - i2) % n
                if idx[tuple(i3)] != c:
                    continue
                k1, k2, k3 = vec(i1), vec(i2), vec(i3)
                r1, r2, r3 = (np.sqrt(k @ k) for k in (k1, k2, k3))
                m1, m2, m3 = k1[2] / r1, k2[2] / r2, k3[2] / r3
                T[t] += 1.0
                # N_l: average over the representatives +-N/2 of Nyquist components
                v2s, v3s = _representatives(k2, n), _representatives(k3, n)
                for i, l in enumerate(ells):
                    acc = 0.0
                    for v2 in v2s:
                        for v3 in v3s:
                            acc += legendre(l, (v2 @ v3) / (r2 * r3))
                    Nl[t, i] += acc / (len(v2s) * len(v3s))
                    for j, lp in enumerate(ells):
                        L3 = legendre(l, m3)
                        if case == 0:
                            P = legendre(lp, m3)
                        elif case == 1:
                            P = 2.0 * legendre(lp, m3)
                        elif case == 2:
                            P = legendre(lp, m3) + legendre(lp, m2)
                        else:
                            P = 2.0 * (legendre(lp, m1) + legendre(lp, m2) + legendre(lp, m3))
                        Ft[t, i, j] += L3 * P
    return Ft, Nl, T


def brute_numerators(delta: np.ndarray, box: float, edges, trips, lmax: int) -> np.ndarray:
    """nt [ne, nt] by explicit loops (small grids only)."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if n > 10:
        raise ValueError("brute force is for N <= 10")
    D = dft(d)
    idx = bin_of_modes(n, edges)
    f = freqs(n)
    npix, vol = float(n) ** 3, float(box) ** 3
    modes = [np.argwhere(idx == b) for b in range(len(edges) - 1)]
    ells = list(range(0, lmax + 1, 2))
    out = np.zeros((len(ells), len(trips)))
    for t, (a, b, c) in enumerate(trips):
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = (-i1 - i2) % n
                if idx[tuple(i3)] != c:
                    continue
                k3 = np.array([f[i3[0]], f[i3[1]], f[i3[2]]], dtype=np.float64)
                m3 = k3[2] / np.sqrt(k3 @ k3)
                prod = (D[tuple(i1)] * D[tuple(i2)] * D[tuple(i3)]).real
                for i, l in enumerate(ells):
                    out[i, t] += legendre(l, m3) * prod
    return vol * vol / npix**3 * out
