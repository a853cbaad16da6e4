"""FP64 oracle for the masked power spectrum with a Monte Carlo Fisher matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Setting (Sec. II.C and Sec. III.C): data d = w * delta on the periodic
N^3 grid, with the window w as the pointing matrix, unit weighting
(S^-1 = I), a global line of sight and l = 0.  The Q derivative maps are
then Q_b[u](n) = Theta_b(n) u(n) in Fourier space (eq. Q-alpha-global).

Discrete normalisation used throughout (numpy DFT conventions, D = DFT,
d = IDFT with 1/N_pix):

* numerator   p_b = (1/2) (V/N_pix^2) sum_{n in b} |D_d(n)|^2
                  = (1/2) N_b P_box_b(d);
* Fisher      F_ab = (1/2) <sum_n conj(V_a(n)) Theta_b(n) A(n)>_a / N_pix
  with A = DFT[a] for white unit-variance fields a (so A^-1 = I and
  <|A(n)|^2> = N_pix) and V_a = DFT[w IDFT[Theta_a DFT[w a]]]: the
  Girard-Hutchinson form of eq. (fish-from-Q) with P = w, S^-1 = I;
* estimate    P_unw = F^-1 p.

With w = 1 the Fisher matrix is (1/2) diag(N_b) exactly in expectation and
P_unw reduces to the box estimator.

The bispectrum's linear term (eq. b-numerator-practical) is averaged over
fields Delta with covariance close to the data's (simulations through the
same window); it vanishes in expectation and lowers the variance where the
window breaks translation invariance.
"""

from __future__ import annotations

import numpy as np

from .polyspec import bin_of_modes, dft, idft, power_spectrum, triangle_counts, triangle_triplets, unit_fields


def mc_fisher_power(w: np.ndarray, grfs, edges) -> np.ndarray:
    """Monte Carlo Fisher matrix from the given white unit-variance fields,
    following the paper's steps: filter the random map by the pointing
    matrix (w a) and by A^-1 (identity here); for every bin apply
    Q_a in Fourier space, weight by P^dagger S^-dagger = w and transform;
    dot with Q^asym_b[A^-1 a] = Theta_b DFT[a] as a Fourier-space sum."""
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    npix = float(n) ** 3
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    F = np.zeros((nb, nb))
    grfs = list(grfs)
    for a in grfs:
        a = np.asarray(a, dtype=np.float64)
        Wa = dft(w * a)
        A = dft(a)
        Qasym = [np.where(idx == b, A, 0.0) for b in range(nb)]
        for ia in range(nb):
            qa = idft(np.where(idx == ia, Wa, 0.0)).real  # Q_a[P a] in real space
            Va = dft(w * qa)  # weighted by P^dagger S^-dagger, back to Fourier space
            for ib in range(nb):
                F[ia, ib] += 0.5 * np.real(np.sum(np.conj(Va) * Qasym[ib])) / npix
    return F / len(grfs)


def fisher_power_exact(w: np.ndarray, edges) -> np.ndarray:
    """Expectation of :func:`mc_fisher_power` over white fields:
    F_ab = (1/2) sum_r xi_w(r) H_a(r) H_b(r), with xi_w(r) = sum_x w(x) w(x+r)
    the window's autocorrelation and H_b = IDFT[Theta_b]."""
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    W = dft(w)
    xi = idft(W.real * W.real + W.imag * W.imag).real
    H = unit_fields(n, edges)
    nb = len(edges) - 1
    Hf = H.reshape(nb, -1)
    return 0.5 * (Hf * xi.reshape(1, -1)) @ Hf.T


def unwindowed_power(data: np.ndarray, box: float, edges, fisher: np.ndarray) -> np.ndarray:
    """P_unw = F^-1 p with p_b = (1/2) N_b P_box_b(data)."""
    n = np.asarray(data).shape[0]
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    nm = np.array([np.count_nonzero(idx == b) for b in range(nb)], dtype=np.float64)
    p = 0.5 * nm * power_spectrum(data, box, edges)
    return np.linalg.solve(fisher, p)


def bispectrum_linear(data: np.ndarray, sims, box: float, edges):
    """Bispectrum with the linear term of eq. (b-numerator-practical), unit
    weighting, normalised like the ideal estimator (divide by <w^3> for the
    windowed form):

        B = (V^2/N_pix) [S(d) - (1/n_sim) sum_i S_lin(d; Delta_i)] / T,
        S(d)  = sum_x G_a[d] G_b[d] G_c[d],
        S_lin = sum_x (G_a[d] G_b[D] G_c[D] + G_a[D] G_b[d] G_c[D] + G_a[D] G_b[D] G_c[d]),

    the linear term being the Monte Carlo average over the given fields
    Delta_i (covariance close to the data's).  Returns (triplets with T > 0,
    B with the term, B without it, A = same normalisation of
    sum_x |G_a G_b G_c| + the mean of the three |mixed| sums)."""
    d = np.asarray(data, dtype=np.float64)
    n = d.shape[0]
    npix, vol = float(n) ** 3, float(box) ** 3
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(n, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep]
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1

    def fields(f):
        F = dft(np.asarray(f, dtype=np.float64))
        return np.stack([idft(np.where(idx == b, F, 0.0)).real for b in range(nb)])

    Gd = fields(d)
    s = np.array([np.sum(Gd[a] * Gd[b] * Gd[c]) for a, b, c in trips])
    sa = np.array([np.sum(np.abs(Gd[a] * Gd[b] * Gd[c])) for a, b, c in trips])
    lin = np.zeros(len(trips))
    la = np.zeros(len(trips))
    sims = list(sims)
    for sim in sims:
        Ge = fields(sim)
        for t, (a, b, c) in enumerate(trips):
            x1, x2, x3 = Gd[a] * Ge[b] * Ge[c], Ge[a] * Gd[b] * Ge[c], Ge[a] * Ge[b] * Gd[c]
            lin[t] += np.sum(x1) + np.sum(x2) + np.sum(x3)
            la[t] += np.sum(np.abs(x1)) + np.sum(np.abs(x2)) + np.sum(np.abs(x3))
    lin /= len(sims)
    la /= len(sims)
    fac = vol * vol / npix / T
    return trips, (s - lin) * fac, s * fac, (sa + la) * fac


def brute_linear_sum(data: np.ndarray, sim: np.ndarray, edges, trips) -> np.ndarray:
    """sum over closed mode triangles of D1 E2 E3 + E1 D2 E3 + E1 E2 D3 with
    D = DFT[data], E = DFT[sim], by explicit loops (N <= 8)."""
    d = np.asarray(data, dtype=np.float64)
    n = d.shape[0]
    if n > 8:
        raise ValueError("brute force is for N <= 8")
    D, E = dft(d), dft(np.asarray(sim, dtype=np.float64))
    idx = bin_of_modes(n, edges)
    modes = [np.argwhere(idx == b) for b in range(len(edges) - 1)]
    out = np.zeros(len(trips), dtype=np.complex128)
    for t, (a, b, c) in enumerate(trips):
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = tuple((-i1 - i2) % n)
                if idx[i3] != c:
                    continue
                j1, j2 = tuple(i1), tuple(i2)
                out[t] += D[j1] * E[j2] * E[i3] + E[j1] * D[j2] * E[i3] + E[j1] * E[j2] * D[i3]
    return out
