"""FP64 oracle for non-cubic grids and boxes: Nx x Ny x Nz cells on a box of
sides Lx x Ly x Lz (Sec. III.D and Sec. IV.D in their ideal limits; the
paper's estimators are written for any geometry and its own survey grids
are non-cubic, Sec. VI.A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (generalising those of ``polyspec`` axis by axis):

* n_i in numpy ``fftfreq(N_i) * N_i`` order, k_i = k_f,i n_i with
  k_f,i = 2 pi / L_i; N_pix = Nx Ny Nz, V = Lx Ly Lz;
* cubic box (Lx = Ly = Lz): bins in units of k_f decided on the integer
  |n|^2, exactly as in ``polyspec`` (any grid shape);
* other boxes: bins in h/Mpc, decided on the FP64 value
  k^2 = (k_f,x^2 nx^2 + k_f,y^2 ny^2) + k_f,z^2 nz^2 with k_f,i^2 = (2 pi / L_i)^2,
  evaluated in exactly that order (the library uses the same expression, so
  both sides put every mode in the same bin);
* P_b = (V/N_pix^2) (1/N_b) sum_{n in b} |D(n)|^2,
  B_abc = (V^2/N_pix) sum_x G_a G_b G_c / T_abc, T_abc = N_pix^2 sum_x H_a H_b H_c,
  closure n1 + n2 + n3 = 0 modulo N_i on every axis.
"""

from __future__ import annotations

import numpy as np

from .polyspec import Result, _triple_sums, dft, idft, triangle_triplets


def _freqs(n: int) -> np.ndarray:
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def cubic_box(box) -> bool:
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    return bool(b[0] == b[1] == b[2])


def _box3(box) -> np.ndarray:
    return np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()


def kmag2_int(shape) -> np.ndarray:
    """Integer |n|^2 on the full grid of the given shape (int64)."""
    fx, fy, fz = (_freqs(n) for n in shape)
    return fx[:, None, None] ** 2 + fy[None, :, None] ** 2 + fz[None, None, :] ** 2


def kmag2_phys(shape, box) -> np.ndarray:
    """k^2 in (h/Mpc)^2 on the full grid, in the order stated above."""
    L = _box3(box)
    kf2 = [(2.0 * np.pi / L[i]) * (2.0 * np.pi / L[i]) for i in range(3)]
    fx, fy, fz = (_freqs(n).astype(np.float64) for n in shape)
    tx = kf2[0] * (fx * fx)
    ty = kf2[1] * (fy * fy)
    tz = kf2[2] * (fz * fz)
    return (tx[:, None, None] + ty[None, :, None]) + tz[None, None, :]


def bin_of_modes(shape, box, edges) -> np.ndarray:
    """Bin index of every mode (-1 outside): integer |n|^2 against k_f-unit
    edges for a cubic box, FP64 k^2 against h/Mpc edges otherwise."""
    e = np.asarray(edges, dtype=np.float64)
    if np.any(np.diff(e) <= 0) or e[0] < 0:
        raise ValueError("bin edges must be non-negative and strictly increasing")
    e2 = e * e
    k2 = kmag2_int(shape).astype(np.float64) if cubic_box(box) else kmag2_phys(shape, box)
    idx = np.searchsorted(e2, k2, side="right") - 1
    idx[(k2 < e2[0]) | (k2 >= e2[-1])] = -1
    return idx


def mode_counts(shape, box, edges) -> np.ndarray:
    idx = bin_of_modes(shape, box, edges)
    return np.bincount(idx[idx >= 0].ravel(), minlength=len(edges) - 1).astype(np.int64)


def power_spectrum(delta, box, edges) -> np.ndarray:
    d = np.asarray(delta, dtype=np.float64)
    npix = float(d.size)
    vol = float(np.prod(_box3(box)))
    D = dft(d)
    p2 = D.real * D.real + D.imag * D.imag
    idx = bin_of_modes(d.shape, box, edges)
    nb = len(edges) - 1
    out = np.zeros(nb)
    for b in range(nb):
        m = idx == b
        if not m.any():
            raise ValueError("a bin contains no grid modes")
        out[b] = p2[m].sum() / m.sum()
    return vol / npix**2 * out


def filtered_fields(delta, box, edges) -> np.ndarray:
    d = np.asarray(delta, dtype=np.float64)
    D = dft(d)
    idx = bin_of_modes(d.shape, box, edges)
    return np.stack([idft(np.where(idx == b, D, 0.0)).real for b in range(len(edges) - 1)])


def unit_fields(shape, box, edges) -> np.ndarray:
    idx = bin_of_modes(shape, box, edges)
    return np.stack([idft((idx == b).astype(np.float64)).real for b in range(len(edges) - 1)])


def triangle_counts(shape, box, edges, trips=None):
    """T_abc (int64) and the raw FP64 sum."""
    trips = triangle_triplets(edges) if trips is None else np.asarray(trips)
    H = unit_fields(shape, box, edges)
    raw, _ = _triple_sums(H, trips)
    raw *= float(np.prod(shape)) ** 2
    return np.rint(raw).astype(np.int64), raw


def bispectrum(delta, box, edges) -> Result:
    """Ideal-limit P and B on the given geometry, triplets with T > 0."""
    d = np.asarray(delta, dtype=np.float64)
    npix = float(d.size)
    vol = float(np.prod(_box3(box)))
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(d.shape, box, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep]
    G = filtered_fields(d, box, edges)
    s, sa = _triple_sums(G, trips, absolute=True)
    scale = vol * vol / npix
    return Result(trips, scale * s / T, T, scale * sa / T, power_spectrum(d, box, edges),
                  mode_counts(d.shape, box, edges))


def brute_sums(delta, box, edges, trips):
    """sum over closed mode triangles of D1 D2 D3 and their number, by explicit
    loops (small grids only)."""
    d = np.asarray(delta, dtype=np.float64)
    if d.size > 12 ** 3:
        raise ValueError("brute force is for small grids")
    shape = np.array(d.shape)
    D = dft(d)
    idx = bin_of_modes(d.shape, box, edges)
    modes = [np.argwhere(idx == b) for b in range(len(edges) - 1)]
    s = np.zeros(len(trips), dtype=np.complex128)
    cnt = np.zeros(len(trips), dtype=np.int64)
    for t, (a, b, c) in enumerate(trips):
        for i1 in modes[a]:
            for i2 in modes[b]:
                i3 = tuple((-i1 - i2) % shape)
                if idx[i3] == c:
                    s[t] += D[tuple(i1)] * D[tuple(i2)] * D[i3]
                    cnt[t] += 1
    return s, cnt


# ------------------------------------------------------------ multipoles
# Line of sight along z; mu = k_z / |k| with the physical wave-vector.  The
# estimators are those of ``oracle.multipoles`` (discrete Fisher matrix for
# P, (2l+1)/T with the Legendre weight on k_3 for B).


def mu2_grid(shape, box) -> np.ndarray:
    """mu^2 = k_z^2 / k^2 on the full grid (0 at k = 0)."""
    L = _box3(box)
    fx, fy, fz = (_freqs(n).astype(np.float64) for n in shape)
    # k^2 / k_f,z^2 with the axis scales k_f,i^2 / k_f,z^2
    sx = (L[2] / L[0]) ** 2
    sy = (L[2] / L[1]) ** 2
    den = sx * fx[:, None, None] ** 2 + sy * fy[None, :, None] ** 2 + fz[None, None, :] ** 2
    num = np.broadcast_to(fz[None, None, :] ** 2, den.shape)
    out = np.zeros(den.shape)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def _legendre_m2(ell: int, m2: np.ndarray) -> np.ndarray:
    if ell == 0:
        return np.ones_like(m2)
    if ell == 2:
        return 1.5 * m2 - 0.5
    if ell == 4:
        return (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0
    raise ValueError("ell must be 0, 2 or 4")


def power_multipoles(delta, box, edges, lmax: int = 4) -> np.ndarray:
    d = np.asarray(delta, dtype=np.float64)
    npix, vol = float(d.size), float(np.prod(_box3(box)))
    D = dft(d)
    p2 = D.real * D.real + D.imag * D.imag
    idx = bin_of_modes(d.shape, box, edges)
    m2 = mu2_grid(d.shape, box)
    ells = list(range(0, lmax + 1, 2))
    L = np.stack([_legendre_m2(l, m2) for l in ells])
    out = np.zeros((len(ells), len(edges) - 1))
    for b in range(len(edges) - 1):
        m = idx == b
        Lb = L[:, m]
        out[:, b] = np.linalg.solve(Lb @ Lb.T, vol / npix**2 * (Lb * p2[m][None, :]).sum(axis=1))
    return out


def bispectrum_multipoles(delta, box, edges, lmax: int = 2):
    """(triplets, B [lmax/2 + 1, n_trip], A [lmax/2 + 1, n_trip]) with A the
    same normalisation of sum_x |G_a G_b g_{c,l}|."""
    d = np.asarray(delta, dtype=np.float64)
    npix, vol = float(d.size), float(np.prod(_box3(box)))
    trips = triangle_triplets(edges)
    T, _ = triangle_counts(d.shape, box, edges, trips)
    keep = T > 0
    trips, T = trips[keep], T[keep]
    D = dft(d)
    idx = bin_of_modes(d.shape, box, edges)
    m2 = mu2_grid(d.shape, box)
    nb = len(edges) - 1
    G0 = np.stack([idft(np.where(idx == b, D, 0.0)).real for b in range(nb)])
    out, absn = [], []
    for ell in range(0, lmax + 1, 2):
        Dl = _legendre_m2(ell, m2) * D
        Gl = G0 if ell == 0 else np.stack([idft(np.where(idx == b, Dl, 0.0)).real for b in range(nb)])
        s = np.array([np.sum(G0[a] * G0[b] * Gl[c]) for a, b, c in trips])
        sa = np.array([np.sum(np.abs(G0[a] * G0[b] * Gl[c])) for a, b, c in trips])
        out.append((2 * ell + 1) * vol * vol / npix * s / T)
        absn.append((2 * ell + 1) * vol * vol / npix * sa / T)
    return trips, np.array(out), np.array(absn)
