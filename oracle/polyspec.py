"""FP64 CPU oracle for the idealized (periodic-box) binned power spectrum and
bispectrum of PolyBin3D (Philcox & Floss, arXiv:2404.07249).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares
no code with the HIP path and must never be reached from the product path.

Everything is float64 NumPy/SciPy; the FFT is a library primitive used as a
step, with no blocking, fusion or reordering beyond the definitions below.

Conventions (discrete form of the Fourier conventions stated at the end of
Sec. I):

* grid side N, N_pix = N^3, box side L, volume V = L^3, k_f = 2 pi / L;
* integer wave-vector n with components in numpy ``fftfreq(N)*N`` order,
  |k| = k_f |n|;
* D(n) = sum_x d(x) exp(-2 pi i n.x / N) (unnormalised DFT); the continuum
  FT is d(k) ~ (V/N_pix) D(n) and int_k -> (1/V) sum_n;
* bins are half-open shells [e_b, e_{b+1}) in units of k_f, decided on the
  integer |n|^2 (the paper recommends integer-k_f binning to avoid
  floating-point edge ties, Sec. VI.A.3, Code Comparison footnote);
* Theta_b(n) = [e_b^2 <= |n|^2 < e_{b+1}^2], N_b = sum_n Theta_b(n).

Definitions (ell = 0, global line of sight, P_fid = m = nbar = 1, which is
the ideal limit of Sec. III.D.1 and Sec. IV.D.1):

* power  P_b  = (V / N_pix^2) (1/N_b) sum_n Theta_b |D(n)|^2
  -- eq. (pk-limit) numerator over the discrete Fisher (the bin volume,
  eq. fish-ideal-continuous), with the box volume V restored so that
  <P_b> equals the input power spectrum.
* filtered field  G_b(x) = IDFT[Theta_b D](x)  (numpy 1/N_pix normalisation)
  -- eq. (g-ell-def) at ell = 0 (the conjugate is immaterial for real d).
* unit field      H_b(x) = IDFT[Theta_b](x).
* triangle count  T_abc = N_pix^2 sum_x H_a H_b H_c, an exact integer equal
  to #{(n1,n2,n3): n_i in bin, n1+n2+n3 = 0 (mod N)} -- N_0 of
  eq. (N-ell-def) evaluated by the separable real-space sum of Sec. IV.C.1.
* bispectrum B_abc = (V^2/N_pix) sum_x G_a G_b G_c / T_abc
  = (V^2/N_pix^3) (1/T) sum_{closed} D(n1) D(n2) D(n3)
  -- the ideal estimator, eq. (ideal-bk) and the closing estimator of
  Sec. IV.D.1 (Delta_alpha and 2l+1 cancel between eq. bk-num-ideal and
  eq. bk-fish-ideal2); the separable form is eq. (beta-def).
* triplets: a <= b <= c with e_c < e_{a+1} + e_{b+1} (some closed triangle
  exists inside the three shells), ordered with c fastest, then b, then a
  (the plotting order of Sec. VI.B.2).  This reading reproduces the 196
  configurations (98 per multipole) printed for 8 bins in Sec. VI.B.1.
  Triplets with T_abc = 0 on the lattice have no estimate and are dropped.
"""

from __future__ import annotations

import math
import os

import concurrent.futures as _cf

import threadpoolctl as _tpc

import numpy as np

try:  # scipy's pocketfft takes a worker count; numpy's does not
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None

__all__ = [
    "freqs",
    "kmag2",
    "bin_of_modes",
    "mode_counts",
    "triangle_triplets",
    "dft",
    "idft",
    "power_spectrum",
    "filtered_fields",
    "unit_fields",
    "triangle_counts",
    "bispectrum",
    "triple_sums",
    "Result",
]


def _workers() -> int:
    return int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


def dft(x: np.ndarray) -> np.ndarray:
    """Unnormalised forward 3D DFT in float64/complex128 (library step)."""
    x = np.asarray(x, dtype=np.float64)
    if _sfft is not None:
        return _sfft.fftn(x, workers=_workers())
    return np.fft.fftn(x)


def idft(x: np.ndarray) -> np.ndarray:
    """Inverse 3D DFT with 1/N_pix normalisation (library step)."""
    if _sfft is not None:
        return _sfft.ifftn(x, workers=_workers())
    return np.fft.ifftn(x)


def rdft(x: np.ndarray) -> np.ndarray:
    """The k_z = 0..n/2 half of the unnormalised 3D DFT of real data (library step)."""
    x = np.asarray(x, dtype=np.float64)
    if _sfft is not None:
        return _sfft.rfftn(x, workers=_workers())
    return np.fft.rfftn(x)


def irdft(x: np.ndarray, n: int) -> np.ndarray:
    """Real inverse 3D DFT (1/N_pix normalisation) of a Hermitian spectrum
    given by its k_z = 0..n/2 half, on an n^3 grid (library step)."""
    if _sfft is not None:
        return _sfft.irfftn(x, s=(n, n, n), workers=_workers())
    return np.fft.irfftn(x, s=(n, n, n))


def freqs(n: int) -> np.ndarray:
    """Integer wave numbers of an n-point DFT, in [-n/2, n/2)."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def kmag2(n: int) -> np.ndarray:
    """Integer |n|^2 on the full n^3 Fourier grid (int64)."""
    f = freqs(n)
    return f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2


def _edge_squares(edges) -> np.ndarray:
    e = np.asarray(edges, dtype=np.float64)
    if e.ndim != 1 or e.size < 2:
        raise ValueError("need at least two bin edges")
    if np.any(np.diff(e) <= 0) or e[0] < 0:
        raise ValueError("bin edges must be non-negative and strictly increasing")
    return e * e


def bin_of_modes(n: int, edges) -> np.ndarray:
    """Bin index of every mode (-1 outside all bins): e_b^2 <= |n|^2 < e_{b+1}^2."""
    k2 = kmag2(n).astype(np.float64)  # exact for |n|^2 < 2^53
    e2 = _edge_squares(edges)
    idx = np.searchsorted(e2, k2, side="right") - 1
    idx[(k2 < e2[0]) | (k2 >= e2[-1])] = -1
    return idx


def mode_counts(n: int, edges) -> np.ndarray:
    """N_b: number of grid modes in each bin (int64)."""
    nb = len(edges) - 1
    idx = bin_of_modes(n, edges)
    return np.bincount(idx[idx >= 0].ravel(), minlength=nb).astype(np.int64)


def triangle_triplets(edges) -> np.ndarray:
    """All (a, b, c), a <= b <= c, with e_c < e_{a+1} + e_{b+1}; c fastest."""
    e = np.asarray(edges, dtype=np.float64)
    nb = e.size - 1
    out = []
    for a in range(nb):
        for b in range(a, nb):
            for c in range(b, nb):
                if e[c] < e[a + 1] + e[b + 1]:
                    out.append((a, b, c))
    return np.asarray(out, dtype=np.int64).reshape(-1, 3)


def power_spectrum(delta: np.ndarray, box: float, edges) -> np.ndarray:
    """P_b = (V/N_pix^2) (1/N_b) sum_{n in b} |D(n)|^2, float64 per bin."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if d.shape != (n, n, n):
        raise ValueError("cubic grid required")
    npix = float(n) ** 3
    vol = float(box) ** 3
    D = dft(d)
    p2 = (D.real * D.real + D.imag * D.imag)
    idx = bin_of_modes(n, edges)
    nb = len(edges) - 1
    sums = np.zeros(nb)
    cnt = np.zeros(nb, dtype=np.int64)
    for b in range(nb):
        m = idx == b
        cnt[b] = int(m.sum())
        sums[b] = p2[m].sum()
    if np.any(cnt == 0):
        raise ValueError("a bin contains no grid modes")
    return vol / npix**2 * sums / cnt


def _half(x: np.ndarray) -> np.ndarray:
    """The k_z >= 0 half (k_z = 0..n/2) of a full n^3 Fourier-grid array."""
    return x[:, :, : x.shape[2] // 2 + 1]


def filtered_fields(delta: np.ndarray, edges, bins=None) -> np.ndarray:
    """G_b = Re IDFT[Theta_b D] for b in ``bins`` (all bins by default).

    Theta_b D is Hermitian for real delta (Theta_b depends on |n| only), so
    its inverse DFT is real and is taken from the k_z >= 0 half by the
    library's real inverse transform."""
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    D = rdft(d)
    idx = _half(bin_of_modes(n, edges))
    nb = len(edges) - 1
    bins = range(nb) if bins is None else bins
    return np.stack([irdft(D * (idx == b), n) for b in bins])


def unit_fields(n: int, edges, bins=None) -> np.ndarray:
    """H_b = Re IDFT[Theta_b] for b in ``bins`` (all bins by default), via
    the real inverse transform of the k_z >= 0 half as above."""
    idx = _half(bin_of_modes(n, edges))
    nb = len(edges) - 1
    bins = range(nb) if bins is None else bins
    return np.stack([irdft((idx == b).astype(np.float64), n) for b in bins])


def triple_sums(fields: np.ndarray, trips: np.ndarray, absolute: bool = False):
    """sum_x F_a F_b F_c for each triplet (and optionally sum_x |F_a F_b F_c|)."""
    return _triple_sums(fields, trips, absolute)


def _triple_sums(fields: np.ndarray, trips: np.ndarray, absolute: bool = False, chunk: int = 4096):
    """sum_x F_a F_b F_c for each triplet (and optionally sum_x |F_a F_b F_c|).

    The voxel sum is taken over contiguous chunks of voxels.  In a chunk
    every pair product F_a F_b the triplets use is formed once (rows of P),
    and S = P F^T (a matrix product) holds sum_x F_a F_b F_c for every such
    pair and every bin c, of which the triplets' entries are taken; the
    chunk sums are added in voxel order.  Chunks are evaluated by a thread
    pool (each writes only its own row of partial sums), so the result does
    not depend on the threads.
    """
    nb = fields.shape[0]
    flat = fields.reshape(nb, -1)
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    pairs = sorted(set((int(a), int(b)) for a, b, _ in trips))
    pid = {p: i for i, p in enumerate(pairs)}
    pa = np.array([p[0] for p in pairs], dtype=np.int64)
    pb = np.array([p[1] for p in pairs], dtype=np.int64)
    rows = np.array([pid[(int(a), int(b))] for a, b, _ in trips], dtype=np.int64)
    cols = trips[:, 2]
    starts = list(range(0, flat.shape[1], chunk))
    part = np.zeros((len(starts), len(trips)))
    parta = np.zeros((len(starts), len(trips))) if absolute else None

    def one(k):
        f = np.ascontiguousarray(flat[:, starts[k]:starts[k] + chunk])
        P = f[pa] * f[pb]
        part[k] = (P @ f.T)[rows, cols]
        if absolute:
            parta[k] = (np.abs(P) @ np.abs(f).T)[rows, cols]

    with _tpc.threadpool_limits(1), _cf.ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(one, range(len(starts))))
    s = np.zeros(len(trips))
    sa = np.zeros(len(trips)) if absolute else None
    for k in range(len(starts)):
        s += part[k]
        if absolute:
            sa += parta[k]
    return s, sa


def triangle_counts(n: int, edges, trips=None) -> tuple[np.ndarray, np.ndarray]:
    """T_abc (exact integers, int64) and the raw float64 value before rounding."""
    trips = triangle_triplets(edges) if trips is None else np.asarray(trips)
    H = unit_fields(n, edges)
    raw, _ = _triple_sums(H, trips)
    raw *= float(n) ** 6
    return np.rint(raw).astype(np.int64), raw


class Result:
    """Bundle returned by :func:`bispectrum`."""

    def __init__(self, trips, bk, counts, absnorm, pk, n_modes):
        self.triplets = trips  # (n_trip, 3) int64, the valid (T > 0) triplets
        self.bk = bk  # (n_trip,) float64, (Mpc/h)^6
        self.counts = counts  # (n_trip,) int64, T_abc
        self.absnorm = absnorm  # (n_trip,) float64, same normalisation of sum|G G G|
        self.pk = pk  # (n_bins,) float64, (Mpc/h)^3
        self.n_modes = n_modes  # (n_bins,) int64

    @property
    def kappa(self):
        """Conditioning A/|B| of each bispectrum bin."""
        with np.errstate(divide="ignore"):
            return self.absnorm / np.abs(self.bk)


def bispectrum(delta: np.ndarray, box: float, edges, trips=None, counts=None) -> Result:
    """Ideal-limit binned bispectrum (ell = 0) of a real periodic field.

    B_abc = (V^2/N_pix) sum_x G_a G_b G_c / T_abc for every triangle-valid
    triplet with T_abc > 0.  ``counts`` may pass precomputed T (they do not
    depend on the data, Sec. IV.D.1).
    """
    d = np.asarray(delta, dtype=np.float64)
    n = d.shape[0]
    if d.shape != (n, n, n):
        raise ValueError("cubic grid required")
    nb = len(edges) - 1
    nm = mode_counts(n, edges)
    if np.any(nm == 0):
        raise ValueError("a bin contains no grid modes")
    all_trips = triangle_triplets(edges) if trips is None else np.asarray(trips)
    if counts is None:
        counts, _ = triangle_counts(n, edges, all_trips)
    keep = counts > 0
    trips_k = all_trips[keep]
    T = counts[keep]
    npix = float(n) ** 3
    vol = float(box) ** 3
    G = filtered_fields(d, edges)
    s, sa = _triple_sums(G, trips_k, absolute=True)
    scale = vol * vol / npix
    bk = scale * s / T
    A = scale * sa / T
    pk = power_spectrum(d, box, edges)
    assert pk.shape == (nb,)
    return Result(trips_k, bk, T, A, pk, nm)


def triplet_sums_sample(delta: np.ndarray, edges, trips) -> np.ndarray:
    """sum_x G_a G_b G_c for a (small) list of triplets, computing only the
    filtered fields those triplets touch.  Used to check large grids on a
    sample of outputs."""
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    need = sorted(set(int(v) for v in trips.ravel()))
    G = filtered_fields(delta, edges, bins=need)
    pos = {b: i for i, b in enumerate(need)}
    remap = np.array([[pos[int(v)] for v in t] for t in trips], dtype=np.int64)
    s, sa = _triple_sums(G, remap, absolute=True)
    return s, sa


def count_sample(n: int, edges, trips) -> np.ndarray:
    """T_abc for a (small) list of triplets via the unit fields they touch."""
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    need = sorted(set(int(v) for v in trips.ravel()))
    H = unit_fields(n, edges, bins=need)
    pos = {b: i for i, b in enumerate(need)}
    remap = np.array([[pos[int(v)] for v in t] for t in trips], dtype=np.int64)
    raw, _ = _triple_sums(H, remap)
    return np.rint(raw * float(n) ** 6).astype(np.int64)


def max_component(edges) -> int:
    """Largest integer |n_i| any mode inside the top edge can have."""
    e_top = float(np.asarray(edges, dtype=np.float64)[-1])
    k = int(math.floor(e_top))
    if k * k >= e_top * e_top:
        k -= 1
    return max(k, 0)


# ------------------------------------------------------------------ masked
def window_moments(w: np.ndarray) -> tuple[float, float]:
    """Means of w^2 and w^3 over the grid (float64)."""
    w = np.asarray(w, dtype=np.float64)
    return float(np.mean(w * w)), float(np.mean(w * w * w))


def windowed_polyspectra(data: np.ndarray, w: np.ndarray, box: float, edges):
    """Conventional windowed estimators for masked data d = w * delta: the
    box estimators of d divided by <w^2> (power) and <w^3> (bispectrum).
    These are the FKP-limit forms of Sec. III.D.2 (normalisation by the
    integral of n^2) and Sec. IV.D.2 (by the integral of n^3), with uniform
    weights and the linear and noise terms dropped.  Returns
    (P, B, (<w^2>, <w^3>), Result of the unnormalised box estimator)."""
    res = bispectrum(np.asarray(data, dtype=np.float64), box, edges)
    m2, m3 = window_moments(w)
    return res.pk / m2, res.bk / m3, (m2, m3), res
