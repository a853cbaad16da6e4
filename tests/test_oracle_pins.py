"""Pins for two oracle routines that previously had none: the pixel window
of the weighted estimators, checked against actual mass assignment, and the
sampled triplet sums / counts used by the large-grid GPU checks, checked
against the full estimator.  Each test also shows that a plausible mistake
(wrong argument or exponent, shuffled bin remap) fails it.
"""

import numpy as np
import pytest

import oracle
import oracle.polyspec as ps
from oracle import weighted as wt
from synthetic import kf_edges, quadratic_field

# ------------------------------------------------------------ pixel window
# The paper leaves the window m(k) general (Sec. III.D.1).  The weighted
# oracle uses m(n) = prod_i sinc(pi n_i / N)^p for nearest-grid-point (p = 1),
# cloud-in-cell (p = 2) and triangular-shaped-cloud (p = 3) assignment.  Here
# the assignment kernels are written out and the window is measured: a
# particle at x0 (cell units) puts W_p(c - x0) on grid point c, so the DFT of
# its density, phase-referred to the particle, is
#   sum_c W_p(c - x0) exp(-2 pi i n (c - x0) / N),
# and its average over the particle's position inside one cell is the window.


def _w_ngp(u):
    return ((u >= -0.5) & (u < 0.5)).astype(np.float64)


def _w_cic(u):
    return np.maximum(0.0, 1.0 - np.abs(u))


def _w_tsc(u):
    a = np.abs(u)
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


_KERNELS = {1: _w_ngp, 2: _w_cic, 3: _w_tsc}


def _measured_window(n_modes, N, order):
    """Average over x0 in [0, 1) of sum_c W(c - x0) e^{-2 pi i n (c - x0)/N},
    by Gauss-Legendre quadrature on [0, 1/2) and [1/2, 1), the pieces on
    which every kernel above is a polynomial in x0."""
    xg, wg = np.polynomial.legendre.leggauss(24)
    x0 = np.concatenate([0.25 + 0.25 * xg, 0.75 + 0.25 * xg])
    w0 = np.concatenate([0.25 * wg, 0.25 * wg])
    cells = np.arange(-3, 5)  # covers the support of every kernel for x0 in [0, 1)
    u = cells[None, :] - x0[:, None]
    W = _KERNELS[order](u)
    out = []
    for n in n_modes:
        ph = np.exp(-2j * np.pi * n * u / N)
        out.append(np.sum(w0 * np.sum(W * ph, axis=1)))
    return np.array(out)


@pytest.mark.parametrize("N", [16, 24, 48])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_window_equals_mass_assignment_average(N, order):
    n = ps.freqs(N).astype(np.int64)  # includes the Nyquist index -N/2
    meas = _measured_window(n, N, order)
    assert np.max(np.abs(meas.imag)) < 1e-13  # symmetric kernels: real window
    m1 = wt.window(N, order)[:, 0, 0]  # the oracle's window along x (n_y = n_z = 0)
    assert np.max(np.abs(m1 - meas.real)) < 1e-12
    # separable: the 3D window is the product of the per-axis measured ones
    m3 = wt.window(N, order)
    rng = np.random.default_rng(N + order)
    for _ in range(20):
        i, j, k = rng.integers(0, N, size=3)
        assert abs(m3[i, j, k] - meas[i].real * meas[j].real * meas[k].real) < 1e-12
    # a wrong argument or exponent is caught by the same comparison
    wrong_arg = np.sinc(n / (2.0 * N)) ** order
    wrong_exp = np.sinc(n / float(N)) ** (order + 1)
    assert np.max(np.abs(wrong_arg - meas.real)) > 1e-3
    assert np.max(np.abs(wrong_exp - meas.real)) > 1e-3


def test_window_noncubic_axes_are_per_axis():
    shape = (8, 12, 16)
    m = wt.window(shape, 2)
    for ax, N in enumerate(shape):
        meas = _measured_window(ps.freqs(N).astype(np.int64), N, 2).real
        line = np.moveaxis(m, ax, 0)[:, 0, 0]
        assert np.max(np.abs(line - meas)) < 1e-12


# ------------------------------------------- sampled triplet sums / counts


def _sample_trips(trips, rng, k):
    pick = rng.choice(len(trips), size=min(k, len(trips)), replace=False)
    sel = trips[np.sort(pick)]
    eq = trips[(trips[:, 0] == trips[:, 1]) & (trips[:, 1] == trips[:, 2])]
    return np.concatenate([sel, eq[:2]])  # always some a = b = c


@pytest.mark.parametrize("n,nbins", [(32, 8), (64, 12)])
def test_sampled_sums_and_counts_match_full_estimator(n, nbins):
    box = 1000.0
    edges = kf_edges(nbins)
    d = quadratic_field(n, box, 1.0, 40 + n).astype(np.float32).astype(np.float64)
    res = oracle.bispectrum(d, box, edges)
    rng = np.random.default_rng(n)
    trips = _sample_trips(res.triplets, rng, 25)
    index = {tuple(t): i for i, t in enumerate(res.triplets.tolist())}
    rows = np.array([index[tuple(t)] for t in trips.tolist()])
    s, sa = oracle.triplet_sums_sample(d, edges, trips)
    T = oracle.count_sample(n, edges, trips)
    scale = float(box) ** 6 / float(n) ** 3
    assert np.array_equal(T, res.counts[rows].astype(np.int64))
    assert np.allclose(scale * s / T, res.bk[rows], rtol=1e-12, atol=1e-12 * np.max(np.abs(res.absnorm)))
    assert np.allclose(scale * sa / T, res.absnorm[rows], rtol=1e-12)


def test_sampled_sums_catch_a_shuffled_remap(monkeypatch):
    """A remap mistake (fields handed back in another order than the bins
    they were asked for) makes the comparison above fail."""
    n, box, edges = 32, 1000.0, kf_edges(8)
    d = quadratic_field(n, box, 1.0, 72).astype(np.float64)
    res = oracle.bispectrum(d, box, edges)
    trips = _sample_trips(res.triplets, np.random.default_rng(3), 25)
    index = {tuple(t): i for i, t in enumerate(res.triplets.tolist())}
    rows = np.array([index[tuple(t)] for t in trips.tolist()])
    good = oracle.triplet_sums_sample(d, edges, trips)[0]
    real = ps.filtered_fields
    monkeypatch.setattr(ps, "filtered_fields", lambda *a, **k: real(*a, **k)[::-1])
    bad = oracle.triplet_sums_sample(d, edges, trips)[0]
    scale = float(box) ** 6 / float(n) ** 3
    T = res.counts[rows]
    assert np.allclose(scale * good / T, res.bk[rows], rtol=1e-12, atol=1e-12 * np.max(res.absnorm))
    assert not np.allclose(scale * bad / T, res.bk[rows], rtol=1e-6)


# ------------------------------------------------ counts in the continuum
# End of Sec. IV.D.1: without discreteness, N_0 = 4 pi int r^2 dr f_a f_b f_c
# with f_b(r) = int k^2 dk / (2 pi^2) j_0(k r) over the shell (P_fid = 1).  In
# units of the fundamental frequency the grid holds one mode per unit volume,
# so the lattice count of ordered closed triangles is T ~ (2 pi)^6 N_0.  The
# shell integral is closed-form: int k^2 j_0(k r) dk = [sin(kr) - kr cos(kr)] / r^3.


def _shell(r, lo, hi):
    g = lambda x: np.sin(x) - x * np.cos(x)  # noqa: E731
    out = np.empty_like(r)
    small = r < 1e-3
    rs = r[~small]
    out[~small] = (g(hi * rs) - g(lo * rs)) / rs**3
    out[small] = (hi**3 - lo**3) / 3.0
    return out / (2.0 * np.pi**2)


def _n0_continuum(edges, trip, rmax=300.0, h=0.002):
    r = np.arange(0.0, rmax + h / 2, h)  # an even number of intervals: Simpson's rule
    y = r * r
    for b in trip:
        y = y * _shell(r, edges[b], edges[b + 1])
    w = np.ones_like(r)
    w[1:-1:2], w[2:-1:2] = 4.0, 2.0
    return 4.0 * np.pi * h / 3.0 * np.sum(w * y)


def test_counts_approach_the_continuum_bessel_integral():
    """Exact lattice counts T against (2 pi)^6 N_0 of the continuum formula,
    on a 96^3 grid (alias-free) with shells of width w = 2 from radius 8:
    the totals agree to 0.5%, the median triplet to 2%, and every triplet
    within the discreteness of its smallest shell, 4 / (e_a w) (a shell of
    radius R and width w holds its continuum volume to O(1 / (R w)))."""
    n, w = 96, 2.0
    edges = np.arange(8.0, 33.0, w)
    trips = ps.triangle_triplets(edges)
    T, _ = ps.triangle_counts(n, edges, trips)
    cont = np.array([(2.0 * np.pi) ** 6 * _n0_continuum(edges, t) for t in trips])
    keep = T > 0
    assert keep.sum() > 300
    rel = T[keep] / cont[keep] - 1.0
    assert abs(T[keep].sum() / cont[keep].sum() - 1.0) < 5e-3
    assert np.median(np.abs(rel)) < 0.02
    assert np.all(np.abs(rel) <= 4.0 / (edges[trips[keep, 0]] * w)), np.abs(rel).max()
    # counting unordered triangles instead (a mistake the formula catches) is far off
    eq = (trips[keep, 0] == trips[keep, 1]) & (trips[keep, 1] == trips[keep, 2])
    assert np.all(np.abs(T[keep][eq] / 6.0 / cont[keep][eq] - 1.0) > 0.5)
