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
