"""Pins for the FP64 oracle against what the paper and mathematics fix.

None of these re-type the oracle's formulas: each compares it with an
independent route (brute-force mode loops, closed forms for plane waves,
exact invariances, the count printed in the paper, statistical recovery of
a known input power spectrum and tree-level bispectrum).
"""

import os

import numpy as np
import pytest

import oracle
from synthetic import gaussian_field, kf_edges, pk_model, quadratic_field, window_mask

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=")
            vals[k.strip()] = [float(x) for x in v.split()]
    return vals


# ---------------------------------------------------------------- binning


def test_triplet_count_matches_paper_setup():
    g = _golden("bk_validation_setup.txt")
    edges = np.array(g["edges"])
    trips = oracle.triangle_triplets(edges)
    assert len(trips) * int(g["n_multipoles"][0]) == int(g["n_configurations"][0])


def test_triplet_count_is_scale_free_and_ordered():
    # config-1 edges (width 2 k_f from k_f) give the same triangle rule
    trips = oracle.triangle_triplets(kf_edges(8))
    assert len(trips) == 98
    # order: c fastest, then b, then a; a <= b <= c
    assert np.all(trips[:, 0] <= trips[:, 1]) and np.all(trips[:, 1] <= trips[:, 2])
    keys = trips[:, 0] * 10000 + trips[:, 1] * 100 + trips[:, 2]
    assert np.all(np.diff(keys) > 0)
    # larger configurations
    assert len(oracle.triangle_triplets(kf_edges(20))) == 1015
    assert len(oracle.triangle_triplets(kf_edges(30))) == 3035


def test_mode_counts_by_explicit_loops():
    n = 12
    edges = np.array([1.0, 2.5, 4.0, 6.0])
    want = np.zeros(3, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                f = [v if v < n // 2 else v - n for v in (i, j, k)]
                r = np.sqrt(f[0] ** 2 + f[1] ** 2 + f[2] ** 2)
                for b in range(3):
                    if edges[b] <= r < edges[b + 1]:
                        want[b] += 1
    assert np.array_equal(oracle.mode_counts(n, edges), want)
    # a mode exactly on an edge goes to the upper bin (half-open bins)
    idx = oracle.bin_of_modes(n, np.array([1.0, 3.0, 5.0]))
    assert idx[3, 0, 0] == 1 and idx[1, 0, 0] == 0


# ------------------------------------------------------ brute-force pins


@pytest.mark.parametrize(
    "n,edges",
    [
        (8, [1.0, 2.0, 3.0, 4.0]),  # aliases: closure wraps modulo N
        (12, [1.0, 2.5, 4.0, 5.5]),
        (16, [2.0, 3.0, 4.5]),
    ],
)
def test_separable_form_equals_brute_force(n, edges):
    edges = np.array(edges)
    rng = np.random.default_rng(n)
    d = rng.standard_normal((n, n, n))
    trips = oracle.triangle_triplets(edges)
    sums, cnt = oracle.brute_sums(d, edges, trips)
    # counts: exact integers
    T, raw = oracle.triangle_counts(n, edges, trips)
    assert np.array_equal(T, cnt)
    assert np.max(np.abs(raw - T)) < 1e-6
    # the imaginary part of the closed-triangle sum vanishes for a real field
    assert np.all(np.abs(sums.imag) <= 1e-9 * np.abs(sums).max())
    # separable real-space sum  N_pix^2 sum_x G_a G_b G_c  ==  sum_closed D D D
    G = oracle.filtered_fields(d, edges)
    npix = float(n) ** 3
    sep = np.array([npix**2 * np.sum(G[a] * G[b] * G[c]) for a, b, c in trips])
    scale = np.abs(sums.real).max()
    assert np.max(np.abs(sep - sums.real)) <= 1e-12 * scale
    # and the estimator normalisation B = V^2/N_pix^3 sum DDD / T
    box = 100.0
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    keep = cnt > 0
    want = box**6 / npix**3 * sums.real[keep] / cnt[keep]
    assert np.allclose(res.bk, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_counts_are_integers_at_32():
    edges = kf_edges(8)
    T, raw = oracle.triangle_counts(32, edges)
    assert np.max(np.abs(raw - T)) < 1e-6
    assert T.min() > 0


# ---------------------------------------------------- closed-form pins


def test_power_parseval_full_cover():
    n, box = 16, 300.0
    rng = np.random.default_rng(3)
    d = rng.standard_normal((n, n, n))
    # bins covering every non-zero mode: |n| in [0.5, N sqrt(3)/2 + 1)
    edges = np.arange(0.5, n * np.sqrt(3) / 2 + 1.5, 1.0)
    nm = oracle.mode_counts(n, edges)
    keep = nm > 0
    edges_ok = np.concatenate([edges[:-1][keep], [edges[-1]]])
    # merge empty bins away by rebuilding edges from non-empty shells
    nm2 = oracle.mode_counts(n, edges_ok)
    assert nm2.sum() == n**3 - 1
    pk = oracle.power_spectrum(d, box, edges_ok)
    npix = float(n) ** 3
    lhs = np.sum(nm2 * pk) * npix**2 / box**3
    rhs = npix * np.sum(d * d) - np.sum(d) ** 2
    assert abs(lhs - rhs) <= 1e-12 * rhs


def test_power_plane_wave():
    n, box = 32, 1000.0
    edges = kf_edges(8)
    x = np.arange(n)
    n0 = (2, 3, 1)  # |n0| = sqrt(14) = 3.74 -> bin 1, [3, 5)
    ph = 2 * np.pi * (n0[0] * x[:, None, None] + n0[1] * x[None, :, None] + n0[2] * x[None, None, :]) / n
    d = np.cos(ph)
    pk = oracle.power_spectrum(d, box, edges)
    nm = oracle.mode_counts(n, edges)
    want = np.zeros(8)
    want[1] = box**3 / (2 * nm[1])
    assert np.allclose(pk, want, rtol=1e-12, atol=1e-12 * want.max())


def _plane_wave_triple(n, edges):
    """Three non-collinear waves n1 + n2 + n3 = 0 in three distinct bins."""
    idx = oracle.bin_of_modes(n, edges)
    rng = np.random.default_rng(11)
    for _ in range(10000):
        n1 = rng.integers(-6, 7, size=3)
        n2 = rng.integers(-6, 7, size=3)
        n3 = -(n1 + n2)
        if np.linalg.matrix_rank(np.stack([n1, n2])) < 2:
            continue
        bins = [int(idx[tuple(v % n)]) for v in (n1, n2, n3)]
        if min(bins) < 0 or len(set(bins)) < 3:
            continue
        # no other sign combination closes
        ok = True
        for s in [(1, 1, -1), (1, -1, 1), (-1, 1, 1)]:
            if np.all((s[0] * n1 + s[1] * n2 + s[2] * n3) % n == 0):
                ok = False
        if ok:
            return (n1, n2, n3), bins
    raise RuntimeError("no triple found")


def test_bispectrum_plane_waves():
    n, box = 32, 1000.0
    edges = kf_edges(8)
    (n1, n2, n3), bins = _plane_wave_triple(n, edges)
    x = np.arange(n)
    d = np.zeros((n, n, n))
    for v in (n1, n2, n3):
        ph = 2 * np.pi * (v[0] * x[:, None, None] + v[1] * x[None, :, None] + v[2] * x[None, None, :]) / n
        d += np.cos(ph)
    res = oracle.bispectrum(d, box, edges)
    a, b, c = sorted(bins)
    t = [i for i, tr in enumerate(res.triplets) if tuple(tr) == (a, b, c)]
    assert len(t) == 1
    want = box**6 / (4.0 * res.counts[t[0]])
    assert abs(res.bk[t[0]] - want) <= 1e-11 * want


# ------------------------------------------------------------ invariances


def test_invariances_and_scaling():
    n, box = 32, 1000.0
    edges = kf_edges(8)
    d = quadratic_field(n, box, 0.5, 7)
    base = oracle.bispectrum(d, box, edges)
    T = None
    variants = [
        np.roll(d, (3, -5, 7), axis=(0, 1, 2)),  # integer translation
        np.transpose(d, (2, 0, 1)),  # axis permutation
        np.roll(d[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)),  # reflection x -> -x
        d + 0.37,  # a constant only touches k = 0, which lies in no bin
    ]
    for v in variants:
        r = oracle.bispectrum(np.ascontiguousarray(v), box, edges, counts=T)
        sc = np.abs(base.absnorm)
        assert np.all(np.abs(r.bk - base.bk) <= 1e-12 * sc)
        assert np.allclose(r.pk, base.pk, rtol=1e-12)
    # scaling by 2 is exact in binary floating point
    r2 = oracle.bispectrum(2.0 * d, box, edges)
    assert np.array_equal(r2.pk, 4.0 * base.pk)
    assert np.array_equal(r2.bk, 8.0 * base.bk)


# ------------------------------------------------------------ statistics


def _grid_binned_pk(n, box, edges):
    kf = 2 * np.pi / box
    k = kf * np.sqrt(oracle.kmag2(n).astype(np.float64))
    idx = oracle.bin_of_modes(n, edges)
    p = pk_model(k)
    return np.array([p[idx == b].mean() for b in range(len(edges) - 1)])


def test_power_recovers_input_statistically():
    n, box = 32, 1000.0
    edges = kf_edges(8)
    runs = np.array([oracle.power_spectrum(gaussian_field(n, box, s), box, edges) for s in range(100)])
    want = _grid_binned_pk(n, box, edges)
    z = (runs.mean(0) - want) / (runs.std(0, ddof=1) / np.sqrt(len(runs)))
    assert np.all(np.abs(z) < 4.5), z


def test_tree_level_bispectrum_and_gaussian_null():
    """Linear-in-f_NL coefficient of B for d = g + f(g^2 - <g^2>) has mean
    2 (P1 P2 + P2 P3 + P3 P1) averaged over the closed triangles in the bin;
    the f-independent part (a Gaussian field) has mean zero."""
    n, box, f = 32, 1000.0, 0.5
    edges = kf_edges(8)
    trips = oracle.triangle_triplets(edges)
    T, _ = oracle.triangle_counts(n, edges, trips)
    c0s, c1s = [], []
    for s in range(120):
        g = gaussian_field(n, box, s)
        g2 = g * g - np.mean(g * g)
        B = {}
        for m in (-2, -1, 1, 2):
            B[m] = oracle.bispectrum(g + m * f * g2, box, edges, trips, T).bk
        c1s.append((8 * (B[1] - B[-1]) - (B[2] - B[-2])) / (12 * f))
        c0s.append((4 * (B[1] + B[-1]) - (B[2] + B[-2])) / 6)
    c1s, c0s = np.array(c1s), np.array(c0s)
    # expectation: sum over closed triangles of 2(P1P2+...) / T, computed as
    # a direct sum over mode pairs binned by |n| (brute force over shells)
    kf = 2 * np.pi / box
    P = pk_model(kf * np.sqrt(oracle.kmag2(n).astype(np.float64)))
    idx = oracle.bin_of_modes(n, edges)
    H = oracle.unit_fields(n, edges)
    A = np.stack([oracle.idft(np.where(idx == b, P, 0.0)).real for b in range(len(edges) - 1)])
    want = np.array(
        [
            2
            * (np.sum(A[a] * A[b] * H[c]) + np.sum(A[a] * H[b] * A[c]) + np.sum(H[a] * A[b] * A[c]))
            / np.sum(H[a] * H[b] * H[c])
            for a, b, c in trips
        ]
    )
    se1 = c1s.std(0, ddof=1) / np.sqrt(len(c1s))
    z1 = (c1s.mean(0) - want) / se1
    assert np.all(np.abs(z1) < 4.5), np.abs(z1).max()
    se0 = c0s.std(0, ddof=1) / np.sqrt(len(c0s))
    z0 = c0s.mean(0) / se0
    assert np.all(np.abs(z0) < 4.5), np.abs(z0).max()
    # the signal is detected: the tree-level term is many standard errors
    assert np.median(np.abs(want) / se1) > 3


def test_tree_expectation_matches_mode_sum_on_tiny_grid():
    """The separable expectation used above equals an explicit loop over
    closed mode triangles (n = 8, all bins)."""
    n, box = 8, 200.0
    edges = np.array([1.0, 2.0, 3.0, 4.0])
    kf = 2 * np.pi / box
    P = pk_model(kf * np.sqrt(oracle.kmag2(n).astype(np.float64)))
    idx = oracle.bin_of_modes(n, edges)
    trips = oracle.triangle_triplets(edges)
    H = oracle.unit_fields(n, edges)
    A = np.stack([oracle.idft(np.where(idx == b, P, 0.0)).real for b in range(3)])
    for a, b, c in trips:
        tot, cnt = 0.0, 0
        for i1 in np.argwhere(idx == a):
            for i2 in np.argwhere(idx == b):
                i3 = (-i1 - i2) % n
                if idx[tuple(i3)] == c:
                    p1, p2, p3 = P[tuple(i1)], P[tuple(i2)], P[tuple(i3)]
                    tot += 2 * (p1 * p2 + p2 * p3 + p1 * p3)
                    cnt += 1
        if cnt == 0:
            continue
        sep = 2 * (np.sum(A[a] * A[b] * H[c]) + np.sum(A[a] * H[b] * A[c]) + np.sum(H[a] * A[b] * A[c])) / np.sum(
            H[a] * H[b] * H[c]
        )
        assert abs(sep - tot / cnt) <= 1e-10 * abs(tot / cnt)


def test_aliasing_reading_modulo_n():
    """At N = 32 with e_top = 17 some closures wrap around the grid
    (3 * 16 >= 32): the count includes them, matching the brute force."""
    n = 8
    edges = np.array([2.0, 3.0, 3.5])
    trips = oracle.triangle_triplets(edges)
    d = np.random.default_rng(5).standard_normal((n, n, n))
    _, cnt = oracle.brute_sums(d, edges, trips)
    T, _ = oracle.triangle_counts(n, edges, trips)
    assert np.array_equal(T, cnt)
    # without wrap-around the count would differ for at least one triplet
    idx = oracle.bin_of_modes(n, edges)
    f = oracle.freqs(n)
    nowrap = []
    for a, b, c in trips:
        m = 0
        for i1 in np.argwhere(idx == a):
            for i2 in np.argwhere(idx == b):
                v = -(f[i1] + f[i2])
                if np.all(np.abs(v) < n // 2) or np.all((v >= -n // 2) & (v < n // 2)):
                    if idx[tuple(v % n)] == c:
                        m += 1
        nowrap.append(m)
    assert not np.array_equal(np.array(nowrap), cnt)


def test_windowed_estimators_unbiased_for_local_field():
    """For d = w * delta with delta = g + f(g^2 - 1), g white unit Gaussian,
    the 2- and 3-point functions of delta are local: <D_d(n) D_d(-n)> =
    sum_x w^2 (1 + 2f^2) and <D_d D_d D_d>_closed = sum_x w^3 (6f + 8f^3).
    The windowed estimators therefore have means V (1 + 2f^2) / N_pix and
    V^2 (6f + 8f^3) / N_pix^2 exactly, for any window; checked over masked
    realizations (a different weighted sphere-with-holes window each time).
    With non-binary weights <w^2> != <w^3>, so normalising B by the wrong
    moment fails."""
    from synthetic import window_mask

    n, box, f = 24, 600.0, 0.3
    edges = kf_edges(6)
    npix = float(n) ** 3
    ps, bs = [], []
    for s in range(80):
        g = np.random.default_rng(7000 + s).standard_normal((n, n, n))
        delta = g + f * (g * g - 1.0)
        # sphere with holes, times smooth-ish positive weights (FKP-like), so
        # that <w^2> and <w^3> differ
        wr = np.random.default_rng(9500 + s).random((n, n, n))
        w = window_mask(n, 9000 + s, radius=0.45, keep=0.9).astype(np.float64) * (0.5 + wr)
        pk, bk, (m2, m3), _ = oracle.windowed_polyspectra(w * delta, w, box, edges)
        assert m3 > 1.1 * m2
        ps.append(pk)
        bs.append(bk)
    ps, bs = np.array(ps), np.array(bs)
    want_p = box**3 * (1 + 2 * f * f) / npix
    want_b = box**6 * (6 * f + 8 * f**3) / npix**2
    zp = (ps.mean(0) - want_p) / (ps.std(0, ddof=1) / np.sqrt(len(ps)))
    zb = (bs.mean(0) - want_b) / (bs.std(0, ddof=1) / np.sqrt(len(bs)))
    assert np.all(np.abs(zp) < 4.5), zp
    assert np.all(np.abs(zb) < 4.5), np.abs(zb).max()
    # the signal is resolved, so a wrong power of the window moment fails
    assert np.median(np.abs(want_b) / (bs.std(0, ddof=1) / np.sqrt(len(bs)))) > 5


# ------------------------------------------------------- masked power (MC)


def test_masked_fisher_exact_without_window_and_brute_force():
    """Without a window the exact Fisher is (1/2) diag(N_b); with one it
    equals the double sum (1/2) sum_{x,y} w(x) w(y) H_a(x-y) H_b(x-y)."""
    from oracle import masked
    from synthetic import window_mask

    n, edges = 8, np.array([1.0, 2.0, 3.0, 4.0])
    F1 = masked.fisher_power_exact(np.ones((n, n, n)), edges)
    nm = oracle.mode_counts(n, edges)
    assert np.allclose(F1, 0.5 * np.diag(nm), atol=1e-10)
    w = window_mask(n, 3, radius=0.4, keep=0.8).astype(np.float64) * (
        0.5 + np.random.default_rng(4).random((n, n, n)))
    F = masked.fisher_power_exact(w, edges)
    H = oracle.unit_fields(n, edges)
    pts = np.array(np.unravel_index(np.arange(n**3), (n, n, n))).T
    wf = w.ravel()
    brute = np.zeros_like(F)
    for i in range(n**3):
        r = (pts[i] - pts) % n  # x - y for every y
        hab = H[:, r[:, 0], r[:, 1], r[:, 2]]  # [nb, n^3]
        brute += 0.5 * wf[i] * (hab * wf[None, :]) @ hab.T
    assert np.allclose(F, brute, rtol=1e-10, atol=1e-10)


def test_masked_fisher_monte_carlo_converges():
    """The Girard-Hutchinson average over white fields is unbiased for the
    exact Fisher matrix (z-test per element over 60 fields)."""
    from oracle import masked
    from synthetic import window_mask

    n, edges = 16, kf_edges(4)
    w = window_mask(n, 11, radius=0.45, keep=0.9).astype(np.float64)
    Fx = masked.fisher_power_exact(w, edges)
    rng = np.random.default_rng(12)
    draws = np.array([masked.mc_fisher_power(w, [rng.standard_normal((n, n, n))], edges) for _ in range(60)])
    se = draws.std(0, ddof=1) / np.sqrt(len(draws))
    z = (draws.mean(0) - Fx) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    # off-diagonal leakage from the window is resolved
    assert np.abs(Fx[0, 1]) > 5 * se[0, 1]


def test_unwindowed_power_unbiased_for_flat_spectrum():
    """Data whose spectrum is flat inside the bins and zero outside them (the
    bandpowers then describe it completely) under a window: F^-1 p with the
    exact Fisher matrix recovers P in every bin, while the windowed
    estimator P / <w^2> does not in the edge bins."""
    from oracle import masked
    from synthetic import window_mask

    n, box, edges = 16, 500.0, kf_edges(4)
    w = window_mask(n, 21, radius=0.45, keep=0.9).astype(np.float64)
    Fx = masked.fisher_power_exact(w, edges)
    inside = oracle.bin_of_modes(n, edges) >= 0
    sigma = 1.7

    def field(s):
        g = np.fft.fftn(np.random.default_rng(400 + s).standard_normal((n, n, n)))
        return sigma * np.fft.ifftn(np.where(inside, g, 0.0)).real

    est, win = [], []
    for s in range(150):
        d = w * field(s)
        est.append(masked.unwindowed_power(d, box, edges, Fx))
        win.append(oracle.power_spectrum(d, box, edges) / np.mean(w * w))
    est, win = np.array(est), np.array(win)
    want = box**3 * sigma**2 / n**3
    z = (est.mean(0) - want) / (est.std(0, ddof=1) / np.sqrt(len(est)))
    assert np.all(np.abs(z) < 4.5), z
    zw = (win.mean(0) - want) / (win.std(0, ddof=1) / np.sqrt(len(win)))
    assert np.abs(zw).max() > 6, zw


# ------------------------------------------------------------ multipoles


def test_bispectrum_multipole_separable_equals_mode_loops():
    """sum_x G_a G_b g_{c,l} N_pix^2 equals the explicit sum over closed mode
    triangles of L_l(mu_3) D1 D2 D3 (Legendre weight on the mode in bin c)."""
    from oracle import multipoles as mp

    n = 8
    edges = np.array([1.0, 2.0, 3.0, 4.0])
    d = quadratic_field(n, 300.0, 0.7, 31)
    trips = oracle.triangle_triplets(edges)
    G0 = mp.weighted_fields(d, edges, 0)
    for ell in (2, 4):
        Gl = mp.weighted_fields(d, edges, ell)
        sep = np.array([np.sum(G0[a] * G0[b] * Gl[c]) for a, b, c in trips]) * float(n) ** 6
        brute = mp.brute_multipole_sums(d, edges, trips, ell)
        assert np.allclose(brute.imag, 0, atol=1e-8 * np.abs(brute).max())
        assert np.allclose(sep, brute.real, rtol=1e-10, atol=1e-10 * np.abs(brute).max())
    # the monopole of the multipole path is the monopole estimator
    _, B = mp.bispectrum_multipoles(d, 300.0, edges, lmax=2)
    assert np.allclose(B[0], oracle.bispectrum(d, 300.0, edges).bk, rtol=1e-12)


def test_power_multipoles_unbiased_for_anisotropic_field():
    """Gaussian field with P(n) = P0 + P2 L2(mu) + P4 L4(mu) (constant in |n|):
    the discrete-Fisher multipoles recover (P0, P2, P4) in every bin."""
    from oracle import multipoles as mp

    n, box = 24, 500.0
    edges = kf_edges(5)
    P0, P2, P4 = 3.0, 1.2, 0.5
    mu = mp.mu_grid(n)
    P = P0 + P2 * mp.legendre(2, mu) + P4 * mp.legendre(4, mu)
    P[0, 0, 0] = 0.0
    npix, vol = float(n) ** 3, box**3
    runs = []
    for s in range(120):
        w = np.fft.fftn(np.random.default_rng(600 + s).standard_normal((n, n, n)))
        d = np.fft.ifftn(w * np.sqrt(P * npix / vol)).real  # <|D(n)|^2> = N_pix^2 P(n) / V
        runs.append(mp.power_multipoles(d, box, edges, lmax=4))
    runs = np.array(runs)
    want = np.array([P0, P2, P4])[:, None] * np.ones(len(edges) - 1)
    z = (runs.mean(0) - want) / (runs.std(0, ddof=1) / np.sqrt(len(runs)))
    assert np.all(np.abs(z) < 4.5), z
    assert np.abs(runs.mean(0)[1]).min() > 5 * (runs.std(0, ddof=1) / np.sqrt(len(runs)))[1].max()


def test_multipoles_symmetries():
    """x <-> y exchange and z reflection leave every multipole unchanged
    (line of sight along z); exchanging z with x changes the quadrupole."""
    from oracle import multipoles as mp

    n, box = 16, 400.0
    edges = kf_edges(4)
    d = quadratic_field(n, box, 1.0, 8)
    P = mp.power_multipoles(d, box, edges)
    _, B = mp.bispectrum_multipoles(d, box, edges, lmax=4)
    for e in (np.swapaxes(d, 0, 1), d[:, :, ::-1]):
        assert np.allclose(mp.power_multipoles(e, box, edges), P, rtol=1e-9, atol=1e-9 * np.abs(P).max())
        assert np.allclose(mp.bispectrum_multipoles(e, box, edges, lmax=4)[1], B, rtol=1e-9,
                           atol=1e-9 * np.abs(B).max())
    Pz = mp.power_multipoles(np.swapaxes(d, 0, 2), box, edges)
    assert not np.allclose(Pz[1], P[1], rtol=1e-3)


# ---------------------------------------------- weighted ideal estimators


def _pfid_table(n, box, edges):
    kf = 2 * np.pi / box
    e2 = int(np.ceil(np.asarray(edges)[-1] ** 2))
    t = pk_model(kf * np.sqrt(np.arange(e2 + 1, dtype=np.float64))) + 500.0
    t[0] = 1.0
    return t


def test_weighted_sums_equal_mode_loops():
    from oracle import weighted as wt

    n, box = 8, 300.0
    edges = np.array([1.0, 2.0, 3.0, 4.0])
    d = quadratic_field(n, box, 0.6, 41)
    pf = _pfid_table(n, box, edges)
    trips, B, n0, _ = wt.weighted_bispectrum(d, box, edges, order=2, pfid=pf)
    num, n0b, qb = wt.brute_weighted_sums(d, edges, trips, order=2, pfid=pf)
    assert np.allclose(n0, n0b, rtol=1e-10)
    npix = float(n) ** 3
    assert np.allclose(B, box**6 / npix**3 * num.real / n0b, rtol=1e-9, atol=1e-9 * np.abs(B).max())
    # shot-noise term through the separable route against the loops
    nbar = 2e-4
    _, Bs, _, _ = wt.weighted_bispectrum(d, box, edges, order=2, pfid=pf, nbar=nbar)
    shot = 1 / nbar**2 + (qb / n0b - 3 / nbar) / nbar
    assert np.allclose(B - Bs, shot, rtol=1e-10)


def test_weighted_reduces_and_deconvolves():
    """Constant P_fid and no window give the unweighted estimators; a window
    applied to the field in Fourier space is undone by the deconvolution."""
    from oracle import weighted as wt

    n, box = 16, 500.0
    edges = kf_edges(4)
    d = quadratic_field(n, box, 1.0, 3)
    res = oracle.bispectrum(d, box, edges)
    const = np.full(int(np.ceil(edges[-1] ** 2)) + 1, 7.0)
    assert np.allclose(wt.weighted_power(d, box, edges, 0, const), res.pk, rtol=1e-12)
    _, B, _, _ = wt.weighted_bispectrum(d, box, edges, 0, const)
    assert np.allclose(B, res.bk, rtol=1e-10, atol=1e-12 * np.abs(res.bk).max())
    for order in (1, 2, 3):
        dw = np.fft.ifftn(np.fft.fftn(d) * wt.window(n, order)).real
        assert np.allclose(wt.weighted_power(dw, box, edges, order), res.pk, rtol=1e-10)
        _, Bw, _, _ = wt.weighted_bispectrum(dw, box, edges, order)
        assert np.allclose(Bw, res.bk, rtol=1e-8, atol=1e-10 * np.abs(res.bk).max())


def test_shot_noise_of_poisson_field_is_removed():
    """Uniform Poisson counts in cells (no clustering): with P_fid = 1/nbar
    (pure noise, so the power model P_fid - 1/nbar is zero) the shot-noise
    corrected P and B average to zero; without the correction they are
    1/nbar and 1/nbar^2."""
    from oracle import weighted as wt

    n, box = 16, 400.0
    edges = kf_edges(4)
    cell = (box / n) ** 3
    lam = 4.0  # mean count per cell
    nbar = lam / cell
    pf = np.full(int(np.ceil(edges[-1] ** 2)) + 1, 1.0 / nbar)
    Ps, Bs = [], []
    for s in range(150):
        cnt = np.random.default_rng(800 + s).poisson(lam, (n, n, n)).astype(np.float64)
        delta = cnt / lam - 1.0
        Ps.append(wt.weighted_power(delta, box, edges, 0, pf, nbar))
        Bs.append(wt.weighted_bispectrum(delta, box, edges, 0, pf, nbar)[1])
    Ps, Bs = np.array(Ps), np.array(Bs)
    zp = Ps.mean(0) / (Ps.std(0, ddof=1) / np.sqrt(len(Ps)))
    zb = Bs.mean(0) / (Bs.std(0, ddof=1) / np.sqrt(len(Bs)))
    assert np.all(np.abs(zp) < 4.5), zp
    assert np.all(np.abs(zb) < 4.5), np.abs(zb).max()
    # the subtracted terms are resolved: without them the means are far from zero
    assert np.all(np.abs((Ps.mean(0) + 1 / nbar) / (Ps.std(0, ddof=1) / np.sqrt(len(Ps)))) > 10)
    assert np.median(np.abs((Bs.mean(0) + 1 / nbar**2) / (Bs.std(0, ddof=1) / np.sqrt(len(Bs))))) > 5


def _field_with_power(n, box, order, c, seed):
    """Hermitian Fourier field with |D/m|^2 = (N_pix^2/V) sum_l c_l L_l(mu)
    exactly (deterministic amplitudes, random phases), returned in real space."""
    from oracle import weighted as wt
    from oracle.multipoles import legendre, mu_grid

    npix, vol = float(n) ** 3, float(box) ** 3
    mu = mu_grid(n)
    shape = sum(cl * legendre(2 * i, mu) for i, cl in enumerate(c))
    assert shape.min() > 0
    amp = wt.window(n, order) * np.sqrt(npix**2 / vol * shape)
    ph = np.random.default_rng(seed).uniform(-np.pi, np.pi, (n, n, n))
    neg = (-np.arange(n)) % n
    ph = 0.5 * (ph - ph[np.ix_(neg, neg, neg)])  # odd phase: D(-n) = conj D(n)
    D = amp * np.exp(1j * ph)
    D[0, 0, 0] = 0.0
    return np.fft.ifftn(D).real


def test_weighted_power_multipoles_recover_anisotropic_power():
    """A field whose deconvolved mode power is exactly c0 + c2 L_2(mu) + c4 L_4(mu)
    gives P_0 = c0 - 1/nbar, P_2 = c2, P_4 = c4 for any P_fid weights: the
    discrete Fisher matrix and the numerator carry the same weights."""
    from oracle import weighted as wt
    from oracle.multipoles import legendre, mu_grid

    n, box = 16, 400.0
    edges = kf_edges(5)
    c0, c2, c4 = 3.0e3, 1.2e3, 4.0e2
    d = _field_with_power(n, box, 2, (c0, c2, c4), 7)
    pf = _pfid_table(n, box, edges)
    nbar = 1e-3
    P = wt.weighted_power_multipoles(d, box, edges, 4, order=2, pfid=pf, nbar=nbar)
    assert np.allclose(P[0], c0 - 1 / nbar, rtol=1e-10)
    assert np.allclose(P[1], c2, rtol=1e-10)
    assert np.allclose(P[2], c4, rtol=1e-10)
    # the couplings are real: L_4 does not average out over the bins of a
    # finite grid, so a diagonal normalisation would bias the monopole
    idx = oracle.bin_of_modes(n, edges)
    L4 = legendre(4, mu_grid(n))
    assert max(abs(L4[idx == b].mean()) for b in range(len(edges) - 1)) > 1e-2


def test_weighted_multipoles_reduce_and_match_mode_loops():
    from oracle import multipoles as ml
    from oracle import weighted as wt

    n, box = 8, 300.0
    edges = np.array([1.0, 2.0, 3.0, 4.0])
    d = quadratic_field(n, box, 0.6, 43)
    pf = _pfid_table(n, box, edges)
    nbar = 5e-4
    trips, Bl = wt.weighted_bispectrum_multipoles(d, box, edges, 4, order=3, pfid=pf, nbar=nbar)
    _, B0, n0, _ = wt.weighted_bispectrum(d, box, edges, 3, pf, nbar)
    assert np.array_equal(Bl[0], B0)
    npix = float(n) ** 3
    for i, ell in enumerate((2, 4), start=1):
        num, n0b, _ = wt.brute_weighted_sums(d, edges, trips, order=3, pfid=pf, ell=ell)
        want = (2 * ell + 1) * box**6 / npix**3 * num.real / n0b
        assert np.allclose(Bl[i], want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    # constant P_fid, no window, no noise: the unweighted multipoles
    n, box = 16, 500.0
    edges = kf_edges(4)
    d = quadratic_field(n, box, 1.0, 5)
    const = np.full(int(np.ceil(edges[-1] ** 2)) + 1, 3.0)
    assert np.allclose(wt.weighted_power_multipoles(d, box, edges, 4, 0, const),
                       ml.power_multipoles(d, box, edges, 4), rtol=1e-10, atol=1e-12)
    t1, B1 = wt.weighted_bispectrum_multipoles(d, box, edges, 2, 0, const)
    t2, B2 = ml.bispectrum_multipoles(d, box, edges, 2)
    assert np.array_equal(t1, t2)
    assert np.allclose(B1, B2, rtol=1e-9, atol=1e-11 * np.abs(B2).max())


# ------------------------------------------------- injected bispectrum


def test_injection_expectation_matches_triangle_loops():
    from oracle import injection as inj
    from synthetic import injection_beta

    n, box = 8, 2 * np.pi / 0.1
    edges = np.array([1.0, 2.0, 3.0, 4.0])

    def beta(k):
        return injection_beta(k, kmin=0.15, kmax=0.35)

    trips, E = inj.expected_bispectrum(n, box, edges, beta, eps=1.0, lmax=2)
    for i, ell in enumerate((0, 2)):
        want = inj.brute_expected(n, box, edges, trips, beta, ell)
        assert np.allclose(E[i], want, rtol=1e-10, atol=1e-12 * np.abs(E[0]).max())
    assert np.abs(E[0]).max() > 0 and np.any(E[0] == 0)  # the filter leaves some triplets empty
    # an isotropic injection has no quadrupole on a cubic grid's closed triangles
    assert np.abs(E[1]).max() < 1e-12 * np.abs(E[0]).max()
    # with a beta that depends on the direction (given on the grid) the
    # quadrupole is live, and the separable form still equals the loops
    from oracle.multipoles import mu_grid

    kf = 2 * np.pi / box
    bgrid = beta(kf * np.sqrt(oracle.kmag2(n).astype(np.float64))) * (1.0 + 0.7 * mu_grid(n) ** 2)
    _, Ea = inj.expected_bispectrum(n, box, edges, bgrid, eps=1.0, lmax=2)
    want = inj.brute_expected(n, box, edges, trips, bgrid, 2)
    assert np.abs(Ea[1]).max() > 1e-2 * np.abs(Ea[0]).max()
    assert np.allclose(Ea[1], want, rtol=1e-10, atol=1e-12 * np.abs(Ea[0]).max())


def test_injected_bispectrum_is_recovered():
    """Sec. VI.B.1 set-up: the estimator's linear response to the injection
    amplitude, [8(B(e)-B(-e)) - (B(2e)-B(-2e))]/(12 e) on one Gaussian seed
    (exact for a cubic polynomial in e), averages to eps-free E[B] for l = 0
    and l = 2 (zero by the cubic symmetry of the grid for an isotropic
    injection)."""
    from oracle import injection as inj
    from oracle import multipoles as ml
    from synthetic import injected_field, injection_beta

    n, box, eps = 32, 2 * np.pi / 0.025, 0.25
    edges = kf_edges(8, 2.0, 2.0)  # [0.05, 0.45) h/Mpc in steps of 0.05
    trips, want = inj.expected_bispectrum(n, box, edges, injection_beta, 1.0, lmax=2)
    c1 = []
    for s in range(40):
        B = {m: ml.bispectrum_multipoles(injected_field(n, box, m * eps, 100 + s), box, edges, 2)[1]
             for m in (-2, -1, 1, 2)}
        c1.append((8 * (B[1] - B[-1]) - (B[2] - B[-2])) / (12 * eps))
    c1 = np.array(c1)
    se = c1.std(0, ddof=1) / np.sqrt(len(c1))
    z = (c1.mean(0) - want) / se
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    assert np.abs(want[1]).max() < 1e-9 * np.abs(want[0]).max()
    live = want[0] != 0
    assert np.median(np.abs(want[0][live]) / se[0][live]) > 5


# --------------------------------------------- bispectrum linear term


def test_linear_term_sums_equal_mode_loops():
    from oracle import masked

    n, box = 8, 300.0
    edges = np.array([1.0, 2.0, 3.0, 4.0])
    w = np.ones((n, n, n))
    w[:, :, :3] = 0.0
    d = w * quadratic_field(n, box, 0.5, 51)
    e = w * gaussian_field(n, box, 52)
    trips, Bc, Bs, _ = masked.bispectrum_linear(d, [e], box, edges)
    T, _ = oracle.triangle_counts(n, edges, trips)
    npix = float(n) ** 3
    lin = masked.brute_linear_sum(d, e, edges, trips)
    assert np.abs(lin.imag).max() < 1e-9 * np.abs(lin.real).max()
    want = box**6 / npix**3 * lin.real / T
    assert np.allclose(Bs - Bc, want, rtol=1e-9, atol=1e-10 * np.abs(want).max())
    res = oracle.bispectrum(d, box, edges)
    assert np.array_equal(res.triplets, trips)
    assert np.allclose(Bs, res.bk, rtol=1e-10, atol=1e-12 * np.abs(res.bk).max())


def test_linear_term_reduces_masked_variance_without_bias():
    """Masked Gaussian data with the linear term estimated from simulations
    through the same window: the large-scale triplets' scatter drops (the
    window breaks translation invariance), and the term averages to zero
    over data realizations (the estimator stays unbiased)."""
    from oracle import masked

    n, box = 24, 1000.0
    edges = kf_edges(5)
    w = window_mask(n, 3, radius=0.3, keep=1.0).astype(np.float64)
    sims = [w * gaussian_field(n, box, 5000 + i) for i in range(40)]
    Bc, Bs = [], []
    for s in range(60):
        trips, bc, bs, _ = masked.bispectrum_linear(w * gaussian_field(n, box, 100 + s), sims, box, edges)
        Bc.append(bc)
        Bs.append(bs)
    Bc, Bs = np.array(Bc), np.array(Bs)
    ratio = Bc.std(0, ddof=1) / Bs.std(0, ddof=1)
    first = trips[:, 0] == 0  # triplets with a leg in the lowest bin
    assert np.median(ratio[first]) < 0.7, ratio[first]
    assert np.median(ratio[~first]) < 1.15
    diff = Bs - Bc  # the subtracted term
    z = diff.mean(0) / (diff.std(0, ddof=1) / np.sqrt(len(diff)))
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()


# --------------------------------------------------- non-cubic geometry


def test_noncubic_reduces_to_cubic():
    from oracle import noncubic as nc

    n, box = 16, 500.0
    edges = kf_edges(5)
    d = quadratic_field(n, box, 1.0, 12)
    a = nc.bispectrum(d, box, edges)
    b = oracle.bispectrum(d, box, edges)
    assert np.array_equal(a.triplets, b.triplets) and np.array_equal(a.counts, b.counts)
    assert np.allclose(a.bk, b.bk, rtol=1e-12, atol=1e-14 * np.abs(b.bk).max())
    assert np.allclose(a.pk, b.pk, rtol=1e-13)


@pytest.mark.parametrize("shape,box,edges", [((8, 6, 4), 300.0, [1.0, 2.0, 3.0]),
                                              ((8, 6, 4), (300.0, 233.0, 171.0), [0.021, 0.045, 0.07, 0.1])])
def test_noncubic_sums_equal_mode_loops(shape, box, edges):
    from oracle import noncubic as nc
    from synthetic import quadratic_field3

    d = quadratic_field3(shape, box, 0.7, 21)
    res = nc.bispectrum(d, box, edges)
    assert len(res.triplets) >= 3
    s, cnt = nc.brute_sums(d, box, edges, res.triplets)
    assert np.array_equal(cnt, res.counts)
    npix = float(np.prod(shape))
    vol = float(np.prod(np.broadcast_to(box, (3,))))
    assert np.abs(s.imag).max() <= 1e-9 * np.abs(s.real).max()
    want = vol * vol / npix**3 * s.real / cnt
    assert np.allclose(res.bk, want, rtol=1e-9, atol=1e-11 * np.abs(want).max())


def test_noncubic_power_and_tree_level_on_anisotropic_box():
    """Gaussian fields on a 24 x 32 x 20 grid of a 600 x 800 x 500 box: P
    averages to the bin mean of the input P(k); the linear-in-f_NL part of B
    of quadratic fields averages to 2(P1P2 + P2P3 + P3P1) over the bin's
    closed triangles (separable form); both with 4.5 standard errors."""
    from oracle import noncubic as nc
    from synthetic import gaussian_field3

    shape, box, f = (24, 32, 20), (600.0, 800.0, 500.0), 0.5
    edges = np.array([0.012, 0.03, 0.05, 0.07, 0.09, 0.11])
    idx = nc.bin_of_modes(shape, box, edges)
    k = np.sqrt(nc.kmag2_phys(shape, box))
    P = pk_model(k)
    nb = len(edges) - 1
    pwant = np.array([P[idx == b].mean() for b in range(nb)])
    trips = oracle.triangle_triplets(edges)
    T, _ = nc.triangle_counts(shape, box, edges, trips)
    trips = trips[T > 0]
    H = nc.unit_fields(shape, box, edges)
    A = np.stack([oracle.idft(np.where(idx == b, P, 0.0)).real for b in range(nb)])
    bwant = np.array([2 * (np.sum(A[a] * A[b] * H[c]) + np.sum(A[a] * H[b] * A[c]) + np.sum(H[a] * A[b] * A[c]))
                      / np.sum(H[a] * H[b] * H[c]) for a, b, c in trips])
    ps, c1s = [], []
    for s in range(100):
        g = gaussian_field3(shape, box, 900 + s)
        g2 = g * g - np.mean(g * g)
        ps.append(nc.power_spectrum(g, box, edges))
        B = {m: nc.bispectrum(g + m * f * g2, box, edges).bk for m in (-2, -1, 1, 2)}
        c1s.append((8 * (B[1] - B[-1]) - (B[2] - B[-2])) / (12 * f))
    ps, c1s = np.array(ps), np.array(c1s)
    zp = (ps.mean(0) - pwant) / (ps.std(0, ddof=1) / np.sqrt(len(ps)))
    assert np.all(np.abs(zp) < 4.5), zp
    se = c1s.std(0, ddof=1) / np.sqrt(len(c1s))
    z = (c1s.mean(0) - bwant) / se
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    assert np.median(np.abs(bwant) / se) > 3


def test_noncubic_multipoles_reduce_and_recover_anisotropic_power():
    """Cubic geometry: the non-cubic multipoles equal ``oracle.multipoles``.
    Anisotropic box: a field whose mode power is exactly c0 + c2 L2 + c4 L4
    in mu = k_z/|k| (physical k) gives back (c0, c2, c4) through the
    discrete Fisher matrix."""
    from oracle import multipoles as ml
    from oracle import noncubic as nc

    n, box = 16, 500.0
    edges = kf_edges(4)
    d = quadratic_field(n, box, 1.0, 5)
    assert np.allclose(nc.power_multipoles(d, box, edges, 4), ml.power_multipoles(d, box, edges, 4),
                       rtol=1e-10, atol=1e-9)
    t1, B1, _ = nc.bispectrum_multipoles(d, box, edges, 2)
    t2, B2 = ml.bispectrum_multipoles(d, box, edges, 2)
    assert np.array_equal(t1, t2)
    assert np.allclose(B1, B2, rtol=1e-9, atol=1e-11 * np.abs(B2).max())
    shape, boxa = (16, 24, 20), (400.0, 650.0, 520.0)
    edges = np.array([0.02, 0.05, 0.08, 0.11, 0.14])
    m2 = nc.mu2_grid(shape, boxa)
    c = (3.0e3, 1.1e3, 4.0e2)
    pw = c[0] + c[1] * (1.5 * m2 - 0.5) + c[2] * (35 * m2 * m2 - 30 * m2 + 3) / 8
    npix, vol = float(np.prod(shape)), float(np.prod(boxa))
    ph = np.random.default_rng(4).uniform(-np.pi, np.pi, shape)
    negs = [(-np.arange(k)) % k for k in shape]
    ph = 0.5 * (ph - ph[np.ix_(*negs)])
    D = np.sqrt(npix**2 / vol * pw) * np.exp(1j * ph)
    D[0, 0, 0] = 0.0
    dfield = np.fft.ifftn(D).real
    P = nc.power_multipoles(dfield, boxa, edges, 4)
    assert np.allclose(P[0], c[0], rtol=1e-9) and np.allclose(P[1], c[1], rtol=1e-9)
    assert np.allclose(P[2], c[2], rtol=1e-8)


def test_weighted_noncubic_grid_deconvolves_per_axis():
    """On a 16 x 24 x 12 grid (box with equal sides) the per-axis window
    sinc(pi n_i / N_i)^p applied in Fourier space is undone, and a constant
    P_fid gives the unweighted non-cubic estimators."""
    from oracle import noncubic as nc
    from oracle import weighted as wt
    from synthetic import quadratic_field3

    shape, box = (16, 24, 12), 400.0
    edges = kf_edges(4)
    d = quadratic_field3(shape, box, 1.0, 31)
    res = nc.bispectrum(d, box, edges)
    const = np.full(int(np.ceil(edges[-1] ** 2)) + 1, 5.0)
    for order in (0, 2, 3):
        dw = np.fft.ifftn(np.fft.fftn(d) * wt.window(shape, order)).real
        assert np.allclose(wt.weighted_power(dw, box, edges, order, const), res.pk, rtol=1e-10)
        trips, B, _, _ = wt.weighted_bispectrum(dw, box, edges, order, const)
        assert np.array_equal(trips, res.triplets)
        assert np.allclose(B, res.bk, rtol=1e-8, atol=1e-10 * np.abs(res.bk).max())


# --------------------------------------------- bispectrum multipole Fisher
def test_bk_fisher_separable_sums_equal_triangle_loops():
    """The separable forms of the discrete ideal Fisher blocks (eq.
    bk-fish-ideal), of N_l (eq. N-ell-def, through the tensor expansion of
    (u2 . u3)^p) and of the numerators (eq. bk-num-ideal) equal explicit
    loops over the closed triangles, in all four bin-degeneracy cases
    (a < b < c, a = b < c, a < b = c, a = b = c), for l, l' <= 4, with
    Nyquist modes in the last bin (directions averaged over +-N/2)."""
    from oracle import bk_fisher as bf

    n, box, edges = 8, 500.0, np.array([1.0, 2.0, 3.0, 4.0, 5.0])  # the last bin holds Nyquist modes
    trips, Ft, Delta, T, Nl = bf.fisher_blocks(n, edges, 4)
    assert sorted({bf._case(*t) for t in trips}) == [0, 1, 2, 3]
    Fb, Nb, Tb = bf.brute_blocks(n, edges, trips, 4)
    assert np.array_equal(T, Tb)
    assert np.abs(Ft - Fb).max() <= 1e-12 * np.abs(Fb).max()
    assert np.abs(Nl - Nb).max() <= 1e-12 * np.abs(Nb).max()
    assert all(np.abs(F - F.T).max() <= 1e-12 * np.abs(F).max() for F in Ft)  # symmetric blocks
    d = quadratic_field(n, box, 1.0, 3)
    nt = bf.numerators(d, box, edges, trips, 4)
    nb = bf.brute_numerators(d, box, edges, trips, 4)
    assert np.abs(nt - nb).max() <= 1e-12 * np.abs(nb).max()
    # Delta of eq. (Delta-alpha-def) in each case
    for t, (a, b, c) in enumerate(trips):
        r = Nl[t] / T[t]
        want = {0: np.ones(3), 1: 2 * np.ones(3), 2: 1 + r, 3: 2 * (1 + 2 * r)}[bf._case(a, b, c)]
        assert np.allclose(Delta[t], want, rtol=0, atol=1e-14)


def test_bk_fisher_limits():
    """l_max = 0 gives the monopole estimator exactly (Delta and the
    permutation factor cancel); the per-triplet mixing R y of the eq.
    (ideal-bk) multipoles equals Delta Ft^+ nt; on an alias-free grid the
    blocks approach the continuum form diag(Delta_l T / (2l+1)) of eq.
    (bk-fish-ideal2)."""
    from oracle import bk_fisher as bf
    from oracle import multipoles as mp

    d = quadratic_field(16, 600.0, 1.0, 5)
    e = np.array([1.0, 3.0, 5.0, 7.0])
    tr0, b0 = bf.bispectrum_multipoles_fisher(d, 600.0, e, 0)
    ref = oracle.bispectrum(d, 600.0, e)
    assert np.array_equal(tr0, ref.triplets)
    assert np.abs(b0[0] - ref.bk).max() <= 1e-12 * np.abs(ref.bk).max()
    tr, b = bf.bispectrum_multipoles_fisher(d, 600.0, e, 4)
    _, y = mp.bispectrum_multipoles(d, 600.0, e, 4)
    trips, Ft, Delta, T, _ = bf.fisher_blocks(16, e, 4)
    R = bf.mixing(Ft, Delta, T, 4)
    by = np.einsum("tij,jt->it", R, y)
    assert np.abs(by - b).max() <= 1e-12 * np.abs(b).max()
    # continuum: 48^3, bins up to 13 k_f (3 x 12 < 48, no aliased closures)
    trips, Ft, Delta, T, _ = bf.fisher_blocks(48, np.array([4.0, 7.0, 10.0, 13.0]), 4)
    ells = np.array([0, 2, 4])
    for t in range(len(trips)):
        s = np.sqrt(Delta[t] * T[t] / (2 * ells + 1))
        M = Ft[t] / np.outer(s, s)
        assert np.abs(np.diag(M) - 1).max() < 0.08
        assert np.abs(M - np.diag(np.diag(M))).max() < 0.05
        assert M[0, 0] == pytest.approx(1.0, abs=1e-12)
