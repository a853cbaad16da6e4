"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only *creates* inputs: Gaussian random fields with a prescribed
power spectrum and the quadratic (local-type) non-Gaussian field built from
them.  It holds none of the estimator's arithmetic (no binning, no shell
filtering, no triplet sums); the oracle and the HIP path each implement that
on their own.

Field model (the workloads of the validation section, Sec. VI, are Gaussian
random fields with a known power spectrum; the quadratic term gives a known
tree-level bispectrum):

    g  : Gaussian, <|g(k)|^2> = V P(k), P(k) = 2e4 (k/0.02)^-1.5 exp(-(k/0.3)^2)
    d  = g + f_NL (g^2 - mean(g^2))

The generator draws ``numpy.random.default_rng(seed).standard_normal`` white
noise in float64, shapes it in Fourier space with sqrt(P N_pix / V), and
returns float64; callers that feed the GPU round it to float32 once and give
the same float32 array to the oracle.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "pk_model",
    "gaussian_field",
    "quadratic_field",
    "kf_edges",
    "field_for",
    "CONFIGS",
    "batch_jobs",
    "window_mask",
    "serve_schedule",
    "injection_beta",
    "injected_field",
    "gaussian_field3",
    "quadratic_field3",
]


def pk_model(k: np.ndarray) -> np.ndarray:
    """Input power spectrum P(k) in (Mpc/h)^3, k in h/Mpc; P(0) = 0."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    m = k > 0
    out[m] = 2e4 * (k[m] / 0.02) ** -1.5 * np.exp(-((k[m] / 0.3) ** 2))
    return out


def _kmag(n: int, box: float) -> np.ndarray:
    """|k| on the rfft half-grid, in h/Mpc."""
    kf = 2.0 * np.pi / box
    f = np.fft.fftfreq(n, d=1.0 / n)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    return kf * np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2)


def gaussian_field(n: int, box: float, seed: int, pk=pk_model) -> np.ndarray:
    """Gaussian random field on an n^3 periodic grid of side ``box`` (float64)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    npix = float(n) ** 3
    vol = float(box) ** 3
    amp = np.sqrt(pk(_kmag(n, box)) * npix / vol)
    amp[0, 0, 0] = 0.0
    return np.fft.irfftn(wk * amp, s=(n, n, n), axes=(0, 1, 2))


def gaussian_field3(shape, box, seed: int, pk=pk_model) -> np.ndarray:
    """Gaussian random field on an Nx x Ny x Nz periodic grid of box sides
    ``box`` (a number or three), float64: <|D(n)|^2> = (N_pix^2 / V) P(|k|)
    with k_i = 2 pi n_i / L_i."""
    shape = tuple(int(s) for s in shape)
    L = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    wk = np.fft.rfftn(w)
    fx = np.fft.fftfreq(shape[0], d=1.0 / shape[0])
    fy = np.fft.fftfreq(shape[1], d=1.0 / shape[1])
    fz = np.arange(shape[2] // 2 + 1, dtype=np.float64)
    k = np.sqrt((2 * np.pi * fx[:, None, None] / L[0]) ** 2 + (2 * np.pi * fy[None, :, None] / L[1]) ** 2
                + (2 * np.pi * fz[None, None, :] / L[2]) ** 2)
    npix = float(np.prod(shape))
    amp = np.sqrt(pk(k) * npix / float(np.prod(L)))
    amp[0, 0, 0] = 0.0
    return np.fft.irfftn(wk * amp, s=shape, axes=(0, 1, 2))


def quadratic_field3(shape, box, fnl: float, seed: int, pk=pk_model) -> np.ndarray:
    """d = g + f_NL (g^2 - mean(g^2)) with g from :func:`gaussian_field3`."""
    g = gaussian_field3(shape, box, seed, pk)
    return g + fnl * (g * g - np.mean(g * g))


def injection_beta(k, kmin: float = 0.1, kmax: float = 0.4, pk=pk_model) -> np.ndarray:
    """beta(k) = P(k)^(2/3) on kmin <= k < kmax, zero elsewhere: the injected
    bispectrum's factor (validation set-up of Sec. VI.B.1)."""
    k = np.asarray(k, dtype=np.float64)
    return np.where((k >= kmin) & (k < kmax), pk(k) ** (2.0 / 3.0), 0.0)


def injected_field(n: int, box: float, eps: float, seed: int, kmin: float = 0.1, kmax: float = 0.4,
                   pk=pk_model) -> np.ndarray:
    """Gaussian field g with an injected bispectrum eps beta1 beta2 beta3
    (Sec. VI.B.1): d = g + (eps/6) IDFT[beta DFT[phi^2]], phi = IDFT[(beta/P) DFT[g]]
    (numpy DFT normalisation, so the volume factors of the continuum form
    cancel).  The same seed gives the same g for every eps."""
    g = gaussian_field(n, box, seed, pk)
    k = _kmag(n, box)
    beta = injection_beta(k, kmin, kmax, pk)
    P = pk(k)
    ratio = np.divide(beta, P, out=np.zeros_like(beta), where=P > 0)
    phi = np.fft.irfftn(np.fft.rfftn(g) * ratio, s=(n, n, n), axes=(0, 1, 2))
    extra = np.fft.irfftn(np.fft.rfftn(phi * phi) * beta, s=(n, n, n), axes=(0, 1, 2))
    return g + (eps / 6.0) * extra


def quadratic_field(n: int, box: float, fnl: float, seed: int, pk=pk_model) -> np.ndarray:
    """d = g + f_NL (g^2 - mean(g^2)) with g from :func:`gaussian_field`."""
    g = gaussian_field(n, box, seed, pk)
    return g + fnl * (g * g - np.mean(g * g))


def kf_edges(n_bins: int, width: float = 2.0, start: float = 1.0) -> np.ndarray:
    """Linear bin edges in units of the fundamental k_f: start + width*j."""
    return start + width * np.arange(n_bins + 1, dtype=np.float64)


# The five workloads (grid, box in Mpc/h, bins, f_NL, seed).  Bins are of
# width 2 k_f starting at k_f.
CONFIGS = {
    "c1": dict(n=32, box=1000.0, n_bins=8, fnl=0.5, seed=0),
    "c2": dict(n=128, box=2000.0, n_bins=20, fnl=1.0, seed=1),
    "c3": dict(n=256, box=2000.0, n_bins=30, fnl=1.0, seed=2),
}


def field_for(name: str, seed: int | None = None) -> tuple[np.ndarray, dict]:
    """Float32 input field for a named workload, plus its parameters."""
    cfg = dict(CONFIGS[name])
    if seed is not None:
        cfg["seed"] = seed
    d = quadratic_field(cfg["n"], cfg["box"], cfg["fnl"], cfg["seed"]).astype(np.float32)
    cfg["edges"] = kf_edges(cfg["n_bins"])
    return d, cfg


def batch_jobs(n_jobs: int = 64, grids=(64, 96, 128), box: float = 2000.0, fnl: float = 1.0,
               seed0: int = 1000, with_fields: bool = True):
    """The batched workload: job i has grid grids[i mod 3], 16 + (i mod 9)
    bins of width 2 k_f from k_f (bins fixed in k_f units, so one box side
    serves every grid), seed seed0 + i.  Returns a list of dicts (n, box,
    edges, seed, and the float32 field when ``with_fields``)."""
    jobs = []
    for i in range(n_jobs):
        n = grids[i % len(grids)]
        job = dict(n=n, box=box, n_bins=16 + (i % 9), fnl=fnl, seed=seed0 + i)
        job["edges"] = kf_edges(job["n_bins"])
        if with_fields:
            job["field"] = quadratic_field(n, box, fnl, job["seed"]).astype(np.float32)
        jobs.append(job)
    return jobs


def window_mask(n: int, seed: int, radius: float = 0.45, keep: float = 0.95) -> np.ndarray:
    """Binary survey-like window on an n^3 grid: voxels whose centre lies
    within ``radius`` box sides of the box centre, each kept with
    probability ``keep`` (independent holes).  float32."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n - 0.5
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    rng = np.random.default_rng(seed)
    holes = rng.random((n, n, n)) < keep
    return ((r2 < radius * radius) & holes).astype(np.float32)


def serve_schedule(n_requests: int, rate: float = 20.0, seed: int = 5, grids=(64, 128, 256, 384),
                   min_bins: int = 10, max_bins: int = 40, max_bins_64: int = 28):
    """A Poisson request stream: exponential inter-arrival times of mean
    1/rate seconds, grid uniform over ``grids``, bin count uniform in
    [min_bins, max_bins] (at most ``max_bins_64`` on 64^3, whose shells
    above |n| = 32 sqrt(3) are empty); field seed 10000 + i, window seed
    20000 + i.  Returns dicts (arrival offset in s, grid, n_bins, edges,
    field_seed, window_seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(grids))
        hi = max_bins_64 if n == 64 else max_bins
        nb = int(rng.integers(min_bins, hi + 1))
        out.append(dict(rid=i, arrival=t, n=n, n_bins=nb, edges=kf_edges(nb), field_seed=10000 + i,
                        window_seed=20000 + i))
    return out
