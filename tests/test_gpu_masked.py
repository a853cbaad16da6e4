"""GPU parity of the masked power spectrum with the Monte Carlo Fisher
matrix (pb3_masked_power) against the FP64 oracle (oracle.masked), on the
same window, data and random fields.

Tolerance: FP32 FFTs and FP32 tile sums flushed to FP64 give a Fisher
matrix within 1e-5 of its largest element and an unwindowed power spectrum
within 1e-4 relative (the solve amplifies the Fisher error by at most the
condition number of the bin-normalised Fisher matrix, below 2 here).
"""

import sys

import numpy as np
import pytest

import oracle
from _gates import masked_power_rtol
from oracle import masked
from synthetic import gaussian_field, kf_edges, quadratic_field, window_mask

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize(
    "n,box,nbins,ngrf",
    [
        (24, 600.0, 5, 3),  # z lines below 64 points: the separate inverse and forward z passes
        (64, 1000.0, 12, 4),  # the z round trip at every half-length line factorisation from here on
        (96, 1500.0, 10, 3),
        (128, 2000.0, 16, 2),
        (192, 2000.0, 8, 2),
    ],
)
def test_masked_power_matches_oracle(torch_cuda, n, box, nbins, ngrf):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    edges = kf_edges(nbins)
    _say(f"[case] masked n={n} bins={nbins} grfs={ngrf}")
    w = window_mask(n, 20000 + n)
    d = (quadratic_field(n, box, 1.0, 10000 + n) * w).astype(np.float32)
    rng = np.random.default_rng(30000 + n)
    grfs = [rng.standard_normal((n, n, n)).astype(np.float32) for _ in range(ngrf)]
    plan = pb3.Plan(n, box, edges, full_grid=True, power_only=n >= 64)
    pk, F = plan.masked_power(_gpu(torch, d), _gpu(torch, w), [_gpu(torch, g) for g in grfs])
    pk, F = pk.cpu().numpy(), F.cpu().numpy()
    F_ref = masked.mc_fisher_power(w.astype(np.float64), [g.astype(np.float64) for g in grfs], edges)
    assert np.all(np.abs(F - F_ref) <= 1e-5 * np.abs(F_ref).max()), np.abs(F - F_ref).max() / np.abs(F_ref).max()
    dg = np.sqrt(np.diag(F_ref))
    assert np.linalg.cond(F_ref / np.outer(dg, dg)) < 10  # well conditioned once the bins are normalised
    p_ref = masked.unwindowed_power(d.astype(np.float64), box, edges, F_ref)
    rtol = masked_power_rtol(F_ref)  # about 4e-5: F and p within 1e-5, Skeel condition number about 2
    assert rtol < 5e-5
    assert np.all(np.abs(pk - p_ref) <= rtol * np.abs(p_ref)), np.abs(pk / p_ref - 1).max()


def test_masked_power_refuses_unequal_sides(torch_cuda):
    """The masked estimator is implemented (and checked against the oracle)
    for cubic grids only; other plans get PB3_EUNSUPPORTED."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    shape = (64, 64, 96)
    plan = pb3.Plan(shape, 1000.0, kf_edges(6), full_grid=True, power_only=True)
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    ws = torch.empty(plan.masked_workspace_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="cubic"):
        plan.masked_power(x, x, [x], workspace=ws)


def test_masked_power_without_window_is_box_estimator_in_expectation(torch_cuda):
    """w = 1: F = (1/2) sum_n Theta_a Theta_b |A|^2 / N_pix is diagonal, so P
    equals the box estimator rescaled by the random fields' mode power."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 32, 800.0, kf_edges(6)
    d = quadratic_field(n, box, 0.5, 5).astype(np.float32)
    grfs = [np.random.default_rng(70 + i).standard_normal((n, n, n)).astype(np.float32) for i in range(2)]
    plan = pb3.Plan(n, box, edges, full_grid=True)
    ones = np.ones((n, n, n), np.float32)
    pk, F = [t.cpu().numpy() for t in plan.masked_power(_gpu(torch, d), _gpu(torch, ones),
                                                         [_gpu(torch, g) for g in grfs])]
    off = F - np.diag(np.diag(F))
    assert np.abs(off).max() <= 1e-5 * np.abs(F).max()
    idx = oracle.bin_of_modes(n, edges)
    want_diag = np.zeros(len(edges) - 1)
    for g in grfs:
        A = np.fft.fftn(g.astype(np.float64))
        p2 = (A.real**2 + A.imag**2) / n**3
        want_diag += np.array([0.5 * p2[idx == b].sum() for b in range(len(edges) - 1)])
    want_diag /= len(grfs)
    assert np.allclose(np.diag(F), want_diag, rtol=1e-5)
    pbox = oracle.power_spectrum(d.astype(np.float64), box, edges)
    nm = oracle.mode_counts(n, edges)
    assert np.allclose(pk, 0.5 * nm * pbox / want_diag, rtol=1e-4)


def test_masked_power_argument_errors(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 96, 2000.0, kf_edges(10)
    plan = pb3.Plan(n, box, edges)  # reduced contraction grid
    assert plan.contract_grid < n
    x = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(pb3.Pb3Error):
        plan.masked_power(x, x, [x])
    full = pb3.Plan(32, 500.0, kf_edges(4), full_grid=True, power_only=True)
    assert full.n_triplets == 0
    y = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(pb3.Pb3Error):
        full.masked_power(y, y, [y], workspace=small)
    with pytest.raises(pb3.Pb3Error):
        full.bispectrum(y)  # no bispectrum tables
    full.power(y)


# --------------------------------------------- bispectrum linear term


@pytest.mark.parametrize("n,box,nbins,nsim,prec", [(32, 600.0, 6, 3, "mixed"), (32, 600.0, 6, 5, "fp32"),
                                                   (64, 1000.0, 10, 4, "mixed"), (96, 2000.0, 10, 2, "fp32")])
def test_bispectrum_linear_matches_oracle(torch_cuda, n, box, nbins, nsim, prec):
    """pb3_bispectrum_linear against the FP64 definition (three mixed-leg
    sums per field).  Bound: the single-call bound on each of the 2 n_sim + 1
    bispectra the GPU combines, |dB| <= 2 e(d) + (1/(2 n_sim)) sum_i [e(D_i + d)
    + e(D_i - d)], e(f) = 1e-5 |B(f)| + 1e-6 A(f)."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    edges = kf_edges(nbins)
    _say(f"[case] linear term n={n} bins={nbins} sims={nsim} prec={prec}")
    w = window_mask(n, 21000 + n, radius=0.35)
    d = (quadratic_field(n, box, 1.0, 11000 + n) * w).astype(np.float32)
    sims = [(gaussian_field(n, box, 31000 + 8 * n + i) * w).astype(np.float32) for i in range(nsim)]
    plan = pb3.Plan(n, box, edges)
    bk = plan.bispectrum_linear(_gpu(torch, d), [_gpu(torch, e) for e in sims], precision=prec).cpu().numpy()
    d64 = d.astype(np.float64)
    trips, bref, bplain, _ = masked.bispectrum_linear(d64, [e.astype(np.float64) for e in sims], box, edges)
    assert np.array_equal(trips, plan.triplets)

    def e(f):
        r = oracle.bispectrum(f, box, edges)
        return 1e-5 * np.abs(r.bk) + 1e-6 * r.absnorm

    lim = 2 * e(d64)
    for x in sims:
        x = x.astype(np.float64)
        lim += (e(x + d64) + e(x - d64)) / (2 * nsim)
    assert np.all(np.abs(bk - bref) <= lim), (np.abs(bk - bref) / lim).max()
    assert np.abs(bref - bplain).max() > 100 * lim.max()  # the term is resolved


def test_bispectrum_linear_identity_and_errors(torch_cuda):
    """With the data itself as the only field, S_lin = 3 S(d), so B = -2 B(d)
    exactly (doubling a field is exact in every kernel); argument errors."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 64, 1000.0, kf_edges(12)
    _say("[case] linear term identity / errors")
    d = _gpu(torch, quadratic_field(n, box, 1.0, 77))
    plan = pb3.Plan(n, box, edges)
    for prec in ("mixed", "fp32"):
        b = plan.bispectrum(d, precision=prec)
        bl = plan.bispectrum_linear(d, [d], precision=prec)
        assert torch.equal(bl, -2.0 * b), prec
    with pytest.raises(pb3.Pb3Error):
        plan.bispectrum_linear(d, [], precision="mixed")
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(pb3.Pb3Error):
        plan.bispectrum_linear(d, [d], workspace=small)
    wplan = pb3.Plan(n, box, edges)
    wplan.set_weights(2, None, 0.0)
    with pytest.raises(pb3.Pb3Error):
        wplan.bispectrum_linear(d, [d])
    ponly = pb3.Plan(n, box, edges, power_only=True)
    with pytest.raises(pb3.Pb3Error):
        ponly.bispectrum_linear(d, [d])
