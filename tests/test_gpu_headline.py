"""Headline workload (256^3 grid, L = 2000 Mpc/h, 30 bins of width 2 k_f,
3035 triangle-valid triplets) against the full FP64 oracle: every bin of P,
every triplet of B and its exact triangle count, in both precisions, and
the same for an integer-voxel translation of the field.

Gate (FP32 FFTs, FP32-accumulated contraction, FP64 normalisation):
  P:  |dP| <= 1e-5 |P|               every bin
  B:  |dB| <= 1e-5 |B| + 1e-6 A      every triplet
with A the same normalisation applied to sum_x |G_a G_b G_c|.  Each case
adds a summary line (max |dB|/A, relative error p50/p99/max, the fraction
of triplets within 1e-5 relative, the worst bin) to the session report.
"""

import sys
import time

import numpy as np
import pytest

import oracle
from synthetic import field_for

pytestmark = pytest.mark.gpu

P_RTOL = 1e-5
B_RTOL = 1e-5
B_ATOL_A = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def headline():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d, cfg = field_for("c3")
    _say("[case] headline 256^3 x 30 bins: FP64 oracle (fields, counts, all 3035 triplets)")
    t0 = time.time()
    res = oracle.bispectrum(d.astype(np.float64), cfg["box"], cfg["edges"])
    _say(f"[case] oracle done in {time.time() - t0:.1f} s")
    return torch, d, cfg, res


def _run(torch, cfg, field, prec):
    import paper_2404_07249_amd as pb3

    plan = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"])
    x = torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32)).cuda()
    pk, bk = plan.polyspectra(x, precision=prec)
    torch.cuda.synchronize()
    return plan, pk.cpu().numpy(), bk.cpu().numpy()


def _summary(label, res, pk, bk):
    db = np.abs(bk - res.bk)
    rel = db / np.abs(res.bk)
    by_a = db / res.absnorm
    worst = int(np.argmax(by_a))
    # worst |dB|/A among the triplets whose largest bin is c, per c
    per_c = [float(by_a[res.triplets[:, 2] == c].max()) for c in range(int(res.triplets[:, 2].max()) + 1)]
    return (f"{label}: P max rel {np.max(np.abs(pk - res.pk) / np.abs(res.pk)):.2e}; "
            f"B max |dB|/A {by_a.max():.2e} at {tuple(int(v) for v in res.triplets[worst])}, "
            f"rel p50 {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}, "
            f"within 1e-5 rel {np.mean(rel <= 1e-5):.3f}; per-c max |dB|/A "
            + " ".join(f"{v:.1e}" for v in per_c))


def _check(res, plan, pk, bk, label, report):
    assert plan.contract_grid == 192
    assert np.array_equal(plan.triplets, res.triplets), label
    _, cnt = plan.norm()
    assert np.array_equal(cnt.astype(np.int64), res.counts), label
    report.append(_summary(label, res, pk, bk))
    _say(report[-1])
    dp = np.abs(pk - res.pk)
    assert np.all(dp <= P_RTOL * np.abs(res.pk)), (label, float((dp / np.abs(res.pk)).max()))
    db = np.abs(bk - res.bk)
    bad = db > B_RTOL * np.abs(res.bk) + B_ATOL_A * res.absnorm
    assert not bad.any(), (label, int(bad.sum()), float((db / res.absnorm).max()))


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_headline_every_triplet(headline, prec, headline_report):
    torch, d, cfg, res = headline
    assert len(res.triplets) == 3035
    plan, pk, bk = _run(torch, cfg, d, prec)
    _check(res, plan, pk, bk, f"256^3 x 30 bins {prec}", headline_report)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_headline_translation_every_triplet(headline, prec, headline_report):
    """An integer-voxel translation leaves the true P and B unchanged, so the
    translated field's estimates meet the same gate against the oracle of
    the original field."""
    torch, d, cfg, res = headline
    shifted = np.roll(d, (17, -3, 101), axis=(0, 1, 2))
    plan, pk, bk = _run(torch, cfg, shifted, prec)
    _check(res, plan, pk, bk, f"256^3 x 30 bins {prec}, translated by (17, -3, 101)", headline_report)
