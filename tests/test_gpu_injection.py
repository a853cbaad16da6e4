"""Validation on the paper's injected-bispectrum set-up (Sec. VI.B.1): fields
with an injected bispectrum eps beta1 beta2 beta3, beta = P^(2/3) on
0.1 <= k < 0.4 h/Mpc, measured in 8 bins of 0.05 h/Mpc on [0.05, 0.45)
with l = 0, 2 (98 triplets per multipole, 196 configurations) through
pb3_multipoles on the matrix cores.

The estimator's linear response to eps on each Gaussian seed (exact for the
cubic polynomial in eps) must average to the oracle's expectation within
4.5 standard errors for every configuration, and one field must match the
FP64 oracle within the multipole parity bound.
"""

import sys

import numpy as np
import pytest

from oracle import injection as inj
from oracle import multipoles as mp
from synthetic import injected_field, injection_beta

pytestmark = pytest.mark.gpu

N, BOX, EPS = 48, 2 * np.pi / 0.025, 0.25
EDGES = 0.05 * np.arange(1, 10, dtype=np.float64)  # h/Mpc, given to the plan
EDGES_KF = 2.0 * np.arange(1, 10, dtype=np.float64)  # the same edges in units of k_f, exact


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_injected_bispectrum_recovered_on_gpu(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    _say(f"[case] injection n={N} bins=8 lmax=2 seeds=48")
    plan = pb3.Plan(N, BOX, EDGES, edges_hmpc=True, lmax=2)
    assert plan.n_triplets == 98
    ekf = EDGES_KF  # EDGES / k_f is 6.000000000000001 etc. in floating point; the plan snaps it
    assert np.array_equal(plan.bins()[0], ekf)
    trips, want = inj.expected_bispectrum(N, BOX, ekf, injection_beta, 1.0, lmax=2)
    assert np.array_equal(trips, plan.triplets)
    # one field against the FP64 oracle
    d = injected_field(N, BOX, EPS, 100).astype(np.float32)
    _, bk = plan.multipoles(torch.from_numpy(d).cuda(), power=False)
    bk = bk.cpu().numpy()
    _, bref = mp.bispectrum_multipoles(d.astype(np.float64), BOX, ekf, 2)
    G0 = mp.weighted_fields(d.astype(np.float64), ekf, 0)
    G2 = mp.weighted_fields(d.astype(np.float64), ekf, 2)
    T = plan.norm()[1]
    for i, Gl in enumerate((G0, G2)):
        A = np.array([np.abs(G0[a] * G0[b] * Gl[c]).sum() for a, b, c in trips]) * (4 * i + 1) * BOX**6 / N**3 / T
        assert np.all(np.abs(bk[i] - bref[i]) <= 1e-5 * np.abs(bref[i]) + 1e-6 * A)
    # the linear response to the injection, averaged over seeds
    c1 = []
    for s in range(48):
        B = {}
        for m in (-2, -1, 1, 2):
            x = torch.from_numpy(injected_field(N, BOX, m * EPS, 100 + s).astype(np.float32)).cuda()
            B[m] = plan.multipoles(x, power=False)[1].cpu().numpy()
        c1.append((8 * (B[1] - B[-1]) - (B[2] - B[-2])) / (12 * EPS))
    c1 = np.array(c1)
    se = c1.std(0, ddof=1) / np.sqrt(len(c1))
    z = (c1.mean(0) - want) / se
    _say(f"max |z| = {np.abs(z).max():.2f}")
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    live = want[0] != 0
    assert np.median(np.abs(want[0][live]) / se[0][live]) > 5  # the injection is detected
