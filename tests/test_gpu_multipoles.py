"""GPU parity of the power and bispectrum multipoles (pb3_multipoles, line
of sight along z) against the FP64 oracle (oracle.multipoles).

Both precisions: split-bf16 x3 on the matrix cores and FP32 tiles.
Tolerance: P_l within 1e-4 of P_0 in every bin (the quadrupole and
hexadecapole of an isotropic field are near zero, so their error is judged
against the monopole); B_l within 1e-5 |B_l| + 1e-6 A_l with
A_l = (2l+1) (V^2/N_pix) sum_x |G_a G_b g_{c,l}| / T, the bound of the
monopole parity tests.
"""

import sys

import numpy as np
import pytest

import oracle
from _gates import multipole_gain, multipole_power_gate
from oracle import multipoles as mp
from synthetic import kf_edges, quadratic_field

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


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
@pytest.mark.parametrize("n,box,nbins,width,lmax", [(32, 600.0, 8, 2.0, 4), (64, 1000.0, 12, 2.0, 2),
                                                    (96, 2000.0, 10, 2.0, 4), (64, 1500.0, 36, 1.5, 2)])
def test_multipoles_match_oracle(torch_cuda, n, box, nbins, width, lmax, prec):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    edges = kf_edges(nbins, width=width)
    _say(f"[case] multipoles n={n} bins={nbins} lmax={lmax} prec={prec}")
    # an anisotropic field: stretch the quadratic field's modes along z
    d = quadratic_field(n, box, 1.0, 70 + n)
    D = np.fft.fftn(d)
    mu = mp.mu_grid(n)
    d = np.fft.ifftn(D * (1.0 + 0.8 * mu * mu)).real.astype(np.float32)
    plan = pb3.Plan(n, box, edges, lmax=lmax)
    assert plan.n_ell == lmax // 2 + 1
    pk, bk = [t.cpu().numpy() for t in plan.multipoles(torch.from_numpy(d).cuda(), precision=prec)]
    d64 = d.astype(np.float64)
    pref = mp.power_multipoles(d64, box, edges, lmax)
    gain = multipole_gain(oracle.bin_of_modes(n, edges), mp.mu_grid(n) ** 2, len(edges) - 1, lmax)
    gate = multipole_power_gate(gain, pref[0])
    assert np.all(np.abs(pk - pref) <= gate), (np.abs(pk - pref) / gate).max()
    assert np.all(np.abs(pk[0] - pref[0]) <= 1e-5 * np.abs(pref[0]))  # the monopole at the P gate
    trips, bref = mp.bispectrum_multipoles(d64, box, edges, lmax)
    assert np.array_equal(trips, plan.triplets)
    T = plan.norm()[1]
    G0 = mp.weighted_fields(d64, edges, 0)
    npix = float(n) ** 3
    for i, ell in enumerate(range(0, lmax + 1, 2)):
        Gl = mp.weighted_fields(d64, edges, ell)
        A = np.array([np.abs(G0[a] * G0[b] * Gl[c]).sum() for a, b, c in trips])
        A *= (2 * ell + 1) * box**6 / npix / T
        lim = 1e-5 * np.abs(bref[i]) + 1e-6 * A
        assert np.all(np.abs(bk[i] - bref[i]) <= lim), (ell, (np.abs(bk[i] - bref[i]) / A).max())
    # the monopole row is the monopole estimator (within the same bound)
    res = oracle.bispectrum(d64, box, edges)
    assert np.all(np.abs(bk[0] - res.bk) <= 1e-5 * np.abs(res.bk) + 1e-6 * res.absnorm)


def test_multipoles_argument_errors(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    plan = pb3.Plan(32, 600.0, kf_edges(6))  # no multipoles
    x = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(pb3.Pb3Error):
        plan.multipoles(x)
    ml = pb3.Plan(32, 600.0, kf_edges(6), lmax=2)
    with pytest.raises(pb3.Pb3Error):
        ml.multipoles(x, workspace=torch.empty(8, dtype=torch.uint8, device="cuda"))
