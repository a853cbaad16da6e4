"""GPU tests of the batched form (pb3_batch_* / pb3_bispectrum_batched).

Every job of a batch must equal, bit for bit, the same plan's single call
on the same field (same kernels, same fixed-order reductions); sampled jobs
are also checked against the FP64 oracle with the parity bound of the
single-call tests.  Graph replays are checked against eager results on
every replay, with eager work and synchronisation between replays.
"""

import sys

import numpy as np
import pytest

import oracle
from synthetic import batch_jobs, kf_edges, quadratic_field

pytestmark = pytest.mark.gpu

B_RTOL = 1e-5
B_ATOL_A = 1e-6
P_RTOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)).cuda()


def _singles(plans, xs, prec):
    out = []
    for p, x in zip(plans, xs):
        pk, bk = p.polyspectra(x, prec)
        out.append((pk.cpu().numpy(), bk.cpu().numpy()))
    return out


def _small_mix(torch):
    """Eleven jobs over three plans; the 32^3 plan has nine jobs, so its
    launches split into groups of eight and one."""
    import paper_2404_07249_amd as pb3

    specs = [(32, 600.0, kf_edges(8)), (48, 900.0, 1.5 + 2.5 * np.arange(7)), (64, 1000.0, kf_edges(12))]
    plans = [pb3.Plan(n, box, e) for n, box, e in specs]
    order = [0, 1, 0, 0, 2, 0, 0, 0, 0, 0, 0]
    jplans = [plans[i] for i in order]
    fields = [quadratic_field(specs[i][0], specs[i][1], 1.0, 500 + j).astype(np.float32) for j, i in enumerate(order)]
    return specs, order, plans, jplans, fields


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_batch_equals_single_calls_bitwise(torch_cuda, prec):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    specs, order, plans, jplans, fields = _small_mix(torch)
    xs = [_gpu(torch, f) for f in fields]
    _say(f"[batch] eager, {len(xs)} jobs, prec={prec}")
    b = pb3.Batch(jplans)
    assert b.groups == 4
    pks, bks = b.run(xs, prec)
    torch.cuda.synchronize()
    ref = _singles(jplans, xs, prec)
    for j, (pk, bk) in enumerate(ref):
        assert np.array_equal(pks[j].cpu().numpy(), pk), j
        assert np.array_equal(bks[j].cpu().numpy(), bk), j
    # one job of each plan against the oracle
    for i, (n, box, e) in enumerate(specs):
        j = order.index(i)
        res = oracle.bispectrum(fields[j].astype(np.float64), box, e)
        assert np.array_equal(jplans[j].triplets, res.triplets)
        pk, bk = ref[j]
        assert np.all(np.abs(pk - res.pk) <= P_RTOL * np.abs(res.pk))
        assert np.all(np.abs(bk - res.bk) <= B_RTOL * np.abs(res.bk) + B_ATOL_A * res.absnorm)


def test_batch_statistic_subsets_and_one_shot(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    specs, order, plans, jplans, fields = _small_mix(torch)
    xs = [_gpu(torch, f) for f in fields]
    ref = _singles(jplans, xs, "mixed")
    ref_p = [p.power(x).cpu().numpy() for p, x in zip(jplans, xs)]  # power-only calls: the same route
    b = pb3.Batch(jplans)
    pks, bks = b.run(xs, "mixed", bispectrum=False)
    assert bks is None
    _, bks = b.run(xs, "mixed", power=False)
    torch.cuda.synchronize()
    for j, (pk, bk) in enumerate(ref):
        assert np.array_equal(pks[j].cpu().numpy(), ref_p[j])
        assert np.all(np.abs(ref_p[j] - pk) <= 1e-13 * np.abs(pk))
        assert np.array_equal(bks[j].cpu().numpy(), bk)
    outs = pb3.bispectrum_batched(jplans, xs, "mixed")
    for j, (_, bk) in enumerate(ref):
        assert np.array_equal(outs[j].cpu().numpy(), bk)


def test_batch_graph_replays_match_eager(torch_cuda):
    """Captured once, replayed with new input contents in the same buffers
    (eager single calls and synchronisation between replays), then run with
    other output buffers (capture again, graph updated)."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    specs, order, plans, jplans, fields = _small_mix(torch)
    xs = [_gpu(torch, f) for f in fields]
    b = pb3.Batch(jplans, graph=True)
    pk_out = [torch.empty(p.n_bins, dtype=torch.float64, device="cuda") for p in jplans]
    bk_out = [torch.empty(p.n_triplets, dtype=torch.float64, device="cuda") for p in jplans]
    for rep in range(4):
        _say(f"[graph] replay {rep}")
        for j, x in enumerate(xs):  # new contents, same buffers
            x.copy_(_gpu(torch, quadratic_field(x.shape[0], 700.0, 1.0, 900 + 31 * rep + j)))
        ref = _singles(jplans, xs, "mixed")  # eager work between replays
        torch.cuda.synchronize()
        b.run(xs, "mixed", pk_outs=pk_out, bk_outs=bk_out)
        torch.cuda.synchronize()
        for j, (pk, bk) in enumerate(ref):
            assert np.array_equal(pk_out[j].cpu().numpy(), pk), (rep, j)
            assert np.array_equal(bk_out[j].cpu().numpy(), bk), (rep, j)
    # other outputs and precision: captured again
    pks, bks = b.run(xs, "fp32")
    torch.cuda.synchronize()
    ref = _singles(jplans, xs, "fp32")
    for j, (pk, bk) in enumerate(ref):
        assert np.array_equal(pks[j].cpu().numpy(), pk)
        assert np.array_equal(bks[j].cpu().numpy(), bk)


def test_batch_bound_workspace_and_errors(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    specs, order, plans, jplans, fields = _small_mix(torch)
    xs = [_gpu(torch, f) for f in fields]
    b = pb3.Batch(jplans, ext_workspace=True)
    with pytest.raises(pb3.Pb3Error):
        b.run(xs, "mixed")  # no workspace bound yet
    ws = torch.empty(b.workspace_bytes // 8 + 1, dtype=torch.float64, device="cuda")
    b.bind_workspace(ws)
    pks, bks = b.run(xs, "mixed")
    torch.cuda.synchronize()
    ref = _singles(jplans, xs, "mixed")
    for j, (pk, bk) in enumerate(ref):
        assert np.array_equal(bks[j].cpu().numpy(), bk)
    with pytest.raises(pb3.Pb3Error):
        pb3.Batch([])
    host = pb3.Plan(32, 600.0, kf_edges(8), host_only=True)
    with pytest.raises(pb3.Pb3Error):
        pb3.Batch([host])


def test_batched_workload_64_jobs(torch_cuda):
    """The batched workload: 64 realizations on 64^3, 96^3 and 128^3 grids
    with 16-24 bins (nine distinct plans), mixed precision, graph replay:
    every job bitwise equal to its single call; one job per grid against
    the oracle on a sample of triplets, and its power spectrum in full."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    jobs = batch_jobs(64)
    cache = {}
    jplans = []
    for jb in jobs:
        key = (jb["n"], jb["n_bins"])
        if key not in cache:
            cache[key] = pb3.Plan(jb["n"], jb["box"], jb["edges"])
        jplans.append(cache[key])
    assert len(cache) == 9
    xs = [_gpu(torch, jb["field"]) for jb in jobs]
    _say("[batch64] graph run")
    b = pb3.Batch(jplans, graph=True)
    pks, bks = b.run(xs, "mixed")
    pks2, bks2 = b.run(xs, "mixed")  # replay
    torch.cuda.synchronize()
    ref = _singles(jplans, xs, "mixed")
    for j, (pk, bk) in enumerate(ref):
        assert np.array_equal(pks[j].cpu().numpy(), pk), j
        assert np.array_equal(bks[j].cpu().numpy(), bk), j
        assert np.array_equal(bks2[j].cpu().numpy(), bk), j
    rng = np.random.default_rng(3)
    for j in (0, 1, 2):
        jb = jobs[j]
        d64 = jb["field"].astype(np.float64)
        p_ref = oracle.power_spectrum(d64, jb["box"], jb["edges"])
        assert np.all(np.abs(ref[j][0] - p_ref) <= P_RTOL * np.abs(p_ref)), j
        trips = jplans[j].triplets
        pick = np.array(sorted(rng.choice(len(trips), 12, replace=False)))
        s, sa = oracle.triplet_sums_sample(d64, jb["edges"], trips[pick])
        T = oracle.count_sample(jb["n"], jb["edges"], trips[pick])
        _, cnt = jplans[j].norm()
        assert np.array_equal(cnt[pick].astype(np.int64), T)
        scale = jb["box"] ** 6 / float(jb["n"]) ** 3
        bref, aref = scale * s / T, scale * sa / T
        assert np.all(np.abs(ref[j][1][pick] - bref) <= B_RTOL * np.abs(bref) + B_ATOL_A * aref), j
