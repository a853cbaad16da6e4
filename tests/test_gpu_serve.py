"""GPU tests of the request loop (paper_2404_07249_amd.serve).

* every request's result in the mix equals, bit for bit, the same request
  computed alone (plan.polyspectra + window_normalize), whatever ran beside
  it or shared its launches;
* masked requests match the FP64 oracle's windowed estimators;
* admission respects the HBM budget (rejection of a job larger than the
  budget, one job at a time under a one-job budget), cancellation and
  expiry of queued requests;
* a short Poisson stream completes with latency statistics.
"""

import sys
import time

import numpy as np
import pytest

import oracle
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


SPECS = [(32, 600.0, kf_edges(8)), (48, 900.0, kf_edges(10)), (64, 1000.0, kf_edges(12))]


def _requests(torch, count=14, masked_every=2, seed0=300):
    from paper_2404_07249_amd.serve import Request

    reqs, host = [], []
    for i in range(count):
        n, box, e = SPECS[(i * 7) % 3 if i % 4 else 0]
        d = quadratic_field(n, box, 1.0, seed0 + i).astype(np.float32)
        w = window_mask(n, seed0 + 1000 + i) if i % masked_every == 0 else None
        data = d * w if w is not None else d
        grfs = sims = None
        if w is not None and i % 4 == 0:
            rng = np.random.default_rng(seed0 + 2000 + i)
            grfs = [torch.from_numpy(rng.standard_normal((n, n, n)).astype(np.float32)).cuda() for _ in range(2)]
        hs = None
        if w is not None and i % 4 == 2:  # simulations through the window: B with the linear term
            hs = [(gaussian_field(n, box, seed0 + 3000 + 8 * i + j) * w).astype(np.float32) for j in range(2)]
            sims = [torch.from_numpy(x).cuda() for x in hs]
        reqs.append(Request(rid=i, grid=n, box=box, edges=e,
                            data=torch.from_numpy(data).cuda(),
                            window=None if w is None else torch.from_numpy(w).cuda(),
                            precision="mixed" if i % 3 else "fp32", grfs=grfs, sims=sims))
        host.append((data, w, hs))
    return reqs, host


def _alone(server, torch, r):
    plan = server.plan_for(r.grid, r.box, r.edges)
    import paper_2404_07249_amd as pb3

    solo = pb3.Plan(r.grid, r.box, r.edges)  # own workspace, same geometry
    if r.sims:
        # the server runs such requests' P as a power-only call and B with the linear term
        pk = solo.power(r.data)
        bk = solo.bispectrum_linear(r.data, r.sims, r.precision)
    else:
        pk, bk = solo.polyspectra(r.data, r.precision)
    if r.window is not None:
        solo.window_normalize(r.window, pk, bk)
    torch.cuda.synchronize()
    assert plan.n_triplets == solo.n_triplets
    return pk.cpu().numpy(), bk.cpu().numpy()


def test_serve_mix_equals_alone_and_oracle(torch_cuda):
    import paper_2404_07249_amd as pb3
    from paper_2404_07249_amd.serve import Server

    torch = torch_cuda
    reqs, host = _requests(torch)
    srv = Server(hbm_budget=8 << 30, max_slots=3)
    for r in reqs:
        srv.submit(r)
    _say("[serve] mix of", len(reqs))
    srv.run_until_idle()
    assert all(srv.done[r.rid].status == "ok" for r in reqs)
    assert srv.stats.max_in_flight >= 2
    assert max(srv.stats.batch_sizes) >= 2  # same-plan requests shared launches
    for r in reqs:
        pk, bk = _alone(srv, torch, r)
        c = srv.done[r.rid]
        assert np.array_equal(c.pk, pk), r.rid
        assert np.array_equal(c.bk, bk), r.rid
        if r.grfs:
            full = pb3.Plan(r.grid, r.box, r.edges, full_grid=True, power_only=True)
            pu, F = full.masked_power(r.data, r.window, r.grfs)
            assert np.array_equal(c.pk_unwindowed, pu.cpu().numpy()), r.rid
            assert np.array_equal(c.fisher, F.cpu().numpy()), r.rid
    assert sum(1 for r in reqs if r.grfs) >= 2
    assert sum(1 for r in reqs if r.sims) >= 2
    # masked requests against the oracle's windowed estimators
    for i in (0, 4):
        r = reqs[i]
        data, w, _ = host[i]
        pw, bw, (m2, m3), res = oracle.windowed_polyspectra(data.astype(np.float64), w, r.box, r.edges)
        c = srv.done[r.rid]
        assert np.allclose(c.moments, [m2, m3], rtol=1e-12, atol=0)
        assert np.all(np.abs(c.pk - pw) <= 1e-5 * np.abs(pw))
        lim = 1e-5 * np.abs(bw) + 1e-6 * res.absnorm / m3
        assert np.all(np.abs(c.bk - bw) <= lim), r.rid
    # a masked request with simulations: the linear term, windowed
    r = reqs[2]
    data, w, hs = host[2]
    d64 = data.astype(np.float64)
    _, blin, _, _ = masked.bispectrum_linear(d64, [x.astype(np.float64) for x in hs], r.box, r.edges)
    m3 = srv.done[r.rid].moments[1]

    def e(f):
        res = oracle.bispectrum(f, r.box, r.edges)
        return 1e-5 * np.abs(res.bk) + 1e-6 * res.absnorm

    lim = 2 * e(d64) + sum(e(x + d64) + e(x - d64) for x in [h.astype(np.float64) for h in hs]) / (2 * len(hs))
    assert np.all(np.abs(srv.done[r.rid].bk - blin / m3) <= lim / m3)


def test_serve_budget_cancel_expire(torch_cuda):
    from paper_2404_07249_amd.serve import Request, Server

    torch = torch_cuda
    n, box, e = SPECS[2]
    reqs = []
    for i in range(6):
        d = quadratic_field(n, box, 1.0, 600 + i).astype(np.float32)
        reqs.append(Request(rid=i, grid=n, box=box, edges=e, data=torch.from_numpy(d).cuda()))
    probe = Server(hbm_budget=1 << 40)
    one = probe.job_bytes(probe.plan_for(n, box, e), False)
    # a budget below one job rejects
    tiny = Server(hbm_budget=1024)
    tiny.submit(reqs[0])
    tiny.run_until_idle()
    assert tiny.done[0].status == "rejected"
    # a one-job budget runs jobs one at a time; queued ones can be cancelled or expire
    srv = Server(hbm_budget=one, max_slots=4, merge_same_plan=False)
    for r in reqs:
        srv.submit(r)
    reqs[4].deadline = time.perf_counter() - 1.0  # already past
    assert srv.cancel(reqs[5].rid)
    srv.run_until_idle()
    assert srv.stats.max_in_flight == 1 and srv.stats.bytes_peak <= one
    assert srv.done[5].status == "cancelled"
    assert srv.done[4].status in ("expired", "ok")
    for r in reqs[:4]:
        c = srv.done[r.rid]
        assert c.status == "ok"
        pk, bk = _alone(srv, torch, r)
        assert np.array_equal(c.bk, bk)


def test_serve_poisson_stream(torch_cuda):
    """A short Poisson stream (mean 200 requests/s) of small jobs, submitted
    at their arrival times while earlier ones run."""
    from paper_2404_07249_amd.serve import Request, Server

    torch = torch_cuda
    rng = np.random.default_rng(5)
    fields = {n: torch.from_numpy(quadratic_field(n, box, 1.0, 40 + n).astype(np.float32)).cuda()
              for n, box, _ in SPECS}
    srv = Server(hbm_budget=4 << 30, max_slots=4)
    t0 = time.perf_counter()
    arrivals = np.cumsum(rng.exponential(1 / 200.0, 40))
    k = 0
    while k < len(arrivals) or not srv.idle:
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k] <= now:
            n, box, e = SPECS[int(rng.integers(0, 3))]
            srv.submit(Request(rid=k, grid=n, box=box, edges=e, data=fields[n], arrival=t0 + arrivals[k]))
            k += 1
        if srv.poll() == 0:
            time.sleep(5e-5)
    s = srv.summary()
    _say("[serve] poisson", s)
    assert s["completed"] == 40
    assert 0 < s["latency_ms"]["p50"] <= s["latency_ms"]["p99"]
