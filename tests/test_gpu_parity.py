"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance (FP32 FFTs, FP32 contraction, FP64 normalisation):
  P:  |dP| <= 1e-5 |P|                      for every bin
  B:  |dB| <= 1e-5 |B| + 1e-6 A             for every triplet
where A is the oracle's normalisation applied to sum_x |G_a G_b G_c|.  The
A term covers triplets whose B is a near-cancelling sum (A/|B| up to 1e4);
for well-conditioned triplets the relative bound 1e-5 is what binds.
Triangle counts are integers and must match exactly.
"""

import sys

import numpy as np
import pytest

import oracle
from synthetic import field_for, kf_edges, quadratic_field

pytestmark = pytest.mark.gpu

P_RTOL = 1e-5
B_RTOL = 1e-5
B_ATOL_A = 1e-6


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


def _check_pb(res, pk, bk, trips, label):
    assert np.array_equal(trips, res.triplets), label
    dp = np.abs(pk - res.pk)
    assert np.all(dp <= P_RTOL * np.abs(res.pk)), (label, (dp / np.abs(res.pk)).max())
    db = np.abs(bk - res.bk)
    lim = B_RTOL * np.abs(res.bk) + B_ATOL_A * res.absnorm
    bad = db > lim
    assert not bad.any(), (label, int(bad.sum()), (db / res.absnorm).max())


def _run_case(torch, n, box, edges, delta32, prec="fp32", **plan_kw):
    import paper_2404_07249_amd as pb3

    _say(f"[case] n={n} box={box} bins={len(edges) - 1} prec={prec} {plan_kw}")
    plan = pb3.Plan(n, box, edges, **plan_kw)
    d = _gpu(torch, delta32)
    pk, bk = plan.polyspectra(d, precision=prec)
    torch.cuda.synchronize()
    return plan, pk.cpu().numpy(), bk.cpu().numpy()


PRECS = ["fp32", "mixed"]


@pytest.mark.parametrize("prec", PRECS)
def test_config1_32cubed_parity(torch_cuda, prec):
    torch = torch_cuda
    d, cfg = field_for("c1")
    plan, pk, bk = _run_case(torch, cfg["n"], cfg["box"], cfg["edges"], d, prec)
    res = oracle.bispectrum(d.astype(np.float64), cfg["box"], cfg["edges"])
    nm, cnt = plan.norm()
    assert np.array_equal(nm, res.n_modes)
    assert np.array_equal(cnt.astype(np.int64), res.counts)
    assert plan.n_triplets == 98
    _check_pb(res, pk, bk, plan.triplets, "c1")


@pytest.mark.parametrize("prec", PRECS)
def test_config2_128cubed_parity(torch_cuda, prec):
    torch = torch_cuda
    d, cfg = field_for("c2")
    plan, pk, bk = _run_case(torch, cfg["n"], cfg["box"], cfg["edges"], d, prec)
    res = oracle.bispectrum(d.astype(np.float64), cfg["box"], cfg["edges"])
    _, cnt = plan.norm()
    assert np.array_equal(cnt.astype(np.int64), res.counts)
    _check_pb(res, pk, bk, plan.triplets, "c2")


@pytest.mark.parametrize(
    "n,box,edges",
    [
        (48, 700.0, 1.5 + 2.5 * np.arange(7)),  # radix-3 grid, non-integer edges, ragged tiles
        (96, 2000.0, kf_edges(10)),  # alias-free reduced contraction grid (M = 64 < N)
        (64, 1000.0, kf_edges(24)),  # full spectrum incl. Nyquist; triplets with T = 0 are dropped
        (16, 300.0, np.array([1.0, 3.0, 5.0, 7.0, 9.0, 13.9])),  # tiny grid, heavy aliasing
        (32, 500.0, np.array([2.0, 4.5])),  # a single bin
        (64, 1500.0, 1.0 + 1.5 * np.arange(37)),  # 36 bins: three 16-bin groups, split launches
        (48, 900.0, 1.0 + 2.0 * np.arange(18)),  # 17 bins: one padded 16-bin group
    ],
)
@pytest.mark.parametrize("prec", PRECS)
def test_ragged_and_edge_cases(torch_cuda, n, box, edges, prec):
    torch = torch_cuda
    d = quadratic_field(n, box, 1.0, 123 + n).astype(np.float32)
    plan, pk, bk = _run_case(torch, n, box, edges, d, prec)
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    _, cnt = plan.norm()
    assert np.array_equal(cnt.astype(np.int64), res.counts)
    _check_pb(res, pk, bk, plan.triplets, f"n={n}")


def test_full_grid_flag_matches_reduced_grid(torch_cuda):
    torch = torch_cuda
    n, box = 96, 2000.0
    edges = kf_edges(10)
    d = quadratic_field(n, box, 1.0, 7).astype(np.float32)
    p1, pk1, bk1 = _run_case(torch, n, box, edges, d)
    p2, pk2, bk2 = _run_case(torch, n, box, edges, d, full_grid=True)
    assert p1.contract_grid == 64 and p2.contract_grid == 96
    assert np.array_equal(p1.norm()[1], p2.norm()[1])
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    _check_pb(res, pk2, bk2, p2.triplets, "full grid")


@pytest.mark.parametrize(
    "n,nbins,m",
    [
        (128, 15, 96),  # alias-free contraction grid of 96 points (bounded kz planes)
        (96, 17, 96),   # the full 96-point grid (every plane up to the Nyquist one)
        (128, 24, 128),
        (64, 19, 64),
    ],
)
def test_fused_producer_line_lengths(torch_cuda, n, nbins, m):
    """The fused kernel's z transforms at each line factorisation of its
    producer (96 points as 12 x 8, 128 as 16 x 8, 64 as 8 x 8), on the
    alias-free and the full grid, both precisions, against the oracle."""
    torch = torch_cuda
    box = 2000.0
    edges = kf_edges(nbins)
    d = quadratic_field(n, box, 1.0, 900 + nbins).astype(np.float32)
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    for prec in PRECS:
        plan, pk, bk = _run_case(torch, n, box, edges, d, prec, fuse=True)
        assert plan.contract_grid == m
        _check_pb(res, pk, bk, plan.triplets, f"{prec} n={n} bins={nbins}")


@pytest.mark.parametrize("prec", PRECS)
def test_determinism_and_exact_scaling(torch_cuda, prec):
    """Fixed-order reductions: repeated calls are bitwise equal, and 2*delta
    gives exactly 4 P and 8 B (power-of-two scaling is exact in binary FP,
    the bf16 split included)."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    d, cfg = field_for("c2")
    plan = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"])
    x = _gpu(torch, d)
    pk1, bk1 = [t.cpu().numpy() for t in plan.polyspectra(x, prec)]
    pk2, bk2 = [t.cpu().numpy() for t in plan.polyspectra(x, prec)]
    assert np.array_equal(pk1, pk2) and np.array_equal(bk1, bk2)
    pk3, bk3 = [t.cpu().numpy() for t in plan.polyspectra(2 * x, prec)]
    assert np.array_equal(pk3, 4 * pk1)
    assert np.array_equal(bk3, 8 * bk1)


@pytest.mark.parametrize("case", ["c1", "48^3x13"])
def test_power_alone_equals_polyspectra_and_streams(torch_cuda, case):
    """P from a power-only call (per-bin sums over the mode lists, its own
    final launch) and P from a P + B call (sums taken by the inverse x pass,
    finished in the bispectrum's final launch) add the same FP64 terms in
    different orders: they agree to 1e-13 relative.  A batch of P + B calls
    equals the single P + B calls bit for bit, also with a bin count that
    leaves part of the last four-bin block idle."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    if case == "c1":
        d, cfg = field_for("c1")
    else:
        cfg = {"n": 48, "box": 900.0, "edges": kf_edges(13)}
        d = quadratic_field(48, 900.0, 1.0, 48013).astype(np.float32)
    _say(f"[case] power alone vs polyspectra {case}")
    plan = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"], ext_workspace=True)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind_workspace(ws)
    x = _gpu(torch, d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pk_a = plan.power(x, stream=s)
        pk_b, bk_b = plan.polyspectra(x, stream=s)
    s.synchronize()
    pa, pb = pk_a.cpu().numpy(), pk_b.cpu().numpy()
    assert np.all(np.abs(pa - pb) <= 1e-13 * np.abs(pa)), np.abs(pa / pb - 1).max()
    bk_c = plan.bispectrum(x)
    torch.cuda.synchronize()
    assert np.array_equal(bk_b.cpu().numpy(), bk_c.cpu().numpy())
    if case != "c1":
        other = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"])
        xs = [x, 0.5 * x, x * x]
        bt = pb3.Batch([other] * len(xs))
        pks, _ = bt.run(xs, precision="mixed")
        pko, _ = bt.run(xs, precision="mixed", bispectrum=False)
        for i, xi in enumerate(xs):
            assert np.array_equal(pks[i].cpu().numpy(), other.polyspectra(xi)[0].cpu().numpy()), i
            assert np.array_equal(pko[i].cpu().numpy(), other.power(xi).cpu().numpy()), i


def test_argument_errors_on_device(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    plan = pb3.Plan(32, 1000.0, kf_edges(8))
    with pytest.raises(ValueError):
        plan.power(torch.zeros((32, 32, 16), device="cuda"))
    with pytest.raises(ValueError):
        plan.power(torch.zeros((32, 32, 32), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        plan.power(np.zeros((32, 32, 32), dtype=np.float32))
    p2 = pb3.Plan(32, 1000.0, kf_edges(8), ext_workspace=True)
    with pytest.raises(pb3.Pb3Error):
        p2.power(torch.zeros((32, 32, 32), device="cuda"))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize(
    "n,box,edges",
    [
        (128, 2000.0, kf_edges(20)),  # contraction grid 128, two 16-bin groups
        (96, 2000.0, kf_edges(10)),  # contraction grid 64, one group
        (64, 1000.0, kf_edges(9)),  # contraction grid 64 = N, one 16-bin group
    ],
)
def test_fused_and_separate_z_pass_agree(torch_cuda, prec, n, box, edges):
    """The inverse z pass fused into the contraction (fields never in HBM)
    and the separate z-pass kernel both meet the parity bound."""
    torch = torch_cuda
    d = quadratic_field(n, box, 1.0, 99 + n).astype(np.float32)
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    p1, pk1, bk1 = _run_case(torch, n, box, edges, d, prec)
    p2, pk2, bk2 = _run_case(torch, n, box, edges, d, prec, fuse=False)
    assert p1.contract_grid == p2.contract_grid
    assert p1.workspace_bytes < p2.workspace_bytes  # no filtered fields in the fused workspace
    _check_pb(res, pk1, bk1, p1.triplets, "fused")
    _check_pb(res, pk2, bk2, p2.triplets, "separate")


@pytest.mark.parametrize(
    "n,nbins,m",
    [
        (384, 10, 64),   # largest forward grid, small alias-free contraction grid
        (384, 40, 256),  # 40 bins: three 16-bin groups, separate z pass, G in HBM
        (256, 40, 256),  # contraction on the full grid (3K = 240 < 256 = N)
    ],
)
def test_large_grids_sampled(torch_cuda, n, nbins, m):
    """Serving-size grids: P for every bin against the oracle, B on a
    sample of triplets drawn from four bins (the oracle builds only those
    filtered fields), exact triangle counts on the sample."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    box = 2000.0
    edges = kf_edges(nbins)
    d = quadratic_field(n, box, 1.0, 10000 + n + nbins).astype(np.float32)
    _say(f"[case] large n={n} bins={nbins}")
    plan = pb3.Plan(n, box, edges)
    assert plan.contract_grid == m
    pk, bk = [t.cpu().numpy() for t in plan.polyspectra(_gpu(torch, d), "mixed")]
    d64 = d.astype(np.float64)
    pk_ref = oracle.power_spectrum(d64, box, edges)
    assert np.all(np.abs(pk - pk_ref) <= P_RTOL * np.abs(pk_ref))
    trips = plan.triplets
    rng = np.random.default_rng(n + nbins)
    bins = set(rng.choice(np.arange(1, nbins - 1), 2, replace=False).tolist()) | {0, nbins - 1}
    cand = [i for i, t in enumerate(trips) if set(t.tolist()) <= bins]
    pick = np.array(sorted(rng.choice(cand, min(10, len(cand)), replace=False)))
    s, sa = oracle.triplet_sums_sample(d64, edges, trips[pick])
    T = oracle.count_sample(n, edges, trips[pick])
    _, cnt = plan.norm()
    assert np.array_equal(cnt[pick].astype(np.int64), T)
    scale = box**6 / float(n) ** 3
    bref, aref = scale * s / T, scale * sa / T
    assert np.all(np.abs(bk[pick] - bref) <= B_RTOL * np.abs(bref) + B_ATOL_A * aref)


def test_autotune_with_cache(torch_cuda, tmp_path, monkeypatch):
    """PB3_FLAG_AUTOTUNE times the launch shapes once and records the choice;
    a second plan of the same geometry reads it from the cache.  The tuned
    plan meets the same parity bound against the oracle."""
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PB3_AUTOTUNE_CACHE", str(cache))
    d, cfg = field_for("c2")
    p1 = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"], autotune=True)
    assert p1.launch_shape["tuned"] == "timed"
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and " | " in lines[0]
    p2 = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"], autotune=True)
    assert p2.launch_shape["tuned"] == "cache"
    assert p2.launch_shape["fused"] == p1.launch_shape["fused"]
    assert p2.launch_shape["contract_wgs"] == p1.launch_shape["contract_wgs"]
    _say(f"[case] autotune choice {p1.launch_shape}")
    res = oracle.bispectrum(d.astype(np.float64), cfg["box"], cfg["edges"])
    for prec in PRECS:
        pk, bk = [t.cpu().numpy() for t in p2.polyspectra(_gpu(torch, d), prec)]
        _check_pb(res, pk, bk, p2.triplets, f"tuned {prec}")


@pytest.mark.parametrize(
    "n,nbins",
    [
        (32, 1),   # one bin, one triplet (0, 0, 0)
        (32, 2),   # two bins in one 16-bin group, mostly padding
        (48, 16),  # one full 16-bin group, no padding
        (64, 17),  # a second group holding a single bin
        (96, 32),  # two full groups, the largest fused contraction
        # the layouts that trim a last group of at most 4 or 8 real bins, at their edges
        (32, 4),
        (32, 5),
        (48, 8),
        (48, 9),
        (64, 20),
        (64, 21),
        (64, 24),
        (64, 25),
        (64, 36),  # three groups (separate z pass only)
        (64, 37),
        (64, 40),
        (64, 41),
    ],
)
def test_bin_count_edges(torch_cuda, n, nbins):
    """Bin counts at the edges of the 16-bin MFMA groups (bins of width
    k_f from k_f), fused and separate z pass, both precisions; triangle
    counts exact."""
    torch = torch_cuda
    box = 1000.0
    edges = 1.0 + np.arange(nbins + 1, dtype=np.float64)
    d = quadratic_field(n, box, 1.0, 700 + nbins).astype(np.float32)
    res = oracle.bispectrum(d.astype(np.float64), box, edges)
    for prec in PRECS:
        for fuse in (True, False):
            plan, pk, bk = _run_case(torch, n, box, edges, d, prec, fuse=fuse)
            _check_pb(res, pk, bk, plan.triplets, f"{prec} fuse={fuse}")
            assert np.array_equal(plan.norm()[1].astype(np.int64), res.counts)
