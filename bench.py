#!/usr/bin/env python3
"""Throughput of the idealized P(k) + bispectrum hot path on one MI355X.

One step = one pass of the whole path over one synthetic field: forward r2c
FFT, shell-binned power spectrum, per-bin shell-filtered inverse FFTs,
triplet contraction and normalisation (pb3_polyspectra).  The plan (bins,
triplets, FP64 triangle counts) is built once, outside the timed region;
the input field is resident in HBM before timing starts.

Workload: 256^3 grid, L = 2000 Mpc/h, 30 bins of width 2 k_f from k_f
(3035 triangle-valid triplets), d = g + f_NL (g^2 - <g^2>) with f_NL = 1.

Prints ONE JSON line (rank 0).  ``--gpus`` above 1 is refused: the library
runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "bispectra/s at 256³×30 bins, mixed vs FP32 at fixed error; p50/p99 latency"

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# plain (non-packed) FP32 vector FMA: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# HBM traffic of the dominant kernel at this workload from two rocprofv3
# counter passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), scaled by what
# the same counters read for a device copy of known size (reads x2.0,
# writes x1.0).  Valid only for the kernel sources it was taken on: the
# figure is dropped (null) once their hash differs.
MEASURED_TRAFFIC = {
    ("contract", "mixed"): {
        "kernel": "k_zcontract<2, 1, true, 192, 66>",
        "contract_wgs": 1024,  # partial-vector writes scale with the accumulation-chunk count
        "fetch_kib": 138396.3, "write_kib": 30720.0, "fetch_factor": 2.0, "write_factor": 1.0,
        "sources": {
            "paper_2404_07249_amd/csrc/contract_mfma.hip":
                "a644e279a7f4f7d5212951b136696c322771c75e980315e1a41750445b1bb553",
            "paper_2404_07249_amd/csrc/fft_dev.h":
                "2752fa569bc89ad3a05efa2efbe4f4ec86f50a872389150178fca1ac9217f2e2",
            "paper_2404_07249_amd/csrc/job.h":
                "0f3d39c847bc50252698d89b0082866e4ca72f6f435cacd590aacb25667591d2",
        },
    },
    ("contract", "fp32"): {
        "kernel": "k_zcontract<2, 1, false, 192, 66>",
        "contract_wgs": 1024,
        "fetch_kib": 139862.5, "write_kib": 30720.0, "fetch_factor": 2.0, "write_factor": 1.0,
        "sources": {
            "paper_2404_07249_amd/csrc/contract_mfma.hip":
                "a644e279a7f4f7d5212951b136696c322771c75e980315e1a41750445b1bb553",
            "paper_2404_07249_amd/csrc/fft_dev.h":
                "2752fa569bc89ad3a05efa2efbe4f4ec86f50a872389150178fca1ac9217f2e2",
            "paper_2404_07249_amd/csrc/job.h":
                "0f3d39c847bc50252698d89b0082866e4ca72f6f435cacd590aacb25667591d2",
        },
    },
}


def measured_traffic(stage: str, precision: str, contract_wgs=None):
    """HBM bytes per launch of ``stage`` from the counter passes, or None
    (no record, sources changed since, or another launch shape)."""
    import hashlib

    t = MEASURED_TRAFFIC.get((stage, precision))
    if t is None:
        return None
    if "contract_wgs" in t and contract_wgs is not None and contract_wgs != t["contract_wgs"]:
        return None
    for rel, digest in t["sources"].items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


def _cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def stage_work(plan_info: dict, precision: str) -> dict:
    """Algorithmic bytes (HBM-bound stages) or flops (contraction) of one
    launch of each stage, from the plan geometry."""
    n, kz, lc, m, nb = plan_info["N"], plan_info["Kz"], plan_info["Lc"], plan_info["M"], plan_info["nb"]
    geom = plan_info["geom"]
    c8, f4 = 8, 4
    w = {}
    w["fwd_z"] = ("hbm", n**3 * f4 + n * n * kz * c8)
    w["fwd_y"] = ("hbm", n * n * kz * c8 + n * lc * kz * c8)
    w["fwd_x"] = ("hbm", n * lc * kz * c8 + lc * lc * kz * c8)
    w["power"] = ("hbm", plan_info["n_modes_half"] * (4 + c8))
    w["inv_x"] = ("hbm", sum(ly * ly * kzn * c8 + m * ly * kzn * c8 for ly, kzn in geom))
    w["inv_y"] = ("hbm", sum(m * ly * kzn * c8 + m * m * kzn * c8 for ly, kzn in geom))
    w["inv_z"] = ("hbm", sum(m * m * kzn * c8 + m**3 * f4 for ly, kzn in geom))
    # the method's work (eq. beta-def): per voxel one product per pair a <= b
    # and a multiply-add per triangle-valid triplet
    n_pairs = nb * (nb + 1) // 2
    w["contract"] = ("flops", float(n_pairs + 2 * plan_info["n_trip"]) * m**3)
    w["reduce"] = ("hbm", 0)
    return w


def dense_gemm_flops(plan_info: dict) -> float:
    """Flops of the contraction recast as a dense GEMM (every pair a <= b
    against every bin c over the M^3 voxels): what the matrix cores would
    execute without the triangle condition, for comparison only."""
    nb, m = plan_info["nb"], plan_info["M"]
    return 2.0 * (nb * (nb + 1) // 2) * nb * m**3


def stage_rates(work: dict, stages: dict, precision: str) -> dict:
    """Achieved rate of every timed stage against its roofline: GB/s of
    algorithmic bytes for the HBM-bound passes, TFLOP/s of the method's
    contraction work for the contraction (which also carries the fused
    inverse z pass)."""
    out = {}
    for k, (kind, amount) in work.items():
        ms = stages.get(k, (0.0, 0))[0]
        if ms <= 0 or amount <= 0:
            continue
        if kind == "flops":
            peak = BF16_PEAK_TFLOPS if precision == "mixed" else FP32_MFMA_PEAK_TFLOPS
            a = amount / (ms * 1e-3) / 1e12
            out[k] = {"TFLOP/s": round(a, 2), "frac": round(a / peak, 4)}
        else:
            a = amount / (ms * 1e-3) / 1e9
            out[k] = {"GB/s": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4)}
    return out


def batched_bench(reps: int = 10, warmup: int = 2, precision: str = "mixed", autotune: bool = True) -> dict:
    """The batched workload (64 realizations on 64^3/96^3/128^3 grids with
    16-24 bins, nine distinct plans): throughput of one call per field on
    one stream, of the batch (shared launches, concurrent plan groups) and
    of the batch replayed from a HIP graph.  P and B for every field."""
    import torch

    import paper_2404_07249_amd as pb3
    from synthetic import batch_jobs

    jobs = batch_jobs(64)
    cache = {}
    plans = []
    for jb in jobs:
        key = (jb["n"], jb["n_bins"])
        if key not in cache:
            cache[key] = pb3.Plan(jb["n"], jb["box"], jb["edges"], autotune=autotune)
        plans.append(cache[key])
    xs = [torch.from_numpy(jb["field"]).cuda() for jb in jobs]
    pk = [torch.empty(p.n_bins, dtype=torch.float64, device="cuda") for p in plans]
    bk = [torch.empty(p.n_triplets, dtype=torch.float64, device="cuda") for p in plans]
    stream = torch.cuda.current_stream()
    eager = pb3.Batch(plans)
    graph = pb3.Batch(plans, graph=True)
    n_l = {id(p): p_launches(p) for p in cache.values()}

    def singles():
        for p, x, a, b in zip(plans, xs, pk, bk):
            p.polyspectra(x, precision, pk_out=a, bk_out=b, stream=stream)

    modes = {
        "single_calls": singles,
        "batch": lambda: eager.run(xs, precision, pk_outs=pk, bk_outs=bk, stream=stream),
        "batch_graph": lambda: graph.run(xs, precision, pk_outs=pk, bk_outs=bk, stream=stream),
    }
    rates, ms = {}, {}
    for name, fn in modes.items():
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rates[name] = len(jobs) * reps / dt
        ms[name] = 1e3 * dt / reps
    return {
        "workload": "64 realizations, grids 64^3/96^3/128^3 (job i: grid (64,96,128)[i%3], 16+(i%9) bins of "
                    "width 2k_f), L=2000 Mpc/h, f_NL=1; P+B per field",
        "precision": precision,
        "plans": len(cache),
        "launch_groups": graph.groups,
        "launches_per_run": graph.launches(),
        "launches_single_calls": sum(n_l[id(p)] for p in plans),
        "bispectra_per_s": rates,
        "ms_per_batch": ms,
        "speedup_graph_vs_single": rates["batch_graph"] / rates["single_calls"],
        "launch_shapes": {f"{k[0]}^3x{k[1]}": [int(p.launch_shape["fused"]), p.launch_shape["contract_wgs"]]
                          for k, p in cache.items()},
    }


def masked_bench(reps: int = 3, warmup: int = 2, n_mc: int = 8) -> dict:
    """The masked power spectrum with its Monte Carlo Fisher matrix (the
    dominant part of a serving request) on full-grid, power-only plans:
    a random window of 95% ones, masked Gaussian data and n_mc white random
    fields, all drawn on the device; ms per call."""
    import torch

    import paper_2404_07249_amd as pb3
    from synthetic import kf_edges

    out = {}
    for n, nb in ((384, 40), (256, 30), (128, 20)):
        plan = pb3.Plan(n, 2000.0, kf_edges(nb), full_grid=True, power_only=True)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        w = (torch.rand((n, n, n), generator=g, device="cuda") < 0.95).float()
        d = torch.randn((n, n, n), generator=g, device="cuda") * w
        grfs = [torch.randn((n, n, n), generator=g, device="cuda") for _ in range(n_mc)]
        ws = torch.empty(plan.masked_workspace_bytes, dtype=torch.uint8, device="cuda")
        for _ in range(warmup):
            plan.masked_power(d, w, grfs, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.masked_power(d, w, grfs, workspace=ws)
        torch.cuda.synchronize()
        out[f"{n}^3x{nb}"] = {"ms_per_call": round(1e3 * (time.perf_counter() - t0) / reps, 2), "n_mc": n_mc,
                              "workspace_gb": round(plan.masked_workspace_bytes / 1e9, 2)}
        del grfs, ws, w, d
        torch.cuda.empty_cache()
    return out


def serving_bench(n_requests: int = 200, rate: float = 20.0, budget_gb: float = 96.0, slots: int = 4,
                  precision: str = "mixed", n_mc: int = 8) -> dict:
    """Poisson request stream through the continuous-batching server: grids
    uniform over 64^3..384^3, 10-40 bins (<= 28 on 64^3), each field times a
    sphere-with-holes window (radius 0.45 L, 5% holes, drawn per request on
    the device), windowed normalisation, and the unwindowed power spectrum
    with a Monte Carlo Fisher matrix from ``n_mc`` white random fields per
    request (drawn on the device, seeds 30000 + 8 i + j).  Plans for every geometry in the
    stream are built and run once before the clock starts (device-resident
    plans, kernels loaded); fields come from a pool of two realizations per
    grid (one at 384^3)."""
    import torch

    from paper_2404_07249_amd.serve import Request, Server
    from synthetic import quadratic_field, serve_schedule

    box = 2000.0
    sched = serve_schedule(n_requests, rate=rate, seed=5)
    pool = {}
    for n in (64, 128, 256, 384):
        k = 1 if n == 384 else 2
        pool[n] = [torch.from_numpy(quadratic_field(n, box, 1.0, 10000 + 97 * n + j).astype(np.float32)).cuda()
                   for j in range(k)]
    spheres = {}
    for n in pool:
        c = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n - 0.5
        r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
        spheres[n] = r2 < 0.45**2
    srv = Server(hbm_budget=int(budget_gb * (1 << 30)), max_slots=slots)
    client = torch.cuda.Stream()
    gen = torch.Generator(device="cuda")

    def make_request(q, arrival):
        n = q["n"]
        with torch.cuda.stream(client):
            # one allocation per request for its window, data and random fields (four sizes in all,
            # which the caching allocator reuses without fragmenting)
            buf = torch.empty((2 + n_mc, n, n, n), dtype=torch.float32, device="cuda")
            w, data = buf[0], buf[1]
            gen.manual_seed(q["window_seed"])
            torch.rand((n, n, n), generator=gen, device="cuda", out=data)
            torch.logical_and(spheres[n], data < 0.95, out=w)
            torch.mul(pool[n][q["field_seed"] % len(pool[n])], w, out=data)
            grfs = []
            for j in range(n_mc):
                gen.manual_seed(30000 + 8 * max(q["rid"], 0) + j)
                grfs.append(torch.randn((n, n, n), generator=gen, device="cuda", out=buf[2 + j]))
            ev = torch.cuda.Event()
            ev.record(client)
        return Request(rid=q["rid"], grid=n, box=box, edges=q["edges"], data=data, window=w,
                       precision=precision, arrival=arrival, ready=ev, grfs=grfs or None)

    # device-resident plans for every geometry of the stream, each run once
    # (kernels loaded, allocator segments cached) before the clock starts
    t_plans = time.perf_counter()
    seen = set()
    for q in sched:
        key = (q["n"], q["n_bins"])
        if key in seen:
            continue
        seen.add(key)
        srv.plan_for(q["n"], box, q["edges"])
        srv.submit(make_request(dict(q, rid=-1 - len(seen)), None))
        srv.run_until_idle()
    t_plans = time.perf_counter() - t_plans
    srv.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while k < len(sched) or not srv.idle:
        now = time.perf_counter() - t0
        while k < len(sched) and sched[k]["arrival"] <= now:
            srv.submit(make_request(sched[k], t0 + sched[k]["arrival"]))
            k += 1
        if srv.poll() == 0:
            time.sleep(5e-5)
    out = srv.summary()
    ms = torch.cuda.memory_stats()
    # allocator retries free the cached blocks and synchronize the device (a stall for every stream in flight)
    out["allocator"] = {"alloc_retries": int(ms.get("num_alloc_retries", 0)),
                        "device_allocs": int(ms.get("num_device_alloc", 0)),
                        "reserved_peak_gb": round(ms.get("reserved_bytes.all.peak", 0) / 2**30, 2)}
    slow = sorted((c for c in srv.done.values() if c.status == "ok"), key=lambda c: -c.latency)[:5]
    by_rid = {q["rid"]: q for q in sched}
    out["slowest"] = [dict(rid=c.rid, grid=by_rid[c.rid]["n"], bins=by_rid[c.rid]["n_bins"],
                           latency_ms=round(1e3 * c.latency, 3), service_ms=round(1e3 * c.service, 3),
                           wait_ms=round(1e3 * c.wait, 3)) for c in slow]
    out.update({
        "workload": f"Poisson stream, mean {rate:g} req/s, {n_requests} requests; grid uniform over "
                    "64^3/128^3/256^3/384^3, 10-40 bins of width 2k_f (<= 28 at 64^3), L=2000 Mpc/h; "
                    "data = window x field, window = sphere r<0.45L with 5% voxel holes; P+B per request, "
                    f"windowed normalisation, unwindowed P with a Monte Carlo Fisher matrix from {n_mc} random "
                    "fields per request",
        "precision": precision,
        "n_mc": n_mc,
        "budget_bytes": srv.budget,
        "slots": slots,
        "plan_build_and_warm_s": t_plans,
        "offered_rate_per_s": rate,
    })
    return out


def multipoles_bench(d32, box, edges, reps: int = 10) -> dict:
    """Power and bispectrum multipoles (l <= 2 and l <= 4, line of sight
    along z) at the headline workload: milliseconds per call and calls/s."""
    import torch

    import paper_2404_07249_amd as pb3

    x = torch.from_numpy(d32).cuda()
    n = d32.shape[0]
    out = {}
    for lmax in (2, 4):
        plan = pb3.Plan(n, box, edges, lmax=lmax)
        ws = torch.empty(int(plan._lib.pb3_multipoles_workspace_bytes(plan._h)), dtype=torch.uint8, device="cuda")
        plan.multipoles(x, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.multipoles(x, workspace=ws)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        out[f"lmax{lmax}"] = {"ms_per_call": round(ms, 3), "calls_per_s": round(1e3 / ms, 2),
                              "n_ell": plan.n_ell, "triplets": plan.n_triplets,
                              "workspace_gb": round(ws.numel() / 1e9, 2)}
    return out


def linear_term_bench(d32, box, edges, n_sim: int = 8, reps: int = 5) -> dict:
    """Bispectrum with the linear term over n_sim simulations (Gaussian
    fields through a survey-like window, data masked by the same window) at
    the headline workload, mixed precision: milliseconds per call."""
    import torch

    import paper_2404_07249_amd as pb3
    from synthetic import gaussian_field, window_mask

    n = d32.shape[0]
    w = window_mask(n, 20000)
    x = torch.from_numpy(d32 * w).cuda()
    sims = [torch.from_numpy((gaussian_field(n, box, 31000 + i) * w).astype(np.float32)).cuda()
            for i in range(n_sim)]
    plan = pb3.Plan(n, box, edges)
    ws = torch.empty(plan.linear_workspace_bytes(n_sim), dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.n_triplets, dtype=torch.float64, device="cuda")
    plan.bispectrum_linear(x, sims, "mixed", out=out, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.bispectrum_linear(x, sims, "mixed", out=out, workspace=ws)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    return {"n_sim": n_sim, "ms_per_call": round(ms, 3), "bispectra_per_call": 2 * n_sim + 1,
            "workspace_gb": round(ws.numel() / 1e9, 2)}


def noncubic_bench(reps: int = 10) -> dict:
    """Non-cubic geometry: power multipoles l = 0, 2, 4 in 44 bins (132
    bandpowers) on a survey-like 192 x 384 x 192 grid whose cells give
    k_Ny ~ 0.6 h/Mpc on every axis, and P + B (mixed precision) on a
    128 x 192 x 96 grid of a 1000 x 1500 x 750 Mpc/h box with 20 bins."""
    import torch

    import paper_2404_07249_amd as pb3
    from synthetic import quadratic_field3

    out = {}
    shape, box = (192, 384, 192), (1005.3, 2010.6, 1005.3)
    edges = 0.01 + 0.0125 * np.arange(45)
    x = torch.from_numpy(quadratic_field3(shape, box, 1.0, 3).astype(np.float32)).cuda()
    plan = pb3.Plan(shape, box, edges, edges_hmpc=True, power_only=True, lmax=4)
    ws = torch.empty(int(plan._lib.pb3_multipoles_workspace_bytes(plan._h)), dtype=torch.uint8, device="cuda")
    plan.multipoles(x, bispectrum=False, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.multipoles(x, bispectrum=False, workspace=ws)
    torch.cuda.synchronize()
    out["power_multipoles"] = {"grid": list(shape), "box": list(box), "bins": plan.n_bins, "n_ell": 3,
                               "ms_per_call": round(1e3 * (time.perf_counter() - t0) / reps, 3)}
    shape, box = (128, 192, 96), (1000.0, 1500.0, 750.0)
    edges = 0.01 + 0.01 * np.arange(21)
    x = torch.from_numpy(quadratic_field3(shape, box, 1.0, 4).astype(np.float32)).cuda()
    plan = pb3.Plan(shape, box, edges, edges_hmpc=True)
    plan.polyspectra(x, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.polyspectra(x, "mixed")
    torch.cuda.synchronize()
    m = plan.contract_grid
    out["polyspectra"] = {"grid": list(shape), "box": list(box), "bins": plan.n_bins, "triplets": plan.n_triplets,
                          "contract_grid": list(m) if isinstance(m, tuple) else [m] * 3,
                          "ms_per_call": round(1e3 * (time.perf_counter() - t0) / reps, 3)}
    return out


def p_launches(plan) -> int:
    """Kernel launches of one single P+B call (a one-job batch)."""
    import paper_2404_07249_amd as pb3

    return pb3.Batch([plan], ext_workspace=True).launches()


def plan_geometry(n, box, edges):
    """Host-side geometry the stage model needs (same rules as the library)."""
    import paper_2404_07249_amd as pb3

    hp = pb3.Plan(n, box, edges, host_only=True)
    m = hp.contract_grid
    e = np.asarray(edges, dtype=np.float64)
    thr = np.ceil(e * e).astype(np.int64)
    k = int(np.floor(np.sqrt(max(thr[-1] - 1, 0))))
    k = min(k, n // 2)
    full = k >= n // 2
    kz = n // 2 + 1 if full else k + 1
    lc = n if full else 2 * k + 1
    geom = []
    for b in range(len(e) - 1):
        kb = min(int(np.floor(np.sqrt(max(thr[b + 1] - 1, 0)))), n // 2)
        kpos = n // 2 - 1 if (full and kb == n // 2) else kb
        geom.append((kb + kpos + 1, kb + 1))
    _, _, nm = hp.bins()
    return dict(N=n, M=m, Kz=kz, Lc=lc, nb=len(e) - 1, geom=geom, n_modes_half=int((nm.sum() + 1) // 2),
                n_trip=hp.n_triplets)


def copy_calibration() -> int:
    """A plain device copy of exactly 256 MiB in and 256 MiB out, three
    times: rocprofv3's FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of this
    copy calibrate the traffic counters of the kernels."""
    import torch

    n = 256 * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "copies": 3}), flush=True)
    return 0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d32: np.ndarray, box: float, edges) -> dict:
    """The FP64 oracle on the host cores for one whole field of the workload:
    forward FFT, P(k), every filtered field and the triplet sums of every
    triangle-valid triplet (the per-field estimator; the data-independent
    triangle counts are plan-time work and not timed)."""
    import oracle

    threads = min(_cores(), int(os.environ.get("OMP_NUM_THREADS", _cores())))
    os.environ["ORACLE_FFT_WORKERS"] = str(threads)
    d = d32.astype(np.float64)
    trips = oracle.triangle_triplets(edges)
    t0 = time.perf_counter()
    oracle.power_spectrum(d, box, edges)
    G = oracle.filtered_fields(d, edges)
    t_fft = time.perf_counter() - t0
    oracle.triple_sums(G, trips)
    per = time.perf_counter() - t0
    return {
        "value": 1.0 / per,
        "unit": "bispectra/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (
            f"one whole 256^3 field: FP64 forward FFT, P(k), all {len(edges) - 1} filtered fields ({t_fft:.2f} s) "
            f"and the sums of all {len(trips)} triplets ({per - t_fft:.2f} s); {threads} threads "
            "(FFT workers and the triplet-sum thread pool)"
        ),
        "seconds": per,
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["mixed", "fp32"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=50)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes instead of timed ones")
    ap.add_argument("--no-multipoles", action="store_true", help="skip the multipole measurement")
    ap.add_argument("--no-linear", action="store_true", help="skip the linear-term measurement")
    ap.add_argument("--no-noncubic", action="store_true", help="skip the non-cubic geometry measurement")
    ap.add_argument("--serve-mc", type=int, default=8, help="random fields per serving request (0: windowed only)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (calibrates the traffic counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched-workload measurement (default launch shapes) and print its JSON")
    ap.add_argument("--masked-only", action="store_true",
                    help="only time the masked power spectrum with 8 Monte Carlo fields and print its JSON")
    args = ap.parse_args(argv)
    if args.copy_calibration:
        return copy_calibration()
    if args.batched_only:
        r = batched_bench(reps=5, warmup=2, precision=args.precision, autotune=False)
        print(json.dumps({"batched": r}), flush=True)
        return 0
    if args.masked_only:
        print(json.dumps({"masked_power": masked_bench()}), flush=True)
        return 0
    if args.gpus != 1:
        print(
            json.dumps({"error": "the library runs on one GPU; --gpus above 1 is not supported", "n_gpus": args.gpus}),
            flush=True,
        )
        return 2

    import torch

    import paper_2404_07249_amd as pb3
    from synthetic import field_for

    d32, cfg = field_for("c3")
    n, box, edges = cfg["n"], cfg["box"], cfg["edges"]
    # the timed plan records no events; a twin with stage timing gives the
    # per-kernel breakdown in a separate pass
    plan = pb3.Plan(n, box, edges, autotune=not args.no_autotune)
    tplan = pb3.Plan(n, box, edges, stage_timing=True, autotune=not args.no_autotune)
    info = plan_geometry(n, box, edges)
    info["n_trip"] = plan.n_triplets
    x = torch.from_numpy(d32).cuda()
    pk = torch.empty(plan.n_bins, dtype=torch.float64, device="cuda")
    bk = torch.empty(plan.n_triplets, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    graph = pb3.Batch([plan], graph=True)  # the same launch sequence, replayed from a HIP graph

    def step(prec):
        plan.polyspectra(x, precision=prec, pk_out=pk, bk_out=bk, stream=stream)

    def gstep(prec):
        graph.run([x], prec, pk_outs=[pk], bk_outs=[bk], stream=stream)

    def timed(fn, prec, steps):
        for _ in range(args.warmup):
            fn(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(prec)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    results = {}
    for prec in (["fp32", "mixed"] if args.precision == "mixed" else ["mixed", "fp32"]):
        dt_eager = timed(step, prec, args.steps)
        dt = timed(gstep, prec, args.steps)
        for _ in range(args.warmup):
            tplan.polyspectra(x, precision=prec, pk_out=pk, bk_out=bk, stream=stream)
        torch.cuda.synchronize()
        tplan.reset_stage_times()
        for _ in range(args.steps):
            tplan.polyspectra(x, precision=prec, pk_out=pk, bk_out=bk, stream=stream)
        torch.cuda.synchronize()
        stages = tplan.stage_times()
        # per-call latency (each call synchronised), after the timed region
        lat = []
        for _ in range(args.latency_calls):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            gstep(prec)
            b.record(stream)
            b.synchronize()
            lat.append(a.elapsed_time(b))
        results[prec] = dict(dt=dt, dt_eager=dt_eager, stages=stages, lat=np.array(lat))
    main_p = args.precision
    r = results[main_p]
    value = args.steps / r["dt_eager"]
    work = stage_work(info, main_p)
    dom = max(r["stages"], key=lambda k: r["stages"][k][0])
    kind, amount = work[dom]
    ms = r["stages"][dom][0]
    if kind == "flops":
        peak = BF16_PEAK_TFLOPS if main_p == "mixed" else FP32_MFMA_PEAK_TFLOPS
        achieved = amount / (ms * 1e-3) / 1e12
        dense = dense_gemm_flops(info) / (ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(dom, main_p, plan.launch_shape["contract_wgs"]),
                "work": "(pairs a<=b + 2 x triplets) x M^3 flops per launch (eq. beta-def)",
                "dense_equivalent": {"TFLOP/s": dense, "frac": dense / peak,
                                     "work": "2 x pairs x bins x M^3 (every pair against every bin)"}}
    else:
        achieved = amount / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(dom, main_p, plan.launch_shape["contract_wgs"])}
    roof["kernel"] = dom
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "bispectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["dt_eager"] / args.steps,
        "graph_value": args.steps / r["dt"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if main_p == "mixed" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 grid, L=2000 Mpc/h, 30 bins of width 2k_f from k_f, 3035 triplets, "
            "quadratic field f_NL=1; P(k)+B(k1,k2,k3) per step",
            "grid": n,
            "contract_grid": plan.contract_grid,
            "bins": plan.n_bins,
            "triplets": plan.n_triplets,
            "precision": main_p,
            "launch_shape": plan.launch_shape,
            "launch": "one pb3_polyspectra call per step (graph_value: the same launch sequence replayed "
                      "from a HIP graph)",
        },
        "latency_ms": {"p50": float(np.percentile(r["lat"], 50)), "p99": float(np.percentile(r["lat"], 99))},
        "other_precision": {
            p: {"value": args.steps / results[p]["dt_eager"],
                "latency_ms": {"p50": float(np.percentile(results[p]["lat"], 50)),
                               "p99": float(np.percentile(results[p]["lat"], 99))}}
            for p in results if p != main_p
        },
        "stages_ms": {k: round(v[0], 5) for k, v in r["stages"].items()},
        "stage_rates": stage_rates(work, r["stages"], main_p),
        "roofline": roof,
    }
    if not args.no_batched:
        line["batched"] = batched_bench(precision=main_p, autotune=not args.no_autotune)
    if not args.no_multipoles:
        line["multipoles"] = multipoles_bench(d32, box, edges)
    if not args.no_linear:
        line["linear_term"] = linear_term_bench(d32, box, edges)
    if not args.no_noncubic:
        line["noncubic"] = noncubic_bench()
    if args.serve_requests > 0:
        line["serving"] = serving_bench(args.serve_requests, precision=main_p, n_mc=args.serve_mc)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(d32, box, edges)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
