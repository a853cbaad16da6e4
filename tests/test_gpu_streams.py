"""Stream safety of the binding's own allocations and the C ABI's pointer
checks.

When a call runs on a stream other than torch's current one and the
binding allocates the outputs or a temporary workspace itself, the caching
allocator must not hand that memory to an allocation on the current stream
while the call's kernels may still use it: each result must equal, bit for
bit, the same call on the current stream even when the current stream
immediately allocates and overwrites memory of the same sizes.
"""

import ctypes as C
import sys

import numpy as np
import pytest

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


def _churn(torch, sizes, rounds=6):
    """Allocate and overwrite blocks of the given byte sizes on the current
    stream (the memory a side-stream call may have just released)."""
    keep = []
    for _ in range(rounds):
        for nb in sizes:
            t = torch.empty(max(int(nb), 1), dtype=torch.uint8, device="cuda")
            t.fill_(0xA5)
            keep.append(t)
    return keep


def test_side_stream_calls_without_workspace(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 32, 800.0, kf_edges(6)
    _say("[case] side-stream temporaries: masked power, linear term, multipoles")
    w = window_mask(n, 123)
    data = _gpu(torch, quadratic_field(n, box, 1.0, 11) * w)
    win = _gpu(torch, w)
    grfs = [_gpu(torch, np.random.default_rng(40 + i).standard_normal((n, n, n))) for i in range(2)]
    sims = [_gpu(torch, gaussian_field(n, box, 60 + i) * w) for i in range(2)]
    pm = pb3.Plan(n, box, edges, full_grid=True)
    pl = pb3.Plan(n, box, edges)
    pml = pb3.Plan(n, box, edges, lmax=2)
    calls = {
        "masked": (lambda st: pm.masked_power(data, win, grfs, stream=st), pm.masked_workspace_bytes),
        "linear": (lambda st: (pl.bispectrum_linear(data, sims, stream=st),), pl.linear_workspace_bytes(2)),
        "multipoles": (lambda st: pml.multipoles(data, stream=st),
                       int(pml._lib.pb3_multipoles_workspace_bytes(pml._h))),
    }
    for name, (fn, ws_bytes) in calls.items():
        ref = [t.clone() for t in fn(None)]
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        for rep in range(3):
            out = fn(side)
            junk = _churn(torch, [ws_bytes, 8 * pm.n_bins, 8 * pl.n_triplets, 8 * pm.n_bins ** 2])
            side.synchronize()
            torch.cuda.synchronize()
            for a, b in zip(out, ref):
                assert torch.equal(a, b), (name, rep)
            del junk


def test_misaligned_fields_are_refused(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n = 32
    plan = pb3.Plan(n, 800.0, kf_edges(6))
    buf = torch.zeros(n ** 3 + 1, dtype=torch.float32, device="cuda")
    shifted = buf[1:].view(n, n, n)  # 4-byte offset
    with pytest.raises(ValueError):
        plan.power(shifted)
    pk = torch.empty(plan.n_bins, dtype=torch.float64, device="cuda")
    st = plan._lib.pb3_power(plan._h, C.c_void_p(shifted.data_ptr()), C.c_void_p(pk.data_ptr()),
                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 1  # PB3_EINVAL, refused on the host before any launch
    assert b"aligned" in plan._lib.pb3_last_error()
