"""The allocation-free power spectrum (pb3_power_noalloc) against pb3_power.

Through the C ABI (the binding's power_noalloc marshals arguments only):
two calls in a row, the headline 256^3 x 30-bin plan and then a smaller
64^3 plan, each bit-identical to pb3_power of an ordinary plan (same
kernels and summation order, different scratch memory); neither call makes
torch allocate; a plan whose workspace exceeds the static array is refused.
"""

import ctypes as C
import sys

import numpy as np
import pytest

from synthetic import field_for, kf_edges, quadratic_field

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


def test_power_noalloc_equals_power_twice(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    d3, c3 = field_for("c3")
    d_small = quadratic_field(64, 1000.0, 1.0, 6401).astype(np.float32)
    cases = [(c3["n"], c3["box"], c3["edges"], d3), (64, 1000.0, kf_edges(12), d_small)]
    for n, box, edges, d in cases:
        _say(f"[case] power_noalloc n={n} bins={len(edges) - 1}")
        ref_plan = pb3.Plan(n, box, edges, power_only=True)
        na_plan = pb3.Plan(n, box, edges, power_only=True, ext_workspace=True)  # no plan workspace at all
        x = torch.from_numpy(d).cuda()
        ref = ref_plan.power(x)
        out = torch.full((na_plan.n_bins,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        na_plan.power_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(out, ref), (n, (out - ref).abs().max().item())


def test_power_noalloc_refuses_a_plan_beyond_the_array(torch_cuda):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    _say("[case] power_noalloc 384^3 x 40 bins (refused)")
    plan = pb3.Plan(384, 2000.0, kf_edges(40), power_only=True, ext_workspace=True)
    x = torch.zeros((384, 384, 384), dtype=torch.float32, device="cuda")
    out = torch.empty(plan.n_bins, dtype=torch.float64, device="cuda")
    st = plan._lib.pb3_power_noalloc(plan._h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 4  # PB3_EUNSUPPORTED, before any launch
    assert b"bytes" in plan._lib.pb3_last_error()
