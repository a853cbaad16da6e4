"""MI355X-native idealized binned power spectrum and bispectrum.

Python binding over the C ABI of ``libpb3.so`` (include/pb3.h).  It only
marshals arguments: every step of the estimator runs in the HIP kernels.
PyTorch supplies device memory and streams.

    import paper_2404_07249_amd as pb3
    plan = pb3.Plan(256, 2000.0, edges_kf)          # bins in units of k_f
    pk, bk = plan.polyspectra(delta_cuda_f32, precision="mixed")
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import Pb3Error  # noqa: F401

__all__ = ["Plan", "Pb3Error", "load_library"]

_PREC = {"fp32": _lib.PREC_FP32, "mixed": _lib.PREC_MIXED_BF16X3, "bf16x3": _lib.PREC_MIXED_BF16X3}


def load_library():
    """Load libpb3.so (ImportError if it has not been built)."""
    return _lib.load()


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """Plan for one grid / box / binning (``pb3_plan``).

    grid: grid points per side N; box: side L in Mpc/h; edges: bin edges
    in units of k_f (or h/Mpc with ``edges_hmpc=True``).
    """

    def __init__(
        self,
        grid: int,
        box: float,
        edges,
        *,
        edges_hmpc: bool = False,
        host_only: bool = False,
        full_grid: bool = False,
        strict: bool = False,
        stage_timing: bool = False,
        ext_workspace: bool = False,
        fuse: bool = True,
    ):
        lib = _lib.load()
        self._lib = lib
        self._h = None
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        g = (C.c_int * 3)(grid, grid, grid)
        b = (C.c_double * 3)(box, box, box)
        flags = 0
        flags |= _lib.FLAG_EDGES_HMPC if edges_hmpc else 0
        flags |= _lib.FLAG_HOST_ONLY if host_only else 0
        flags |= _lib.FLAG_FULL_GRID if full_grid else 0
        flags |= _lib.FLAG_STRICT if strict else 0
        flags |= _lib.FLAG_STAGE_TIMING if stage_timing else 0
        flags |= _lib.FLAG_EXT_WORKSPACE if ext_workspace else 0
        flags |= 0 if fuse else _lib.FLAG_NO_FUSION
        h = C.c_void_p()
        _lib.check(
            lib.pb3_plan_create(g, b, e.ctypes.data_as(C.POINTER(C.c_double)), int(e.size), flags, C.byref(h))
        )
        self._h = h
        self.grid = int(grid)
        self.box = float(box)
        self._workspace = None

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pb3_plan_destroy(self._h)
            self._h = None

    def close(self):
        self.__del__()

    # ---------------------------------------------------------------- info
    @property
    def n_bins(self) -> int:
        return int(self._lib.pb3_n_bins(self._h))

    @property
    def n_triplets(self) -> int:
        return int(self._lib.pb3_n_triplets(self._h))

    @property
    def contract_grid(self) -> int:
        return int(self._lib.pb3_contract_grid(self._h))

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.pb3_plan_workspace_bytes(self._h))

    def bins(self):
        """(edges in k_f units, mean |k| per bin in h/Mpc, mode counts N_b)."""
        nb = self.n_bins
        edges = np.zeros(nb + 1)
        kmean = np.zeros(nb)
        nm = np.zeros(nb, dtype=np.int64)
        _lib.check(self._lib.pb3_get_bins(self._h, edges.ctypes.data, kmean.ctypes.data, nm.ctypes.data))
        return edges, kmean, nm

    @property
    def triplets(self) -> np.ndarray:
        t = np.zeros((self.n_triplets, 3), dtype=np.int32)
        if t.size:
            _lib.check(self._lib.pb3_get_triplets(self._h, t.ctypes.data))
        return t

    def norm(self):
        """(N_b per bin, T_abc per triplet) from the plan's FP64 count pass."""
        nm = np.zeros(self.n_bins, dtype=np.int64)
        cnt = np.zeros(self.n_triplets, dtype=np.float64)
        _lib.check(self._lib.pb3_norm(self._h, nm.ctypes.data, cnt.ctypes.data))
        return nm, cnt

    def bind_workspace(self, tensor):
        """Use a caller-owned CUDA tensor (>= workspace_bytes) as workspace."""
        nbytes = tensor.numel() * tensor.element_size()
        _lib.check(self._lib.pb3_plan_bind_workspace(self._h, C.c_void_p(tensor.data_ptr()), nbytes))
        self._workspace = tensor

    # ------------------------------------------------------------- compute
    def _check_field(self, delta):
        import torch

        n = self.grid
        if not isinstance(delta, torch.Tensor) or delta.device.type != "cuda":
            raise TypeError("delta must be a CUDA tensor")
        if delta.dtype != torch.float32 or tuple(delta.shape) != (n, n, n) or not delta.is_contiguous():
            raise ValueError(f"delta must be a contiguous float32 tensor of shape ({n}, {n}, {n})")

    def _out(self, out, count, like):
        import torch

        if out is None:
            return torch.empty(count, dtype=torch.float64, device=like.device)
        if out.dtype != torch.float64 or out.numel() < count or not out.is_contiguous() or out.device != like.device:
            raise ValueError("out must be a contiguous float64 tensor on the field's device")
        return out

    def power(self, delta, out=None, stream=None):
        self._check_field(delta)
        pk = self._out(out, self.n_bins, delta)
        _lib.check(
            self._lib.pb3_power(self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr()), _stream_handle(stream))
        )
        return pk

    def bispectrum(self, delta, precision: str = "fp32", out=None, stream=None):
        self._check_field(delta)
        bk = self._out(out, self.n_triplets, delta)
        _lib.check(
            self._lib.pb3_bispectrum(
                self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(bk.data_ptr()), _PREC[precision],
                _stream_handle(stream),
            )
        )
        return bk

    def polyspectra(self, delta, precision: str = "fp32", pk_out=None, bk_out=None, stream=None):
        self._check_field(delta)
        pk = self._out(pk_out, self.n_bins, delta)
        bk = self._out(bk_out, self.n_triplets, delta)
        _lib.check(
            self._lib.pb3_polyspectra(
                self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr()), C.c_void_p(bk.data_ptr()),
                _PREC[precision], _stream_handle(stream),
            )
        )
        return pk, bk

    def stage_times(self) -> dict:
        """Mean milliseconds per kernel stage over the calls since the last
        reset (plans made with ``stage_timing=True``): {stage: (ms, calls)}."""
        buf = (C.c_float * 16)()
        cnt = (C.c_int * 16)()
        n = C.c_int(0)
        _lib.check(self._lib.pb3_stage_times(self._h, buf, cnt, 16, C.byref(n)))
        return {self._lib.pb3_stage_name(i).decode(): (float(buf[i]), int(cnt[i])) for i in range(n.value)}

    def reset_stage_times(self):
        _lib.check(self._lib.pb3_stage_timing_reset(self._h))
