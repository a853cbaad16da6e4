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

__all__ = ["Plan", "Batch", "Pb3Error", "load_library"]

_PREC = {"fp32": _lib.PREC_FP32, "mixed": _lib.PREC_MIXED_BF16X3, "bf16x3": _lib.PREC_MIXED_BF16X3}


def load_library():
    """Load libpb3.so (ImportError if it has not been built)."""
    return _lib.load()


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _on_stream(tensor, stream):
    """Mark a tensor this module allocated (an output or a temporary
    workspace) as used by ``stream``: torch's caching allocator then does not
    hand its memory to another allocation until the work queued on that
    stream so far has finished, even when it was allocated on another one."""
    import torch

    if stream is not None and tensor is not None and stream != torch.cuda.current_stream(tensor.device):
        tensor.record_stream(stream)
    return tensor


class Plan:
    """Plan for one grid / box / binning (``pb3_plan``).

    grid: grid points per side N; box: side L in Mpc/h; edges: bin edges
    in units of k_f (or h/Mpc with ``edges_hmpc=True``).
    """

    def __init__(
        self,
        grid,
        box,
        edges,
        *,
        edges_hmpc: bool = False,
        host_only: bool = False,
        full_grid: bool = False,
        strict: bool = False,
        stage_timing: bool = False,
        ext_workspace: bool = False,
        fuse: bool = True,
        autotune: bool = False,
        power_only: bool = False,
        lmax: int = 0,
        bk_fisher: bool = False,
    ):
        lib = _lib.load()
        self._lib = lib
        self._h = None
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        g3 = tuple(int(v) for v in np.broadcast_to(np.asarray(grid), (3,)))
        b3 = tuple(float(v) for v in np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
        g = (C.c_int * 3)(*g3)
        b = (C.c_double * 3)(*b3)
        flags = 0
        flags |= _lib.FLAG_EDGES_HMPC if edges_hmpc else 0
        flags |= _lib.FLAG_HOST_ONLY if host_only else 0
        flags |= _lib.FLAG_FULL_GRID if full_grid else 0
        flags |= _lib.FLAG_STRICT if strict else 0
        flags |= _lib.FLAG_STAGE_TIMING if stage_timing else 0
        flags |= _lib.FLAG_EXT_WORKSPACE if ext_workspace else 0
        flags |= 0 if fuse else _lib.FLAG_NO_FUSION
        flags |= _lib.FLAG_AUTOTUNE if autotune else 0
        flags |= _lib.FLAG_POWER_ONLY if power_only else 0
        if lmax not in (0, 2, 4):
            raise ValueError("lmax must be 0, 2 or 4")
        flags |= {0: 0, 2: _lib.FLAG_LMAX2, 4: _lib.FLAG_LMAX4}[lmax]
        flags |= _lib.FLAG_BK_FISHER if bk_fisher else 0
        h = C.c_void_p()
        _lib.check(
            lib.pb3_plan_create(g, b, e.ctypes.data_as(C.POINTER(C.c_double)), int(e.size), flags, C.byref(h))
        )
        self._h = h
        self.shape = g3  # (Nx, Ny, Nz)
        self.boxes = b3  # (Lx, Ly, Lz)
        # a cubic geometry keeps the scalar forms
        self.grid = g3[0] if g3[0] == g3[1] == g3[2] else g3
        self.box = b3[0] if b3[0] == b3[1] == b3[2] else b3
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
    def contract_grid(self):
        """M (cubic contraction grid) or (Mx, My, Mz)."""
        m = (C.c_int * 3)()
        _lib.check(self._lib.pb3_grid3(self._h, None, m))
        m3 = (int(m[0]), int(m[1]), int(m[2]))
        return m3[0] if m3[0] == m3[1] == m3[2] else m3

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.pb3_plan_workspace_bytes(self._h))

    @property
    def launch_shape(self) -> dict:
        """{"fused": bool, "contract_wgs": int, "tuned": "default"|"cache"|"timed"}."""
        f, w, t = C.c_int(), C.c_int(), C.c_int()
        _lib.check(self._lib.pb3_plan_launch_shape(self._h, C.byref(f), C.byref(w), C.byref(t)))
        return {"fused": bool(f.value), "contract_wgs": int(w.value),
                "tuned": {0: "default", 1: "cache", 2: "timed"}[t.value]}

    def bins(self):
        """(edges in k_f units (a box with equal sides) or h/Mpc, mean |k| per
        bin in h/Mpc, mode counts N_b)."""
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

        shape = self.shape
        if not isinstance(delta, torch.Tensor) or delta.device.type != "cuda":
            raise TypeError("delta must be a CUDA tensor")
        if delta.dtype != torch.float32 or tuple(delta.shape) != shape or not delta.is_contiguous():
            raise ValueError(f"delta must be a contiguous float32 tensor of shape {shape}")
        if delta.data_ptr() % 8 != 0:  # the forward pass reads pairs of values
            raise ValueError("delta must start at an 8-byte aligned address")

    def _out(self, out, count, like, stream=None):
        import torch

        if out is None:
            return _on_stream(torch.empty(count, dtype=torch.float64, device=like.device), stream)
        if out.dtype != torch.float64 or out.numel() < count or not out.is_contiguous() or out.device != like.device:
            raise ValueError("out must be a contiguous float64 tensor on the field's device")
        return out

    def power(self, delta, out=None, stream=None):
        self._check_field(delta)
        pk = self._out(out, self.n_bins, delta, stream)
        _lib.check(
            self._lib.pb3_power(self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr()), _stream_handle(stream))
        )
        return pk

    def power_noalloc(self, delta, out, stream=None):
        """``pb3_power_noalloc``: P into the caller's ``out`` (n_bins float64)
        with the library's static scratch; allocates nothing."""
        self._check_field(delta)
        if out is None:
            raise ValueError("power_noalloc needs an output tensor (it allocates nothing)")
        pk = self._out(out, self.n_bins, delta)
        _lib.check(self._lib.pb3_power_noalloc(self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr()),
                                               _stream_handle(stream)))
        return pk

    def bispectrum(self, delta, precision: str = "fp32", out=None, stream=None):
        self._check_field(delta)
        bk = self._out(out, self.n_triplets, delta, stream)
        _lib.check(
            self._lib.pb3_bispectrum(
                self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(bk.data_ptr()), _PREC[precision],
                _stream_handle(stream),
            )
        )
        return bk

    def polyspectra(self, delta, precision: str = "fp32", pk_out=None, bk_out=None, stream=None):
        self._check_field(delta)
        pk = self._out(pk_out, self.n_bins, delta, stream)
        bk = self._out(bk_out, self.n_triplets, delta, stream)
        _lib.check(
            self._lib.pb3_polyspectra(
                self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr()), C.c_void_p(bk.data_ptr()),
                _PREC[precision], _stream_handle(stream),
            )
        )
        return pk, bk

    def window_normalize(self, window, pk=None, bk=None, scratch=None, stream=None):
        """Divide P by <w^2> and B by <w^3> in place (masked data d = w delta);
        returns (<w^2>, <w^3>) as a float64 CUDA tensor of two entries."""
        import torch

        self._check_field(window)
        if pk is None and bk is None:
            raise ValueError("nothing to normalise")
        if scratch is None:
            scratch = _on_stream(torch.empty(_lib.WINDOW_SCRATCH, dtype=torch.float64, device=window.device), stream)
        elif scratch.dtype != torch.float64 or scratch.numel() < _lib.WINDOW_SCRATCH:
            raise ValueError("scratch must hold PB3_WINDOW_SCRATCH float64 values")
        _lib.check(self._lib.pb3_window_normalize(
            self._h, C.c_void_p(window.data_ptr()), C.c_void_p(pk.data_ptr() if pk is not None else 0),
            C.c_void_p(bk.data_ptr() if bk is not None else 0), C.c_void_p(scratch.data_ptr()),
            _stream_handle(stream)))
        return scratch[:2]

    @property
    def masked_workspace_bytes(self) -> int:
        return int(self._lib.pb3_masked_power_workspace_bytes(self._h))

    def masked_power(self, data, window, grfs, pk_out=None, fisher_out=None, workspace=None, stream=None):
        """Unwindowed P of masked data d = w delta with the Monte Carlo Fisher
        matrix from the white unit-variance fields ``grfs`` (plans made with
        ``full_grid=True``).  Returns (P, F)."""
        import torch

        self._check_field(data)
        self._check_field(window)
        for g in grfs:
            self._check_field(g)
        pk = self._out(pk_out, self.n_bins, data, stream)
        nb = self.n_bins
        fm = fisher_out if fisher_out is not None else _on_stream(
            torch.empty((nb, nb), dtype=torch.float64, device=data.device), stream)
        if workspace is None:
            workspace = _on_stream(torch.empty(self.masked_workspace_bytes, dtype=torch.uint8, device=data.device),
                                   stream)
        ga = (C.c_void_p * len(grfs))(*[g.data_ptr() for g in grfs])
        _lib.check(self._lib.pb3_masked_power(
            self._h, C.c_void_p(data.data_ptr()), C.c_void_p(window.data_ptr()), ga, len(grfs),
            C.c_void_p(pk.data_ptr()), C.c_void_p(fm.data_ptr()), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_handle(stream)))
        return pk, fm

    def linear_workspace_bytes(self, n_sim: int) -> int:
        return int(self._lib.pb3_bispectrum_linear_workspace_bytes(self._h, int(n_sim)))

    def bispectrum_linear(self, data, sims, precision: str = "mixed", out=None, workspace=None, stream=None):
        """B with the bispectrum numerator's linear term averaged over the
        fields ``sims`` (about the data's covariance, e.g. simulations through
        the same window); units of :meth:`bispectrum`."""
        import torch

        self._check_field(data)
        for g in sims:
            self._check_field(g)
        bk = self._out(out, self.n_triplets, data, stream)
        if workspace is None:
            workspace = _on_stream(
                torch.empty(self.linear_workspace_bytes(len(sims)), dtype=torch.uint8, device=data.device), stream)
        sa = (C.c_void_p * len(sims))(*[g.data_ptr() for g in sims])
        _lib.check(self._lib.pb3_bispectrum_linear(
            self._h, C.c_void_p(data.data_ptr()), sa, len(sims), C.c_void_p(bk.data_ptr()), _PREC[precision],
            C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(), _stream_handle(stream)))
        return bk

    @property
    def weights_table_len(self) -> int:
        """Entries the P_fid table of :meth:`set_weights` needs (|n|^2 = 0 .. len-1)."""
        return int(self._lib.pb3_weights_table_len(self._h))

    def set_weights(self, window_order: int = 0, pfid=None, nbar: float = 0.0):
        """Weighted ideal estimators: pixel-window deconvolution of the given
        order (0 none, 1 NGP, 2 CIC, 3 TSC), P_fid weights (array over integer
        |n|^2, or a callable of k in h/Mpc), Poisson shot noise for nbar > 0."""
        tab = None
        if pfid is not None and not isinstance(self.box, tuple):  # unequal box sides: the library refuses
            n = self.weights_table_len
            if callable(pfid):
                kf = 2 * np.pi / self.box
                tab = np.asarray(pfid(kf * np.sqrt(np.arange(n, dtype=np.float64))), dtype=np.float64)
                tab[0] = 1.0
            else:
                tab = np.ascontiguousarray(np.asarray(pfid, dtype=np.float64))
        ptr = tab.ctypes.data if tab is not None else None
        _lib.check(self._lib.pb3_plan_set_weights(self._h, int(window_order), ptr,
                                                  0 if tab is None else int(tab.size), float(nbar)))

    @property
    def n_ell(self) -> int:
        return int(self._lib.pb3_n_ell(self._h))

    def multipole_mixing(self) -> np.ndarray:
        """Per-triplet blocks R [n_trip, n_ell, n_ell] that map the eq.
        (ideal-bk) multipoles to the Fisher-normalised ones (plans made with
        ``bk_fisher=True``)."""
        ne, nt = self.n_ell, self.n_triplets
        out = np.zeros((nt, ne, ne), dtype=np.float64)
        _lib.check(self._lib.pb3_multipole_mixing(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def multipoles(self, delta, power: bool = True, bispectrum: bool = True, precision: str = "mixed",
                   workspace=None, stream=None):
        """(P_l [n_ell, n_bins] or None, B_l [n_ell, n_trip] or None) for
        l = 0, 2, (4) with the line of sight along z (plans made with lmax > 0)."""
        import torch

        self._check_field(delta)
        ne = self.n_ell
        pk = torch.empty((ne, self.n_bins), dtype=torch.float64, device=delta.device) if power else None
        bk = torch.empty((ne, self.n_triplets), dtype=torch.float64, device=delta.device) if bispectrum else None
        _on_stream(pk, stream)
        _on_stream(bk, stream)
        if workspace is None:
            nbytes = int(self._lib.pb3_multipoles_workspace_bytes(self._h))
            workspace = _on_stream(torch.empty(max(nbytes, 1), dtype=torch.uint8, device=delta.device), stream)
        _lib.check(self._lib.pb3_multipoles(
            self._h, C.c_void_p(delta.data_ptr()), C.c_void_p(pk.data_ptr() if pk is not None else 0),
            C.c_void_p(bk.data_ptr() if bk is not None else 0), _PREC[precision], C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_handle(stream)))
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


def _ptr_array(values):
    arr = (C.c_void_p * len(values))()
    for i, v in enumerate(values):
        arr[i] = v
    return arr


class Batch:
    """Many fields through one or more plans in shared launches
    (``pb3_batch``).  Jobs that use the same ``Plan`` object run in the same
    kernel launches (up to 8 per launch); different plans run concurrently
    on internal streams.  ``graph=True`` captures the run into a HIP graph
    and replays it while the arguments stay the same.  The plans must stay
    alive as long as the batch.
    """

    def __init__(self, plans, *, graph: bool = False, ext_workspace: bool = False):
        lib = _lib.load()
        self._lib = lib
        self._h = None
        self.plans = list(plans)
        arr = _ptr_array([p._h.value for p in self.plans])
        flags = (_lib.BATCH_GRAPH if graph else 0) | (_lib.BATCH_EXT_WORKSPACE if ext_workspace else 0)
        h = C.c_void_p()
        _lib.check(lib.pb3_batch_create(arr, len(self.plans), flags, C.byref(h)))
        self._h = h
        self._workspace = None

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pb3_batch_destroy(self._h)
            self._h = None

    def close(self):
        self.__del__()

    @property
    def n_jobs(self) -> int:
        return len(self.plans)

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.pb3_batch_workspace_bytes(self._h))

    def launches(self, power: bool = True, bispectrum: bool = True) -> int:
        return int(self._lib.pb3_batch_launches(self._h, int(power), int(bispectrum)))

    @property
    def groups(self) -> int:
        return int(self._lib.pb3_batch_groups(self._h))

    def bind_workspace(self, tensor):
        nbytes = tensor.numel() * tensor.element_size()
        _lib.check(self._lib.pb3_batch_bind_workspace(self._h, C.c_void_p(tensor.data_ptr()), nbytes))
        self._workspace = tensor

    def run(self, deltas, precision: str = "mixed", pk_outs=None, bk_outs=None, power: bool = True,
            bispectrum: bool = True, stream=None):
        """Run every job; returns (list of P tensors or None, list of B tensors or None)."""
        import torch

        if len(deltas) != self.n_jobs:
            raise ValueError("one field per job")
        for p, d in zip(self.plans, deltas):
            p._check_field(d)
        pks = bks = None
        if power:
            pks = pk_outs if pk_outs is not None else [
                _on_stream(torch.empty(p.n_bins, dtype=torch.float64, device=d.device), stream)
                for p, d in zip(self.plans, deltas)]
            for p, o, d in zip(self.plans, pks, deltas):
                p._out(o, p.n_bins, d)
        if bispectrum:
            bks = bk_outs if bk_outs is not None else [
                _on_stream(torch.empty(p.n_triplets, dtype=torch.float64, device=d.device), stream)
                for p, d in zip(self.plans, deltas)]
            for p, o, d in zip(self.plans, bks, deltas):
                p._out(o, p.n_triplets, d)
        da = _ptr_array([d.data_ptr() for d in deltas])
        pa = _ptr_array([o.data_ptr() for o in pks]) if pks is not None else None
        ba = _ptr_array([o.data_ptr() for o in bks]) if bks is not None else None
        _lib.check(self._lib.pb3_batch_run(self._h, da, pa, ba, _PREC[precision], _stream_handle(stream)))
        return pks, bks


def bispectrum_batched(plans, deltas, precision: str = "mixed", stream=None):
    """One-shot ``pb3_bispectrum_batched``: allocates, runs, synchronises."""
    import torch

    lib = _lib.load()
    for p, d in zip(plans, deltas):
        p._check_field(d)
    outs = [_on_stream(torch.empty(p.n_triplets, dtype=torch.float64, device=d.device), stream)
            for p, d in zip(plans, deltas)]
    _lib.check(lib.pb3_bispectrum_batched(
        _ptr_array([p._h.value for p in plans]), _ptr_array([d.data_ptr() for d in deltas]),
        _ptr_array([o.data_ptr() for o in outs]), len(plans), _PREC[precision], _stream_handle(stream)))
    return outs
