"""CPU checks of the native library: it loads, exports every symbol the
public header declares, and its host-side plan logic (bins, triplets,
contraction grid, argument errors) agrees with the oracle.  No kernel is
launched here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from synthetic import kf_edges

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2404_07249_amd", "libpb3.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libpb3.so not built (run __graft_entry__.build())")


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "pb3.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pb3_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    from paper_2404_07249_amd import _lib

    lib = C.CDLL(LIB)
    syms = _header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding declares each one
    declared = {n for n, _, _ in _lib.SIGNATURES}
    assert set(syms) == declared


def _plan(n, box, edges, **kw):
    import paper_2404_07249_amd as pb3

    return pb3.Plan(n, box, edges, host_only=True, **kw)


@pytest.mark.parametrize("n,nb,ntrip,m", [(32, 8, 98, 32), (128, 20, 1015, 128), (256, 30, 3035, 192)])
def test_host_plan_matches_oracle(n, nb, ntrip, m):
    edges = kf_edges(nb)
    p = _plan(n, 1000.0, edges)
    assert p.n_bins == nb
    assert p.n_triplets == ntrip  # host-only plans report the candidates
    assert np.array_equal(p.triplets, oracle.triangle_triplets(edges))
    e, kmean, nm = p.bins()
    assert np.array_equal(e, edges)
    if n <= 128:
        assert np.array_equal(nm, oracle.mode_counts(n, edges))
    assert p.contract_grid == m


def test_mode_counts_full_spectrum_with_nyquist():
    # top edge beyond N/2: the compact spectrum is the full one, Nyquist modes binned
    n = 16
    edges = np.array([1.0, 4.0, 7.0, 9.5, 14.0])
    p = _plan(n, 100.0, edges)
    _, _, nm = p.bins()
    assert np.array_equal(nm, oracle.mode_counts(n, edges))
    assert p.contract_grid == n


def test_edges_in_hmpc_are_snapped():
    n, box = 64, 1500.0
    kf = 2 * np.pi / box
    edges_kf = kf_edges(10)
    p = _plan(n, box, edges_kf * kf, edges_hmpc=True)
    e, _, nm = p.bins()
    assert np.array_equal(e, edges_kf)
    assert np.array_equal(nm, oracle.mode_counts(n, edges_kf))


@pytest.mark.parametrize(
    "n,edges,status",
    [
        (33, [1.0, 3.0], "EINVAL"),  # odd grid
        (100, [1.0, 3.0], "EUNSUPPORTED"),  # factor 5
        (32, [3.0, 1.0], "EINVAL"),  # unsorted
        (32, [1.0], "EINVAL"),  # one edge
        (32, [1.2, 1.3], "EINVAL"),  # a bin with no modes
        (32, list(range(1, 51)), "EUNSUPPORTED"),  # 49 bins
    ],
)
def test_plan_errors(n, edges, status):
    import paper_2404_07249_amd as pb3

    with pytest.raises(pb3.Pb3Error) as ei:
        _plan(n, 100.0, np.array(edges, dtype=float))
    assert status in str(ei.value)


@pytest.mark.parametrize("shape,box,edges,hmpc", [
    ((32, 48, 64), 1000.0, [1.0, 3.0, 5.0, 7.0, 9.0], False),
    ((64, 48, 32), (1000.0, 800.0, 500.0), [0.01, 0.03, 0.05, 0.07, 0.09, 0.11], True),
    ((192, 384, 192), (1015.8, 1911.0, 1057.7), list(0.005 + 0.01 * np.arange(13)), True)])
def test_noncubic_host_plan_matches_oracle(shape, box, edges, hmpc):
    """Host tables of a non-cubic plan: mode counts per bin and the triplet
    list equal the non-cubic oracle's; the contraction grid is chosen per axis."""
    from oracle import noncubic as nc

    p = _plan(shape, box, edges, edges_hmpc=hmpc)
    assert p.shape == tuple(shape)
    e, kmean, nm = p.bins()
    assert np.allclose(e, edges, rtol=0, atol=0)
    assert np.array_equal(nm, nc.mode_counts(shape, box, edges))
    assert np.array_equal(p.triplets, oracle.triangle_triplets(edges))
    m = p.contract_grid
    m3 = m if isinstance(m, tuple) else (m, m, m)
    assert all(mi <= ni for mi, ni in zip(m3, shape))


def test_noncubic_plan_errors():
    from paper_2404_07249_amd import _lib

    lib = _lib.load()
    e = (C.c_double * 2)(1.0, 3.0)

    def create(grid, box, flags=0):
        h = C.c_void_p()
        st = lib.pb3_plan_create((C.c_int * 3)(*grid), (C.c_double * 3)(*box), e, 2, _lib.FLAG_HOST_ONLY | flags,
                                 C.byref(h))
        if h.value:
            lib.pb3_plan_destroy(h)
        return st, lib.pb3_last_error()

    st, msg = create((32, 32, 64), (100.0, 100.0, 200.0))  # unequal sides need h/Mpc edges
    assert st == 1 and b"h/Mpc" in msg
    assert create((32, 30, 64), (100.0, 100.0, 100.0))[0] == 4  # 30 is not an implemented length
    assert create((32, 33, 64), (100.0, 100.0, 100.0))[0] == 1  # odd
    assert create((32, 48, 64), (100.0, 100.0, 100.0))[0] == 0


def test_host_only_plan_refuses_compute():
    import paper_2404_07249_amd as pb3
    from paper_2404_07249_amd import _lib

    p = _plan(32, 100.0, kf_edges(4))
    lib = _lib.load()
    pk = (C.c_double * 4)()
    st = lib.pb3_power(p._h, C.c_void_p(1), pk, None)
    assert st == 1
    with pytest.raises(pb3.Pb3Error):
        p.norm()


def test_batch_rejects_host_only_and_empty():
    """Batch argument checks that need no device: an empty job list and a
    host-only plan are EINVAL."""
    import paper_2404_07249_amd as pb3
    from paper_2404_07249_amd import _lib

    lib = _lib.load()
    h = C.c_void_p()
    assert lib.pb3_batch_create(None, 0, 0, C.byref(h)) == 1
    p = _plan(32, 100.0, kf_edges(4))
    arr = (C.c_void_p * 2)(p._h.value, p._h.value)
    assert lib.pb3_batch_create(arr, 2, 0, C.byref(h)) == 1
    assert not h.value
    assert lib.pb3_batch_create(arr, 2, 0x80, C.byref(h)) == 1  # unknown flag
    with pytest.raises(pb3.Pb3Error):
        pb3.Batch([p])


def test_launch_shape_query_on_host_plan():
    p = _plan(64, 1000.0, kf_edges(8))
    shape = p.launch_shape
    assert shape["tuned"] == "default" and shape["contract_wgs"] > 0


def test_power_only_plan_has_no_triplets():
    import paper_2404_07249_amd as pb3

    p = pb3.Plan(128, 1000.0, kf_edges(40), host_only=True, power_only=True)
    full = pb3.Plan(128, 1000.0, kf_edges(40), host_only=True)
    assert p.n_triplets == 0 and full.n_triplets > 0
    assert p.workspace_bytes < full.workspace_bytes


def test_multipole_plans_on_host():
    import paper_2404_07249_amd as pb3

    p = pb3.Plan(32, 500.0, kf_edges(6), host_only=True, lmax=4)
    assert p.n_ell == 3
    assert pb3.Plan(32, 500.0, kf_edges(6), host_only=True).n_ell == 1
    # one shell of the six axis modes has two mu^2 values: l = 0, 2, 4 cannot be separated
    with pytest.raises(pb3.Pb3Error):
        pb3.Plan(32, 500.0, np.array([1.0, 1.2]), host_only=True, lmax=4)
    assert pb3.Plan(32, 500.0, np.array([1.0, 1.2]), host_only=True, lmax=2).n_ell == 2
    with pytest.raises(ValueError):
        pb3.Plan(32, 500.0, kf_edges(6), host_only=True, lmax=3)


def test_contraction_tiles_hold_every_triplet_once():
    """Host logic of the MFMA tile layouts (the library's internal C++
    functions, called directly): for every bin count the kernels support,
    each triplet a <= b <= c has one partial-vector slot inside the tiles,
    no two triplets share one, and the layouts that trim a last 16-bin group
    of at most 4 or 8 real bins use fewer tiles than the full one."""
    lib = C.CDLL(LIB)
    loc = getattr(lib, "_ZN3pb311mfma_locateEbiiii")
    loc.restype, loc.argtypes = C.c_int, [C.c_bool, C.c_int, C.c_int, C.c_int, C.c_int]
    til = getattr(lib, "_ZN3pb310mfma_tilesEbi")
    til.restype, til.argtypes = C.c_int, [C.c_bool, C.c_int]
    for nb in range(1, 49):
        for ab in (False, True):
            nt = til(ab, nb)
            slots = [loc(ab, nb, a, b, c) for a in range(nb) for b in range(a, nb) for c in range(b, nb)]
            assert min(slots) >= 0 and max(slots) < 256 * nt, (nb, ab)
            assert len(set(slots)) == len(slots), (nb, ab)
    full = {1: 6, 2: 30, 3: 88}  # tiles of the untrimmed layout per group count
    for nb, want in [(4, 2), (8, 4), (16, 6), (17, 21), (20, 21), (21, 27), (24, 27), (25, 30), (32, 30),
                     (36, 74), (40, 84), (41, 88)]:
        assert til(False, nb) == want <= full[(nb + 15) // 16], nb
