"""Host-side checks of the C-ABI library that need no GPU: the shared library
loads, exports every function ``include/msrsb.h`` declares, and its host logic
(grid validation, rectilinear support tables) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle.msrsb import support_1d
from workloads import make_config0, make_config2, make_homogeneous

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

capi = pytest.importorskip("paper_2001_01624_amd.capi", reason="libmsrsb.so not built")


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "msrsb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msrsb_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    import ctypes

    lib = ctypes.CDLL(capi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.EXPORTED)


def test_default_options():
    o = capi.default_options()
    assert o.omega == pytest.approx(2 / 3) and o.omega_s == pytest.approx(2 / 3)
    assert o.n_bins == 4 and o.max_dyn_blocks == 4096 and o.restart == 30
    assert o.smoother == capi.SMOOTH_JACOBI and o.precision == capi.FP64 and o.outer == capi.RICHARDSON


@pytest.mark.parametrize("n,m", [(15, 3), (8, 2), (10, 3), (5, 5), (7, 1), (60, 6), (220, 10), (85, 5), (37, 8),
                                 (128, 8), (9, 4), (2, 2), (1, 1)])
def test_axis_support_matches_oracle(n, m):
    lo, nv, slo, shi = capi.axis_support(n, m)
    sets = support_1d(n, m)
    for J, members in enumerate(sets):
        assert slo[J] == members[0] and shi[J] == members[-1]
        assert members == list(range(members[0], members[-1] + 1))
    for i in range(n):
        mine = [J for J in range(m) if i in sets[J]]
        assert mine == list(range(lo[i], lo[i] + nv[i]))


def test_axis_support_rejects_bad_sizes():
    with pytest.raises(capi.MsrsbError):
        capi.axis_support(3, 4)
    with pytest.raises(capi.MsrsbError):
        capi.axis_support(3, 0)


def test_validate_accepts_generated_models():
    assert capi.validate_grid(make_config0(0)) == capi.OK
    assert capi.validate_grid(make_config2(dims=(16, 20, 9), seed=1)) == capi.OK


def test_validate_rejects_bad_input():
    p = make_homogeneous((5, 4, 2))
    q = p.with_source()
    q.tx = p.tx.copy(); q.tx[3] = -1.0
    assert capi.validate_grid(q) == capi.E_INVAL
    q.tx = p.tx.copy(); q.tx[3] = np.nan
    assert capi.validate_grid(q) == capi.E_INVAL
    q.tx = p.tx.copy(); q.tx[4] = 1.0  # last column: face leaves the box
    assert capi.validate_grid(q) == capi.E_INVAL
    q.tx = p.tx.copy()
    q.active = p.active.copy(); q.active[7] = False  # faces still touch it
    assert capi.validate_grid(q) == capi.E_INVAL
    q.active = p.active.copy()
    q.bc_trans = np.zeros_like(p.bc_trans)  # no anchor: singular
    assert capi.validate_grid(q) == capi.E_SINGULAR
    q.bc_trans = p.bc_trans.copy()
    q.bc_cell = p.bc_cell.copy(); q.bc_cell[0] = 10 ** 6
    assert capi.validate_grid(q) == capi.E_INVAL
    q.bc_cell = p.bc_cell.copy()
    q.source = np.full(p.n_cells, np.inf)
    assert capi.validate_grid(q) == capi.E_INVAL


def test_footprint_is_positive_and_grows():
    p = make_config0(0)
    parts = [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}]
    f64 = capi.footprint_bytes(p, parts)
    mixed = capi.footprint_bytes(p, parts, capi.default_options(precision="mixed"))
    gm = capi.footprint_bytes(p, parts, capi.default_options(outer="gmres"))
    assert f64 > 3600 * 8 * 10 and gm > f64 and mixed > 0
    assert capi.footprint_bytes(p, [{"kind": "cartesian", "coarse_dims": (100, 1, 1)}]) == 0


def _bare_grid(nx, ny, nz):
    # only the box size: msrsb_footprint_bytes reads no per-cell array
    g = capi.Grid()
    g.nx, g.ny, g.nz = nx, ny, nz
    return g


def _footprint(dims, cd, **opt):
    import ctypes

    parts = capi._parts([{"kind": "cartesian", "coarse_dims": cd}])
    o = capi.default_options(**opt)
    return int(capi._lib.msrsb_footprint_bytes(ctypes.byref(_bare_grid(*dims)), 1, parts.arr, ctypes.byref(o)))


def test_footprint_rejects_grids_beyond_32_bit_slot_offsets():
    # a 3-D rectilinear stage keeps 8 slots per cell; the basis kernels address
    # them with 32-bit byte offsets, so 8 slots * N * 8 bytes must stay < 2^31
    assert _footprint((256, 256, 511), (8, 8, 8)) > 0          # N < 2^25: 8 * N * 8 < 2^31
    assert _footprint((256, 256, 512), (8, 8, 8)) == 0         # N = 2^25: 8 * N * 8 = 2^31
    assert _footprint((256, 600, 500), (8, 8, 8)) == 0         # N = 76.8 M: slots overflow
    assert _footprint((256, 600, 500), (8, 8, 8), precision="mixed") == 0
    # fewer split axes, fewer slots: a 1-D partition of the same grid fits
    assert _footprint((256, 600, 500), (8, 1, 1)) > 0
    # more than (2^31 - 1) / 8 cells is refused outright
    assert _footprint((1024, 1024, 300), (1, 1, 1)) == 0


class _FakeDeviceTensor:
    """Just enough of a tensor's interface for the binding's argument checks."""

    def __init__(self, n, device=0, dtype="float64", contiguous=True):
        import types

        self.is_cuda = True
        self._n, self._c = n, contiguous
        self.dtype = f"torch.{dtype}"
        self.device = types.SimpleNamespace(index=device)

    def is_contiguous(self):
        return self._c

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def test_binding_rejects_wrong_vectors_before_any_call():
    assert capi._dptr(_FakeDeviceTensor(10), n=10, device=0).value == 0x1000
    for bad in (_FakeDeviceTensor(9), _FakeDeviceTensor(11), _FakeDeviceTensor(10, device=1),
                _FakeDeviceTensor(10, dtype="float32"), _FakeDeviceTensor(10, contiguous=False)):
        with pytest.raises(capi.MsrsbError) as e:
            capi._dptr(bad, n=10, device=0)
        assert e.value.code == capi.E_INVAL


# --- static partition builders (host functions of the library) against the oracle

def _small_models():
    from workloads import make_config1, make_lognormal_box, rng_for

    return [make_config2(dims=(9, 8, 5), seed=3), make_config1(dims=(12, 14, 6), seed=1),
            make_lognormal_box((20, 16, 3), rng_for(9, 2), sigma=2.0, corr=(2.0, 2.0, 1.0))]


@pytest.mark.parametrize("radius", [0, 1, 2, 5])
def test_partition_wells_matches_oracle(radius):
    import oracle as O

    for k, prob in enumerate(_small_models()):
        rng = np.random.default_rng(100 + k)
        cells = np.nonzero(prob.active)[0]
        wells = [rng.choice(cells, size=int(rng.integers(1, 5)), replace=False) for _ in range(4)]
        wells.append(wells[0][:1])  # a cell shared by two wells goes to the lower index
        got = capi.partition_wells(prob, wells, radius)
        assert np.array_equal(got, O.well_partition(prob, wells, radius))


@pytest.mark.parametrize("n_bins,cd,min_cells", [(2, (1, 1, 1), 0), (4, (3, 2, 1), 5), (3, (2, 2, 2), 12),
                                                 (6, (1, 1, 1), 40)])
def test_partition_indicator_matches_oracle(n_bins, cd, min_cells):
    import oracle as O

    for prob in _small_models():
        ind = np.log(prob.perm)
        ind = np.round(ind, 1)  # ties between cells exercise the rank order
        got = capi.partition_indicator(prob, ind, n_bins, cd, min_cells)
        assert np.array_equal(got, O.indicator_partition(prob, ind, n_bins, cd, min_cells))


def test_partition_builders_reject_bad_input():
    prob = make_config0(0)
    with pytest.raises(capi.MsrsbError):
        capi.partition_wells(prob, [np.array([-1])], 1)
    with pytest.raises(capi.MsrsbError):
        capi.partition_wells(prob, [np.array([0])], -1)
    ind = np.zeros(prob.n_cells)
    ind[5] = np.nan
    with pytest.raises(capi.MsrsbError):
        capi.partition_indicator(prob, ind, 4, (2, 2, 1), 0)
    with pytest.raises(capi.MsrsbError):
        capi.partition_indicator(prob, np.zeros(prob.n_cells), 0, (2, 2, 1), 0)


# --- face-list input for box grids (msrsb_faces_to_box)

@pytest.mark.parametrize("mk", [lambda: make_config0(3), lambda: make_config2(dims=(9, 11, 6), seed=5),
                                lambda: make_homogeneous((4, 1, 7))])
def test_faces_to_box_round_trip(mk):
    # the oracle's own face enumeration of a model, shuffled, gives back the
    # model's structured arrays bit for bit
    from oracle.msrsb import _faces

    prob = mk()
    a, b, t = _faces(prob)
    perm = np.random.default_rng(4).permutation(a.size)
    tx, ty, tz = capi.faces_to_box(prob.dims, np.stack([a, b], axis=1)[perm], t[perm])
    assert np.array_equal(tx, prob.tx) and np.array_equal(ty, prob.ty) and np.array_equal(tz, prob.tz)


def test_faces_to_box_rejects_non_box_faces():
    dims = (4, 3, 2)
    ok = [[0, 1], [0, 4], [0, 12]]
    capi.faces_to_box(dims, ok, [1.0, 2.0, 3.0])
    for cells, t in (([[3, 4]], [1.0]),      # x "neighbours" across a row end
                     ([[8, 12]], [1.0]),     # y neighbours across a layer end
                     ([[0, 2]], [1.0]),      # not adjacent
                     ([[1, 0]], [1.0]),      # descending pair
                     ([[0, 24]], [1.0]),     # outside the box
                     ([[0, 1], [0, 1]], [1.0, 1.0]),  # the same face twice
                     ([[0, 1]], [-1.0]), ([[0, 1]], [np.nan]), ([[0, 1]], [np.inf])):
        with pytest.raises(capi.MsrsbError) as ei:
            capi.faces_to_box(dims, cells, t)
        assert ei.value.code == capi.E_INVAL
