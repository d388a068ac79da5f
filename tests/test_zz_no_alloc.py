"""The allocation-free export (msrsb_export_stage_noalloc) against
msrsb_export_stage through the C ABI: identical block ids, slot tables, basis
values and coarse operators, for rectilinear, fault-cut and dynamic stages in
FP64 and mixed precision, on two calls in a row with the second on a smaller
grid (the staging array keeps the first call's contents), and the grid-size
limit of the staging array."""
import numpy as np
import pytest

from workloads import make_config1, make_config2, make_homogeneous, pressure_increment_pair, rng_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def capi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi as c
    return c


def say(*a):
    print(*a, flush=True)


def _solver(capi, prob, precision):
    parts = [{"kind": "cartesian", "coarse_dims": (3, 4, 2)}, {"kind": "fault_cut", "parent": 0}]
    g = capi.Solver(prob, parts, capi.default_options(precision=precision, smoother="ilu0_rb"))
    g.update_basis(max_sweeps=12, tol=0.0)
    dp = pressure_increment_pair(prob, rng_for(8, 1))[0]
    g.add_dynamic_basis([torch.as_tensor(dp).cuda()])
    return g


def _same(a, b):
    assert a["M"] == b["M"] and a["n_slots"] == b["n_slots"]
    for key in ("block", "slot_block", "values", "Ac"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_export_matches_export(capi, precision):
    big = make_config2(dims=(24, 30, 12), seed=3)
    small = make_config1(dims=(10, 14, 6), seed=4)
    for prob in (big, small):  # second call on a smaller grid
        say(f"noalloc export {precision} dims={prob.dims}")
        g = _solver(capi, prob, precision)
        for k in range(g.num_stages()):
            ref = g.export_stage(k)
            got = g.export_stage(k, noalloc=True)
            _same(got, ref)
        g.close()


def test_noalloc_export_values_only(capi):
    prob = make_config1(dims=(12, 10, 6), seed=5)
    say("noalloc export values only")
    g = _solver(capi, prob, "mixed")
    import ctypes as C

    for k in range(g.num_stages()):
        M, kind, ns = g.stage_info(k)
        ref = g.export_stage(k, coarse=False)["values"].reshape(-1)
        vals = np.full(ns * g.N, np.nan)
        rc = capi._lib.msrsb_export_stage_noalloc(g.h, k, None, None, vals.ctypes.data_as(C.POINTER(C.c_double)),
                                                  None)
        assert rc == capi.OK
        assert np.array_equal(vals, ref)
    g.close()


def test_noalloc_export_rejects_grid_above_limit(capi):
    n = capi.NOALLOC_MAX_CELLS
    prob = make_homogeneous((129, 128, 128))
    assert prob.n_cells > n
    say("noalloc export size limit", prob.dims)
    g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}])
    with pytest.raises(capi.MsrsbError) as ei:
        g.export_stage(0, noalloc=True)
    assert ei.value.code == capi.E_INVAL
    g.close()
