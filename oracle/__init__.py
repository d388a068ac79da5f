"""CPU FP64 oracle of the multiscale restricted-smoothing pressure solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.
"""
from .msrsb import (  # noqa: F401
    OracleError,
    assemble,
    cartesian_partition,
    cartesian_support,
    fault_cut_partition,
    graph_partition,
    well_partition,
    indicator_partition,
    msrsb_basis,
    galerkin,
    coarse_factor,
    coarse_solve,
    jacobi_correction,
    ilu0_factor,
    ilu0_apply,
    ilu0_rb_fill,
    red_black_order,
    zline_red_black_order,
    natural_order,
    dynamic_partition,
    indicator,
    fluxes,
    fv_restriction,
    fv_multiscale_pressure,
    conservative_pressure,
    reconstructed_fluxes,
    cell_imbalance,
    Oracle,
)
