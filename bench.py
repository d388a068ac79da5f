#!/usr/bin/env python3
"""Throughput of the MI355X MsRSB pressure solver: fine cells solved per
second to 1e-6 relative residual on the layered five-spot model
(60 x 220 x 85 = 1,122,000 cells, 20 x 10 x 2 cells, smooth lognormal top /
sinusoidal-channel bottom, five-spot wells).

One step = one request on the device-resident model: build the multibasis
prolongations from scratch (restricted smoothing to tol 1e-3, at most 100
sweeps, Galerkin operators, coarse inverses), solve from zero for source q1,
re-solve for a changed source q2 (a new injector), add a dynamic stage from
the increment x2 - x1, solve for q3, and compute fluxes.  Every solve runs to
||b - A x|| <= 1e-6 ||b|| (checked on the true FP64 residual).  Value = 3 *
active cells * steps / wall time (inputs already in HBM; model setup, i.e.
validation, assembly and integer partition tables, is timed apart as setup_ms).

The same line carries the mixed-precision request, the faulted model with a
fault-cut and two dynamic stages, the serving stream, the batched ensemble,
a per-class kernel table (HIP events), the roofline of the largest kernel
class (the fine-grid pass of the residual-restriction) and the oracle timed
on the host's cores.

Prints one JSON line (progress on stderr).  `--gpus N` with N > 1 exits: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine cells solved/s to 1e-6 rel. residual (FP64 plain vs mixed+served); p50/p99"
HBM_PEAK_GBS = 8000.0
DIMS = (60, 220, 85)
STAGES = [(10, 10, 5), (6, 22, 17)]
# GMRES restart length of the request: with the z-line ILU(0) smoother,
# restarts 10..31 all need 39-42 iterations per solve on this model, and 16
# and 20 are the fastest (fewer basis vectors per step)
RESTART = 16
RTOL = 1e-6
TWOPHASE_DT = 2.0e4  # time step of the two-phase leg (model units; plain Newton diverges at 2e5)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel", default="auto",
                    help="kernel class of the roofline object; auto: the single-kernel class with the largest "
                         "time per request, from the kernel table taken before the timed steps")
    ap.add_argument("--no-table", action="store_true", help="skip the per-class kernel table")
    ap.add_argument("--smoother", default="ilu0_line", choices=["ilu0_line", "ilu0_rb", "jacobi"],
                    help="fine-scale smoother of every GPU leg and of the oracle baseline")
    ap.add_argument("--no-faulted", action="store_true", help="skip the faulted-model (two-stage + dynamic) leg")
    ap.add_argument("--faulted-only", action="store_true",
                    help="profiling aid: run only the faulted-model request and print its record")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-only", action="store_true",
                    help="profiling aid: run only the mixed-precision request and print its record")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1200)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched ensemble (also skipped by --no-serve)")
    ap.add_argument("--ensemble-members", type=int, default=256)
    ap.add_argument("--ensemble-batch-only", action="store_true",
                    help="profiling aid: run only the batched ensemble (set-up on one thread) and print its record")
    ap.add_argument("--no-static", action="store_true", help="skip the static-stage (well, indicator) leg")
    ap.add_argument("--no-fv", action="store_true", help="skip the finite-volume leg")
    ap.add_argument("--no-twophase", action="store_true", help="skip the two-phase CPR leg")
    ap.add_argument("--extras-only", action="store_true",
                    help="profiling aid: run only the static-stage, finite-volume and two-phase legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain copy of this size (counter calibration)")
    return ap.parse_args()


def workload(dims=DIMS, seed=0):
    """Model plus the three sources of a request (injector only; injector split
    with a new column; the new column rescaled)."""
    import numpy as np

    from workloads import make_config1, rng_for

    prob = make_config1(dims=dims, seed=seed)
    nx, ny, nz = prob.dims
    rng = rng_for(4, seed)
    q1 = prob.source.copy()
    inj = prob.wells["injector"]
    cx, cy = int(rng.integers(nx // 4, 3 * nx // 4)), int(rng.integers(ny // 4, 3 * ny // 4))
    col = np.array([cx + nx * (cy + ny * k) for k in range(nz)])
    col = col[prob.active[col]]
    q2 = q1 * 0.5
    q2[col] += 0.5 / col.size
    q3 = q2.copy()
    q3[col] *= rng.uniform(0.5, 1.5)
    return prob, [q1, q2, q3]


# algorithmic bytes per active cell for one launch of each kernel class
# (structured 7-point storage: three face T and the diagonal per cell)
SMOOTHER_NAMES = {"ilu0_line": "ILU(0) in z-line red-black order", "ilu0_rb": "red-black ILU(0)",
                  "jacobi": "damped Jacobi"}


def bytes_per_cell(kernel, ns, mixed, smoother="ilu0_line"):
    sp = 4 if mixed else 8       # working precision of the sweeps and the smoother
    sb = 2 if mixed else 8       # stored basis (BF16 in mixed precision)
    if smoother == "ilu0_line":  # r, x in/out, three T, diagonal, pivot, z coupling, scratch written and read
        smooth = 8 + 16 + 3 * sp + 8 + 2 * sp + 16
    else:                        # r, x in/out, three T, diagonal, pivot
        smooth = 44 if mixed else 64
    return {
        "sweep": 2 * ns * sp + 3 * sp + 8,        # read P, write P, three face T, diagonal
        "restrict_rows": 48 + ns * sb,            # P, x, b, three face T, diagonal (residual fused)
        "restrict": 48 + ns * sb,                 # the same, with the final gather of the partial sums
        "prolong": ns * sb + 16,                  # P, x read and written
        "residual": 56,                           # x, b, r, three face T, diagonal
        "smooth": smooth,
    }.get(kernel)  # the "matvec" class is the Arnoldi pass A (matrix-vector product fused with dots): no entry


def gpu_leg(args, precision):
    import numpy as np
    import torch

    from paper_2001_01624_amd import capi

    prob, sources = workload()
    parts = [{"kind": "cartesian", "coarse_dims": cd} for cd in STAGES]
    opt = capi.default_options(smoother=args.smoother, outer="gmres", restart=RESTART, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = capi.Solver(prob, parts, opt)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    q = [torch.as_tensor(s).cuda() for s in sources]
    N = prob.n_cells
    x1 = torch.zeros(N, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    x3 = torch.zeros_like(x1)
    info = {}

    def step():
        rec = {}
        t = time.perf_counter()
        g.clear_dynamic_basis()
        sweeps = []
        for k in range(len(STAGES)):
            sw, _ = g.update_basis(stage=k, max_sweeps=100, tol=1e-3)
            sweeps.append(sw)
        x1.zero_()
        it1, r1, c1 = g.solve(x1, source=q[0], rtol=RTOL, max_iters=3000)
        x2.copy_(x1)
        it2, r2, c2 = g.solve(x2, source=q[1], rtol=RTOL, max_iters=3000)
        d = x2 - x1
        nd = g.add_dynamic_basis([d])
        x3.copy_(x2)
        it3, r3, c3 = g.solve(x3, source=q[2], rtol=RTOL, max_iters=3000)
        g.fluxes(x3)
        torch.cuda.synchronize()
        rec["ms"] = 1e3 * (time.perf_counter() - t)
        rec["iters"] = [it1, it2, it3]
        rec["relres"] = [r1, r2, r3]
        rec["status"] = [c1, c2, c3]
        rec["sweeps"] = sweeps
        rec["dyn_blocks"] = nd
        return rec

    for _ in range(args.warmup):
        step()
    n_act = prob.n_active
    ns = 8
    # per-class kernel times (untimed requests), and the roofline's class
    table = None if args.no_table else kernel_table(g, step, ns, precision, n_act, args.smoother)
    roof_class = args.kernel
    if roof_class == "auto":
        cand = table if table is not None else kernel_table(g, step, ns, precision, n_act, args.smoother,
                                                            ROOF_CANDIDATES)
        roof_class = max(ROOF_CANDIDATES, key=lambda c: cand[c]["ms_per_request"])
    torch.cuda.synchronize()
    recs = []
    g.profile_begin(roof_class, 200000)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = g.profile_end()
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    ms = sorted(rec["ms"] for rec in recs)
    cells = 3 * n_act * args.steps
    roof = roofline(roof_class, ns, precision, n_act, kern_ms, launches, args.smoother)
    out = {
        "value": cells / wall,
        "ms_per_step": 1e3 * wall / args.steps,
        "p50_ms": ms[len(ms) // 2],
        "p99_ms": ms[min(len(ms) - 1, int(round(0.99 * (len(ms) - 1))))],
        "setup_ms": setup_ms,
        "iters": [rec["iters"] for rec in recs][-1],
        "sweeps": recs[-1]["sweeps"],
        "dyn_blocks": recs[-1]["dyn_blocks"],
        "relres": max(max(rec["relres"]) for rec in recs),
        "all_converged": all(s == 0 for rec in recs for s in rec["status"]),
        "roofline": roof,
        "kernel_table": table,
        "cells": n_act,
    }
    g.close()
    return out


ROOF_KERNEL = {"restrict_rows": "k_restrict_rows", "sweep": "k_sweep", "restrict": "k_restrict_rows+k_restrict_gather",
               "prolong": "k_prolong_rows", "residual": "k_residual_rows"}
SMOOTH_KERNEL = {"ilu0_line": "k_lilu_reg (three colour passes)", "ilu0_rb": "k_ilu_zm", "jacobi": "k_jacobi"}


def roofline(kernel, ns, precision, n_act, kern_ms, launches, smoother):
    """Roofline object of one kernel class: algorithmic bytes per launch over
    the average launch time from the HIP events of the timed steps."""
    bpc = bytes_per_cell(kernel, ns, precision == "mixed", smoother)
    if bpc is None or launches == 0:
        return None
    per_launch = bpc * n_act
    avg_s = kern_ms / launches / 1e3
    ach = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_record(kernel, precision),
            "kernel": SMOOTH_KERNEL[smoother] if kernel == "smooth" else ROOF_KERNEL.get(kernel, kernel),
            "kernel_class": kernel, "launches": launches,
            "avg_launch_us": round(1e6 * avg_s, 2), "algorithmic_bytes_per_cell": bpc,
            "algorithmic_bytes_per_launch": per_launch}


TABLE_CLASSES = ("restrict_rows", "restrict", "sweep", "prolong", "smooth", "residual", "ortho", "matvec", "coarse",
                 "rap", "inverse")


# single-kernel classes the roofline object may name (the fine-grid passes of
# the basis construction and of the multistage cycle)
ROOF_CANDIDATES = ("sweep", "restrict_rows", "prolong", "residual")


def kernel_table(g, step, ns, precision, n_act, smoother, classes=None):
    """One extra (untimed) request per kernel class, that class's launches
    bracketed by HIP events: launches and milliseconds per request, average
    launch, and achieved bandwidth where the algorithmic bytes are known."""
    out = {}
    for cls in classes or TABLE_CLASSES:
        g.profile_begin(cls, 200000)
        step()
        ms, n = g.profile_end()
        row = {"launches": n, "ms_per_request": round(ms, 3), "avg_us": round(1e3 * ms / n, 2) if n else None}
        bpc = bytes_per_cell(cls, ns, precision == "mixed", smoother)
        if bpc is not None and n:
            gbs = bpc * n_act / (ms / n / 1e3) / 1e9
            row.update({"bytes_per_cell": bpc, "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        out[cls] = row
    return out


def faulted_leg(args):
    """The faulted model (60x220x85, three planar faults, 5 % inactive cells)
    in mixed precision with a rectilinear stage (10x10x5 coarse blocks), its
    fault-cut stage and up to two dynamic stages: one request = both bases
    from scratch, then five solves with a moved or rescaled source/sink pair,
    the increments of the last two solutions becoming dynamic stages from
    the third solve on (the serving loop's recipe)."""
    import torch

    from paper_2001_01624_amd import capi
    from workloads import make_config2, rng_for
    from workloads.requests import source_sequence

    prob = make_config2(seed=0)
    sources = source_sequence(prob, rng_for(6, 0), 5)
    parts = [{"kind": "cartesian", "coarse_dims": (10, 10, 5)}, {"kind": "fault_cut", "parent": 0}]
    opt = capi.default_options(smoother=args.smoother, outer="gmres", restart=RESTART, precision="mixed")
    g = capi.Solver(prob, parts, opt)
    q = [torch.as_tensor(s).cuda() for s in sources]
    N = prob.n_cells
    xs = [torch.zeros(N, dtype=torch.float64, device="cuda") for _ in q]

    def step():
        rec = {"iters": [], "relres": [], "status": [], "dyn": [], "solve_ms": []}
        t = time.perf_counter()
        g.clear_dynamic_basis()
        rec["sweeps"] = [g.update_basis(stage=k, max_sweeps=100, tol=1e-3)[0] for k in range(len(parts))]
        for k in range(len(q)):
            ts = time.perf_counter()
            if k >= 2:
                incs = [xs[k - 1] - xs[k - 2]] + ([xs[k - 2] - xs[k - 3]] if k >= 3 else [])
                rec["dyn"].append(g.add_dynamic_basis(incs))
            if k == 0:
                xs[0].zero_()
            else:
                xs[k].copy_(xs[k - 1])
            it, rel, rc = g.solve(xs[k], source=q[k], rtol=RTOL, max_iters=3000)
            torch.cuda.synchronize()
            rec["solve_ms"].append(1e3 * (time.perf_counter() - ts))
            rec["iters"].append(it)
            rec["relres"].append(rel)
            rec["status"].append(rc)
        rec["ms"] = 1e3 * (time.perf_counter() - t)
        return rec

    for _ in range(args.warmup):
        step()
    recs = [step() for _ in range(args.steps)]
    wall = sum(r["ms"] for r in recs) / 1e3
    n_act = prob.n_active
    out = {"value": len(q) * n_act * len(recs) / wall, "unit": "cells/s", "ms_per_request": 1e3 * wall / len(recs),
           "solve_ms_3_to_5": [round(x, 2) for x in recs[-1]["solve_ms"][2:]], "iters": recs[-1]["iters"],
           "sweeps": recs[-1]["sweeps"], "dyn_blocks": recs[-1]["dyn"],
           "max_relres": max(max(r["relres"]) for r in recs),
           "all_converged": all(s == 0 for r in recs for s in r["status"]), "cells": n_act,
           "stages": [g.stage_info(k)[:3:2] for k in range(len(parts))],
           "workload": "faulted 60x220x85 (3 faults, 5% inactive), mixed precision, rectilinear 10x10x5 + fault-cut "
                       "+ <=2 dynamic stages, GMRES(16), 5 solves per request (source/sink pair moved or rescaled)"}
    out["kernel_table"] = None if args.no_table else kernel_table(g, step, 8, "mixed", n_act, args.smoother)
    g.close()
    return out


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, 1e3 * (time.perf_counter() - t)


def static_leg(args):
    """Static stages (partition type "Static": well bases and an indicator
    agglomeration, GRAPH stages on the explicit-slot kernels) added to the
    request's two general stages on the 60x220x85 model, FP64: both bases
    built (<= 100 sweeps, tol 1e-3) and three GMRES solves from zero, per
    stage set; the oracle on the 30x110x21 sample with the well stage beside."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2001_01624_amd import capi

    prob, sources = workload()
    base = [{"kind": "cartesian", "coarse_dims": cd} for cd in STAGES]

    def wells_of(p):
        prod = p.wells["producers"]
        return [p.wells["injector"]] + [prod[k * (prod.size // 4):(k + 1) * (prod.size // 4)] for k in range(4)]

    wb = capi.partition_wells(prob, wells_of(prob), 3)
    ib = capi.partition_indicator(prob, np.log(prob.perm), 4, (10, 10, 5), 64)
    sets = {"general": base,
            "general+wells": base + [{"kind": "graph", "block_of_cell": wb, "overlap": 8}],
            "general+indicator": base + [{"kind": "graph", "block_of_cell": ib, "overlap": 2}]}
    q = [torch.as_tensor(x).cuda() for x in sources]
    x = torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda")
    out = {}
    for name, parts in sets.items():
        g = capi.Solver(prob, parts, capi.default_options(smoother=args.smoother, outer="gmres", restart=RESTART))

        def request():
            sw = [g.update_basis(stage=k, max_sweeps=100, tol=1e-3)[0] for k in range(len(parts))]
            its, rels = [], []
            for qk in q:
                x.zero_()
                it, rel, rc = g.solve(x, source=qk, rtol=RTOL, max_iters=3000)
                its.append(it)
                rels.append(rel if rc == capi.OK else float("inf"))
            return sw, its, rels

        request()
        (sw, its, rels), ms = _timed(request)
        out[name] = {"request_ms": round(ms, 2), "value": 3 * prob.n_active / (ms / 1e3), "iters": its,
                     "sweeps": sw, "max_relres": max(rels),
                     "stages": [list(g.stage_info(k)[:2]) for k in range(len(parts))]}
        g.close()
    sp, ss = workload(dims=(30, 110, 21))
    t = time.perf_counter()
    o = O.Oracle(sp, [{"kind": "cartesian", "coarse_dims": (5, 5, 1)}, {"kind": "cartesian", "coarse_dims": (3, 11, 4)},
                      {"kind": "graph", "block_of_cell": O.msrsb.well_partition(sp, wells_of(sp), 3), "overlap": 8}],
                 smoother=args.smoother)
    o.update_basis(100, 1e-3)
    _, oit, _, _ = o.solve_gmres(source=ss[0], rtol=RTOL, restart=RESTART, max_iters=3000)
    out["oracle_sample"] = {"seconds": round(time.perf_counter() - t, 2), "cells": sp.n_active, "iters": oit,
                            "what": "30x110x21 sample, general stages 5x5x1 and 3x11x4 plus the well stage: "
                                    "set-up, bases and one solve"}
    out["workload"] = ("60x220x85 layered model, FP64, z-line ILU(0), GMRES(16); static stages: five wells "
                       "(injector + producers in four groups, radius 3, support overlap 8) and a log-permeability "
                       "agglomeration (4 bins, parent blocks 10x10x5, >= 64 cells, overlap 2); request = bases + "
                       "three solves from zero")
    return out


def fv_leg(args):
    """Finite-volume mode (msrsb_solve_fv) on the 60x220x85 model: the
    10x10x5 stage's basis, then for each of the request's three sources the
    multiscale pressure with R_fv and conservative fine fluxes from the
    per-block Neumann problems; the oracle on the 30x110x21 sample beside."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2001_01624_amd import capi

    prob, sources = workload()
    parts = [{"kind": "cartesian", "coarse_dims": STAGES[0]}]
    g = capi.Solver(prob, parts, capi.default_options(smoother=args.smoother))
    g.update_basis(max_sweeps=100, tol=1e-3)
    q = [torch.as_tensor(x).cuda() for x in sources]
    g.solve_fv(0, q[0])
    recs = []
    for qk in q:
        (p, pf, face, bcf, its, imb), ms = _timed(lambda: g.solve_fv(0, qk))
        recs.append((ms, its, imb / float(torch.abs(qk).max())))
    g.close()
    sp, ss = workload(dims=(30, 110, 21))
    t = time.perf_counter()
    o = O.Oracle(sp, [{"kind": "cartesian", "coarse_dims": (5, 5, 1)}])
    o.update_basis(100, 1e-3)
    o.solve_fv(0, ss[0])
    return {"ms_per_solve": [round(r[0], 2) for r in recs], "value": prob.n_active / (np.mean([r[0] for r in recs]) / 1e3),
            "unit": "cells/s", "local_iters": [r[1] for r in recs],
            "max_cell_imbalance_over_max_source": max(r[2] for r in recs),
            "oracle_sample": {"seconds": round(time.perf_counter() - t, 2), "cells": sp.n_active,
                              "what": "30x110x21 sample, 5x5x1 stage: set-up, basis, one finite-volume solve"},
            "workload": "60x220x85 layered model, FP64, 10x10x5 stage (<= 100 sweeps, tol 1e-3); per source: "
                        "p_ms = P A_fv^-1 R_fv b and fine fluxes from per-block Neumann problems to 1e-12"}


def twophase_leg(args):
    """Two-phase fully implicit time steps with the CPR preconditioner on the
    60x220x85 model (water injected at the injector column, producers held at
    their connection pressures): three backward-Euler steps with Newton,
    GMRES(30) on the full system, the multistage cycle of the two general
    stages as the pressure predictor and red-black block ILU(0) as the
    corrector, dynamic bases from the Newton pressure updates (Dp(Inf));
    the two-phase oracle on a 16x20x6 sample beside."""
    import numpy as np
    import torch

    from oracle import twophase as TP
    import oracle as O
    from paper_2001_01624_amd import capi, twophase
    from workloads import make_config1

    fluid = dict(mu_w=1.0, mu_o=5.0, n_w=2.0, n_o=2.0)
    prob, _ = workload()
    parts = [{"kind": "cartesian", "coarse_dims": cd} for cd in STAGES]
    g = capi.Solver(prob, parts, capi.default_options(smoother=args.smoother, outer="gmres"))
    g.update_basis(max_sweeps=100, tol=1e-3)
    pv = np.full(prob.n_cells, 0.2 * np.prod(prob.h)) * prob.active
    tp = capi.TwoPhase(g, pv, fluid, restart=30)
    p = torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda")
    s = torch.as_tensor(np.full(prob.n_cells, 0.2) * prob.active).cuda()
    dt = TWOPHASE_DT
    steps, last = [], None
    for k in range(3):
        st, ms = _timed(lambda: twophase.time_step(tp, p, s, dt, newton_tol=1e-6, lin_rtol=1e-6, lin_max=1000,
                                                   last_dp=last))
        last = st["last_dp"]
        steps.append({"ms": round(ms, 1), "newton": st["newton"], "linear": st["linear"],
                      "converged": not st.get("failed") and st["res"][-1] <= 1e-6 * st["res"][0]})
    tp.close()
    g.close()
    tot = sum(x["ms"] for x in steps)
    small = make_config1(dims=(16, 20, 6), seed=5)
    t = time.perf_counter()
    o = O.Oracle(small, [{"kind": "cartesian", "coarse_dims": (2, 2, 2)}], smoother="ilu0_rb")
    o.update_basis(30, 1e-3)
    ot = TP.TwoPhase(small, np.full(small.n_cells, 0.2 * np.prod(small.h)) * small.active, fluid, dt, o)
    z = np.zeros(small.n_cells)
    s0 = np.full(small.n_cells, 0.2) * small.active
    _, _, oits, _, _ = ot.newton_step(z, s0.copy(), s0, rtol=1e-6)
    return {"ms_per_step": round(tot / len(steps), 1), "value": len(steps) * prob.n_active / (tot / 1e3),
            "unit": "cell-steps/s", "steps": steps,
            "oracle_sample": {"seconds": round(time.perf_counter() - t, 2), "cells": small.n_active,
                              "gmres_iters": oits, "what": "16x20x6 sample: set-up, basis, one Newton step with "
                                                          "GMRES + CPR to 1e-6"},
            "workload": f"60x220x85 layered model, water/oil (mu 1/5 cP, Corey 2/2), dt {dt:g}, three steps from "
                        "s = 0.2, Newton to 1e-6, GMRES(30) + CPR (multistage cycle of the 10x10x5 and 6x22x17 "
                        "stages with z-line ILU(0); red-black block ILU(0) of the full system)"}


def serve_leg(args):
    """The same seeded Poisson stream (200 requests/s; 10 % layered
    60x220x85 models with two general stages, 90 % ensemble members
    32..128 x 32..128 x 8..16 with one 8x8x4 stage; 1-5 solves each) served
    two ways: FP64, one request at a time; mixed precision with eight
    concurrent slots (continuous batching, HBM-footprint admission; eight
    measured best: 4, 6, 12 and 16 slots gave less)."""
    from paper_2001_01624_amd import capi
    from paper_2001_01624_amd.serve import Server
    from workloads.requests import poisson_stream

    Server(slots=1).run(poisson_stream(2, 200.0, seed=99), realtime=False)  # load kernels
    out = {}
    for name, slots, prec in (("fp64_plain", 1, "fp64"), ("mixed_served", 8, "mixed")):
        reqs = poisson_stream(args.serve_requests, 200.0, seed=0)
        opt = capi.default_options(smoother=args.smoother, outer="gmres", precision=prec)
        st = Server(slots=slots, options=opt, rtol=RTOL).run(reqs, realtime=True)
        out[name] = {"cells_per_s": st["cells_per_s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                     "solves": st["solves"], "requests": st["completed"], "makespan_s": st["makespan_s"],
                     "all_converged": st["all_converged"], "max_relres": st["max_relres"], "slots": slots}
    # maximum sustainable rate: the same stream with every request available at once
    reqs = poisson_stream(args.serve_requests, 200.0, seed=0)
    opt = capi.default_options(smoother=args.smoother, outer="gmres", precision="mixed")
    st = Server(slots=8, options=opt, rtol=RTOL).run(reqs, realtime=False)
    out["mixed_served"]["max_rate_cells_per_s"] = st["cells_per_s"]
    out["speedup"] = out["mixed_served"]["cells_per_s"] / out["fp64_plain"]["cells_per_s"]
    out["stream"] = (f"{args.serve_requests} requests, Poisson 200/s, 10% layered 60x220x85 (2 stages), 90% "
                     f"ensemble members (1 stage 8x8x4), 1-5 solves each, rtol {RTOL}")
    return out


def ensemble_leg(args):
    """Ensemble of members of 32..128 x 32..128 x 8..16 cells (one 8x8x4
    stage), one solve each to 1e-6 with the member's own source, in FP64 and
    in mixed precision.  Batched: every member set up on its own context (8
    host threads), then one msrsb_batch over all of them (basis sweeps,
    Galerkin operators, inverses and the GMRES cycle each one launch per
    kernel over all members); reported device-resident (basis + solve, as the
    request legs) and end to end (with set-up and teardown).  For comparison
    the same members through the serving loop, eight concurrent contexts.
    End to end, the pipelined form (serve.run_ensemble: batches of 64
    members, the next batch set up and the previous one torn down on host
    threads while the current one runs).  Per solve, the largest difference
    of the mixed solution from the FP64 one relative to the FP64 solution's
    largest entry."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    from paper_2001_01624_amd import capi
    from paper_2001_01624_amd.serve import Server, run_ensemble
    from workloads.requests import ensemble_batch

    out, sols = {}, {}
    for prec in ("fp64", "mixed"):
        opt = capi.default_options(smoother=args.smoother, outer="gmres", precision=prec, restart=RESTART)
        reqs = ensemble_batch(args.ensemble_members, seed=0)
        cells = sum(r.cells for r in reqs)
        stream = torch.cuda.Stream()
        rec = None
        for rep in range(2):  # the second run is reported (the first pages in code and pool memory)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with ThreadPoolExecutor(1 if args.ensemble_batch_only else 8) as ex:
                gs = list(ex.map(lambda r: capi.Solver(r.problem, r.partitions, opt, stream=stream), reqs))
            xs = [torch.zeros(g.N, dtype=torch.float64, device="cuda") for g in gs]
            qs = [torch.as_tensor(r.sources[0]).to("cuda") for r in reqs]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            B = capi.Batch(gs, stream=stream)
            sweeps = B.update_basis(max_sweeps=100, tol=1e-3)
            t2 = time.perf_counter()
            it, rel, st = B.solve(xs, sources=qs, rtol=RTOL, max_iters=3000)
            t3 = time.perf_counter()
            B.close()
            x_host = [x.cpu().numpy() for x in xs]
            for g in gs:
                g.close()
            t4 = time.perf_counter()
            rec = {"cells_per_s": cells / (t3 - t1), "cells_per_s_one_batch_end_to_end": cells / (t4 - t0),
                   "basis_s": t2 - t1, "solve_s": t3 - t2, "setup_s": t1 - t0, "teardown_s": t4 - t3,
                   "iters_mean": float(np.mean(it)), "iters_max": int(max(it)), "sweeps_max": int(max(sweeps)),
                   "all_converged": all(s == 0 for s in st), "max_relres": float(max(rel))}
        sols[prec] = x_host
        if args.ensemble_batch_only:
            out[prec] = {"batched": rec}
            continue
        reqs = ensemble_batch(args.ensemble_members, seed=0)
        pipe = run_ensemble(reqs, opt, chunk=64, threads=8, rtol=RTOL)
        rec["pipelined_end_to_end"] = {"cells_per_s": pipe["cells_per_s"], "makespan_s": pipe["makespan_s"],
                                       "all_converged": pipe["all_converged"], "chunk": 64, "host_threads": 8}
        reqs = ensemble_batch(args.ensemble_members, seed=0)
        sv = Server(slots=8, options=opt, rtol=RTOL, dynamic=False).run(reqs, realtime=False)
        out[prec] = {"batched": rec,
                     "eight_slots": {"cells_per_s": sv["cells_per_s"], "makespan_s": sv["makespan_s"],
                                     "all_converged": sv["all_converged"], "max_relres": sv["max_relres"]}}
    err = [float(np.abs(m - f).max() / np.abs(f).max()) for m, f in zip(sols["mixed"], sols["fp64"])]
    out["mixed_vs_fp64_error"] = {"max": max(err), "median": float(np.median(err)),
                                  "per_solve": [float(f"{e:.3e}") for e in err]}
    out["members"] = args.ensemble_members
    out["cells"] = int(cells)
    return out


def _template_text(text, name):
    """Text of the template `name` in a source: from the template line
    before its definition to the closing brace at column 0 (None if absent)."""
    k = text.find(f" void {name}(")
    if k < 0:
        return None
    start = text.rfind("template", 0, k)
    end = text.find("\n}\n", k)
    if start < 0 or end < 0:
        return None
    return text[start:end + 3]


def kernel_source_hash(path, name):
    """sha256 of the text of the kernel template `name` in `path` and of the
    device body it runs (`name` without its k_ prefix, + `_body`), if any."""
    text = open(path).read()
    kern = _template_text(text, name)
    if kern is None:
        return None
    body = _template_text(text, name[2:] + "_body") if name.startswith("k_") else None
    return hashlib.sha256(((body or "") + kern).encode()).hexdigest()


def traffic_record(kernel, precision):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2001_01624_amd", "csrc", rec.get("source", "k_sweep.hip"))
    if not os.path.exists(src):
        return None
    if kernel_source_hash(src, rec.get("function", "k_sweep")) != rec.get("sha256"):
        return None
    return rec.get("bytes_per_launch")


def cpu_leg(smoother):
    """The oracle, as it stands, on a bounded sample of the same request
    (same recipe and block shapes at 30 x 110 x 21 cells): basis, three
    solves, dynamic stage, fluxes.  Single thread."""
    import oracle as O

    prob, sources = workload(dims=(30, 110, 21))
    parts = [{"kind": "cartesian", "coarse_dims": (5, 5, 1)}, {"kind": "cartesian", "coarse_dims": (3, 11, 4)}]
    t0 = time.perf_counter()
    o = O.Oracle(prob, parts, smoother=smoother)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.update_basis(100, 1e-3)
    x1, i1, r1, s1 = o.solve_gmres(source=sources[0], rtol=RTOL, restart=RESTART, max_iters=3000)
    x2, i2, r2, s2 = o.solve_gmres(source=sources[1], x0=x1, rtol=RTOL, restart=RESTART, max_iters=3000)
    o.add_dynamic_basis([x2 - x1])
    x3, i3, r3, s3 = o.solve_gmres(source=sources[2], x0=x2, rtol=RTOL, restart=RESTART, max_iters=3000)
    o.fluxes(x3)
    t = time.perf_counter() - t0
    print(json.dumps({"value": 3 * prob.n_active / t, "seconds": t, "setup_s": setup, "cells": prob.n_active,
                      "iters": [i1, i2, i3]}))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Cores this process may use: the affinity mask, capped by
    OMP_NUM_THREADS where the host sets a share."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = os.environ.get("OMP_NUM_THREADS")
    if share and share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return max(1, n)


def run_cpu_baseline(smoother):
    """The oracle leg on one thread, then on every host core: as many
    single-threaded oracle processes as cores, each solving the same sample
    request, started together (throughput = their cells over the wall time
    from the first start to the last finish)."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "--smoother", smoother]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    one = json.loads(r.stdout.strip().splitlines()[-1])
    cores = host_cores()
    t0 = time.perf_counter()
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
             for _ in range(cores)]
    outs = [p.communicate(timeout=1800) for p in procs]
    wall = time.perf_counter() - t0
    if any(p.returncode != 0 for p in procs):
        return {"error": next(o[1][-500:] for p, o in zip(procs, outs) if p.returncode != 0)}
    recs = [json.loads(o[0].strip().splitlines()[-1]) for o in outs]
    # each process's own timed region (setup excluded) bounds the wall time used for the rate
    span = max(rec["seconds"] for rec in recs)
    allc = sum(3 * rec["cells"] for rec in recs) / span
    return {"value": allc, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"same request recipe at 30x110x21 ({one['cells']} cells, general blocks 6x22x21 and "
                      f"~10x10x5): basis + 3 GMRES solves + dynamic stage + fluxes; {cores} single-threaded oracle "
                      f"processes at once, one request each (slowest {span:.1f} s, all {wall:.1f} s with oracle "
                      f"set-up); one thread alone: {one['seconds']:.1f} s; host {_cpu_model()}, "
                      f"{os.cpu_count()} hardware threads",
            "one_thread": {"value": one["value"], "cores": 1, "seconds": one["seconds"]},
            "iters": one["iters"]}


def main():
    args = parse()
    if args.cpu_leg:
        cpu_leg(args.smoother)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver path is single-GPU "
              f"and no multi-GPU run is built", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X", file=sys.stderr)
        sys.exit(1)
    if args.faulted_only:
        rec = faulted_leg(args)
        print(json.dumps({"leg": "faulted", "metric": METRIC, **rec}))
        return
    if args.ensemble_batch_only:
        rec = ensemble_leg(args)
        print(json.dumps({"leg": "ensemble_batch", **rec}))
        return
    if args.extras_only:
        for name, fn, skip in (("static", static_leg, args.no_static), ("fv", fv_leg, args.no_fv),
                               ("twophase", twophase_leg, args.no_twophase),
                               ("ensemble", ensemble_leg, args.no_ensemble)):
            if not skip:
                t = time.perf_counter()
                rec = fn(args)
                print(json.dumps({"leg": name, **rec, "leg_s": round(time.perf_counter() - t, 1)}), flush=True)
        return
    if args.mixed_only:
        rec = gpu_leg(args, "mixed")
        print(json.dumps({"leg": "mixed", "metric": METRIC, "value": rec["value"], "unit": "cells/s",
                          "ms_per_step": rec["ms_per_step"], "iters": rec["iters"], "max_relres": rec["relres"],
                          "roofline": rec["roofline"]}))
        return
    def leg(name, fn, *a):
        t = time.perf_counter()
        out = fn(*a)
        print(f"[bench] {name} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
        return out

    f64 = leg("fp64 request", gpu_leg, args, "fp64")
    mixed = None if args.no_mixed else leg("mixed request", gpu_leg, args, "mixed")
    faulted = None if args.no_faulted else leg("faulted request", faulted_leg, args)
    served = None if args.no_serve else leg("serving stream", serve_leg, args)
    ensemble = None if (args.no_serve or args.no_ensemble) else leg("ensemble", ensemble_leg, args)
    static = None if args.no_static else leg("static stages", static_leg, args)
    fv = None if args.no_fv else leg("finite volume", fv_leg, args)
    two = None if args.no_twophase else leg("two-phase", twophase_leg, args)
    cpu = None if args.no_cpu_baseline else leg("oracle baseline", run_cpu_baseline, args.smoother)
    line = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "layered lognormal+channel five-spot 60x220x85 (20x10x2 cells); general stages "
                               "10x10x5 and 6x22x17 coarse blocks; MsRSB tol 1e-3 <= 100 sweeps; "
                               f"{SMOOTHER_NAMES[args.smoother]}; "
                               f"GMRES({RESTART}) with the multistage cycle; 3 solves per request (+1 dynamic stage)",
                   "cells": f64["cells"], "solves_per_step": 3, "rtol": RTOL},
        "p50_ms": f64["p50_ms"],
        "p99_ms": f64["p99_ms"],
        "setup_ms": f64["setup_ms"],
        "iters": f64["iters"],
        "sweeps": f64["sweeps"],
        "dyn_blocks": f64["dyn_blocks"],
        "max_relres": f64["relres"],
        "all_converged": f64["all_converged"],
        "roofline": f64["roofline"],
        "cpu_baseline": cpu,
    }
    if mixed is not None:
        line["mixed"] = {"value": mixed["value"], "ms_per_step": mixed["ms_per_step"], "p50_ms": mixed["p50_ms"],
                         "p99_ms": mixed["p99_ms"], "iters": mixed["iters"], "sweeps": mixed["sweeps"],
                         "max_relres": mixed["relres"], "all_converged": mixed["all_converged"],
                         "roofline": mixed["roofline"], "kernel_table": mixed["kernel_table"],
                         "dtype": "f32 sweeps/smoother, bf16 basis, f64 residual"}
    line["kernel_table"] = f64["kernel_table"]
    if faulted is not None:
        line["faulted"] = faulted
    if served is not None:
        line["served"] = served
    if ensemble is not None:
        line["ensemble"] = ensemble
    if static is not None:
        line["static_stages"] = static
    if fv is not None:
        line["finite_volume"] = fv
    if two is not None:
        line["two_phase"] = two
    line["host"] = platform.node()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
