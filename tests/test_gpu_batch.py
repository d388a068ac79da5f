"""Ensemble batch on the GPU: one launch per kernel over all members.

Each member's sweep count, GMRES iteration counts, residuals and solutions
are compared with the same member solved on its own context, bit for bit:
the batched kernels run the single-context kernel bodies on each member's own
grid, so any difference is a defect.  The members span the launch shapes the
batch groups by (rows of at most / more than 64 cells, coarse GEMV widths,
Arnoldi steps that do / do not sum their own partials, eight and four slots
per cell, odd x sizes, a single layer, inactive cells and dropped blocks).  The batch solutions also meet the tolerance on
the FP64 residual recomputed by the oracle."""
import numpy as np
import pytest

import oracle as O
from workloads import make_config1, make_config2, make_lognormal_box, rng_for
from workloads.requests import source_sequence

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def capi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi as c
    return c


def members():
    """(problem, coarse dims) pairs covering the batch's launch groups."""
    return [
        (make_lognormal_box((24, 20, 8), rng_for(7, 1), sigma=2.0, corr=(2, 2, 2)), (3, 3, 2)),
        (make_lognormal_box((70, 33, 12), rng_for(7, 2), sigma=2.0, corr=(3, 3, 3)), (8, 4, 3)),
        (make_lognormal_box((96, 96, 10), rng_for(7, 3), sigma=2.0, corr=(4, 4, 4)), (12, 12, 2)),
        (make_lognormal_box((33, 47, 16), rng_for(7, 4), sigma=2.0, corr=(2, 2, 2)), (4, 6, 4)),
        (make_config2(dims=(30, 44, 12), seed=3), (4, 5, 3)),
        (make_config1(dims=(20, 36, 14), seed=1), (4, 3, 2)),
        # four slots per cell: no split along z (3-D and a single layer)
        (make_lognormal_box((40, 30, 10), rng_for(7, 5), sigma=2.0, corr=(2, 2, 2)), (5, 3, 1)),
        (make_lognormal_box((48, 40, 1), rng_for(7, 6), sigma=2.0, corr=(2, 2, 1)), (6, 5, 1)),
    ]


def sources_for(ms, k=2):
    out = []
    for i, (prob, _) in enumerate(ms):
        out.append(source_sequence(prob, rng_for(8, i), k))
    return out


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).to("cuda")


def alone(capi, ms, srcs, opt, rtol, max_iters, keep=(False, False)):
    """Each member on its own context: sweeps, then two solves (the second
    from the first solution; keep[1] = True solves it with the source kept)."""
    res = []
    for (prob, cd), qs in zip(ms, srcs):
        g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}], opt)
        sw, _ = g.update_basis(stage=0, max_sweeps=100, tol=1e-3)
        x = torch.zeros(g.N, dtype=torch.float64, device="cuda")
        r = {"sweeps": sw, "it": [], "rel": [], "rc": [], "x": []}
        for q, kp in zip(qs, keep):
            it, rel, rc = g.solve(x, source=None if kp else dev(q), rtol=rtol, max_iters=max_iters)
            torch.cuda.synchronize()
            r["it"].append(it)
            r["rel"].append(rel)
            r["rc"].append(rc)
            r["x"].append(x.clone())
        g.close()
        res.append(r)
    return res


def batched(capi, ms, srcs, opt, rtol, max_iters, keep=(False, False)):
    gs = [capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}], opt) for prob, cd in ms]
    B = capi.Batch(gs)
    sw = B.update_basis(max_sweeps=100, tol=1e-3)
    xs = [torch.zeros(g.N, dtype=torch.float64, device="cuda") for g in gs]
    out = {"sweeps": sw, "it": [], "rel": [], "rc": [], "x": []}
    for s in range(len(srcs[0])):
        qs = [None if keep[s] else dev(q[s]) for q in srcs]
        it, rel, st = B.solve(xs, sources=None if keep[s] else qs, rtol=rtol, max_iters=max_iters)
        torch.cuda.synchronize()
        out["it"].append(it)
        out["rel"].append(rel)
        out["rc"].append(st)
        out["x"].append([x.clone() for x in xs])
    B.close()
    for g in gs:
        g.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone(capi, precision):
    ms = members()
    srcs = sources_for(ms)
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision=precision, restart=16)
    print("batch vs alone", precision, [p.dims for p, _ in ms], flush=True)
    a = alone(capi, ms, srcs, opt, 1e-6, 400)
    b = batched(capi, ms, srcs, opt, 1e-6, 400)
    assert b["sweeps"] == [r["sweeps"] for r in a]
    for s in range(2):
        for k, r in enumerate(a):
            assert r["rc"][s] == 0 and b["rc"][s][k] == 0
            assert b["it"][s][k] == r["it"][s], (s, k)
            assert b["rel"][s][k] == r["rel"][s], (s, k)
            assert torch.equal(b["x"][s][k], r["x"][s]), (s, k)
    print("iterations", b["it"], flush=True)


def test_batch_kept_source_and_iteration_cap(capi):
    # the second solve keeps each member's source (NULL array); a cap of 3
    # iterations stops every member short of the tolerance, as alone
    ms = members()[:4]
    srcs = sources_for(ms)
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision="fp64", restart=2)
    a = alone(capi, ms, srcs, opt, 1e-6, 3, keep=(False, True))
    b = batched(capi, ms, srcs, opt, 1e-6, 3, keep=(False, True))
    for s in range(2):
        for k, r in enumerate(a):
            assert r["rc"][s] == capi.E_NOCONV and b["rc"][s][k] == capi.E_NOCONV
            assert (b["it"][s][k], b["rel"][s][k]) == (r["it"][s], r["rel"][s]), (s, k)
            assert torch.equal(b["x"][s][k], r["x"][s]), (s, k)


def test_batch_meets_tolerance_on_oracle_residual(capi):
    ms = members()[:3] + members()[4:5]
    srcs = sources_for(ms, k=1)
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision="mixed", restart=16)
    b = batched(capi, ms, srcs, opt, 1e-6, 400, keep=(False,))
    for k, ((prob, cd), qs) in enumerate(zip(ms, srcs)):
        o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": cd}])
        x = b["x"][0][k].cpu().numpy()
        true = np.linalg.norm(o.residual(x, source=qs[0])) / np.linalg.norm(O.msrsb.rhs_for(prob, o.cells, qs[0]))
        assert 0.0 < b["rel"][0][k] <= 1e-6 and true <= 1.0001e-6, (k, b["rel"][0][k], true)


def test_batch_rejects(capi):
    ms = members()[:2]
    ok = capi.default_options(smoother="ilu0_line", outer="gmres")
    gs = [capi.Solver(p, [{"kind": "cartesian", "coarse_dims": cd}], ok) for p, cd in ms]
    with pytest.raises(capi.MsrsbError) as e:
        capi.Batch([gs[0], gs[0]])
    assert e.value.code == capi.E_INVAL
    B = capi.Batch(gs)
    xs = [torch.zeros(g.N, dtype=torch.float64, device="cuda") for g in gs]
    with pytest.raises(capi.MsrsbError) as e:
        B.solve(xs)
    assert e.value.code == capi.E_STATE
    B.close()
    prob, cd = ms[0]
    bad = [
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}], capi.default_options(smoother="jacobi",
                                                                                           outer="gmres")),
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}], capi.default_options(smoother="ilu0_line")),
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}, {"kind": "cartesian", "coarse_dims": (2, 2, 1)}],
                    ok),
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": cd}],
                    capi.default_options(smoother="ilu0_line", outer="gmres", precision="mixed")),
    ]
    for k, g in enumerate(bad):
        with pytest.raises(capi.MsrsbError) as e:
            capi.Batch([gs[1], g])
        assert e.value.code == capi.E_INVAL and "member 1" in str(e.value), k
    for g in gs + bad:
        g.close()


def test_pipelined_ensemble_equals_alone(capi):
    # batches of two members, set up and torn down on host threads while the
    # previous batch runs: every member's result is that of its own solve
    from paper_2001_01624_amd.serve import run_ensemble
    from workloads.requests import Request

    ms = members()[:5]
    srcs = sources_for(ms, k=1)
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision="mixed", restart=16)
    a = alone(capi, ms, srcs, opt, 1e-6, 400, keep=(False,))
    reqs = [Request(k, 0.0, p, [{"kind": "cartesian", "coarse_dims": cd}], [q[0]], "member")
            for k, ((p, cd), q) in enumerate(zip(ms, srcs))]
    st = run_ensemble(reqs, opt, chunk=2, threads=3, rtol=1e-6, max_iters=400, keep_solutions=True)
    assert st["all_converged"] and st["completed"] == len(ms)
    for r, ra in zip(reqs, a):
        assert r.iters == ra["it"] and r.relres == ra["rel"]
        assert np.array_equal(r.solutions[0], ra["x"][0].cpu().numpy()), r.rid


def test_batch_edge_cases(capi):
    # a batch of one member; no sweeps (the indicator basis); no iterations
    # (the initial residual only); then an ordinary solve: each as alone
    prob, cd = members()[3]
    q = source_sequence(prob, rng_for(8, 40), 1)[0]
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision="fp64", restart=16)
    parts = [{"kind": "cartesian", "coarse_dims": cd}]
    res = {}
    for mode in ("alone", "batch"):
        g = capi.Solver(prob, parts, opt)
        x = torch.zeros(g.N, dtype=torch.float64, device="cuda")
        out = []
        if mode == "alone":
            sw, _ = g.update_basis(stage=0, max_sweeps=0, tol=1e-3)
            out.append(g.solve(x, source=dev(q), rtol=1e-6, max_iters=0))
            out.append(g.solve(x, source=None, rtol=1e-6, max_iters=400))
        else:
            B = capi.Batch([g])
            sw = B.update_basis(max_sweeps=0, tol=1e-3)[0]
            it, rel, st = B.solve([x], sources=[dev(q)], rtol=1e-6, max_iters=0)
            out.append((it[0], rel[0], st[0]))
            it, rel, st = B.solve([x], rtol=1e-6, max_iters=400)
            out.append((it[0], rel[0], st[0]))
            B.close()
        torch.cuda.synchronize()
        res[mode] = (sw, out, x.clone())
        g.close()
    a, b = res["alone"], res["batch"]
    assert a[0] == b[0] == 0
    assert a[1] == b[1], (a[1], b[1])
    assert a[1][0][0] == 0 and a[1][0][2] == capi.E_NOCONV and a[1][1][2] == 0
    assert torch.equal(a[2], b[2])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ensemble_configuration_sampled(capi, precision):
    # the benchmark's ensemble configuration (members of 32..128 x 32..128 x
    # 8..16 cells, one 8x8x4 stage, GMRES(16), z-line ILU(0)) in one batch of
    # 32 members; four sampled members solved alone give the same sweeps,
    # iterations, residuals and solutions
    from workloads.requests import ensemble_batch

    reqs = ensemble_batch(32, seed=0)
    opt = capi.default_options(smoother="ilu0_line", outer="gmres", precision=precision, restart=16)
    gs = [capi.Solver(r.problem, r.partitions, opt) for r in reqs]
    B = capi.Batch(gs)
    sw = B.update_basis(max_sweeps=100, tol=1e-3)
    xs = [torch.zeros(g.N, dtype=torch.float64, device="cuda") for g in gs]
    it, rel, st = B.solve(xs, sources=[dev(r.sources[0]) for r in reqs], rtol=1e-6, max_iters=3000)
    torch.cuda.synchronize()
    B.close()
    assert all(s == 0 for s in st)
    for k in (0, 7, 15, 31):
        g = capi.Solver(reqs[k].problem, reqs[k].partitions, opt)
        swk, _ = g.update_basis(stage=0, max_sweeps=100, tol=1e-3)
        x = torch.zeros(g.N, dtype=torch.float64, device="cuda")
        itk, relk, rck = g.solve(x, source=dev(reqs[k].sources[0]), rtol=1e-6, max_iters=3000)
        torch.cuda.synchronize()
        assert (swk, itk, relk, rck) == (sw[k], it[k], rel[k], st[k]), k
        assert torch.equal(x, xs[k]), k
        g.close()
    for g in gs:
        g.close()
