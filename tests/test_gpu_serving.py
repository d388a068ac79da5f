"""Continuous-batching serving loop on the GPU: a request's results are the
same alone and in the mix, admission respects the HBM budget, oversized
requests are rejected without blocking the rest, and every solve meets the
tolerance on the FP64 residual recomputed by the oracle."""
import numpy as np
import pytest

import oracle as O
from workloads import make_config1, make_lognormal_box, rng_for
from workloads.requests import Request, source_sequence

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi, serve
    return capi, serve


def small_requests(n=6, seed=0, min_sources=1):
    rng = rng_for(6, seed)
    models = [make_lognormal_box((24, 20, 8), rng_for(6, 100 + k), sigma=2.0, corr=(2, 2, 2)) for k in range(3)]
    big = make_config1(dims=(20, 36, 14), seed=seed)
    reqs = []
    t = 0.0
    for r in range(n):
        t += rng.exponential(0.002)
        if r % 3 == 2:
            prob, parts, kind = big, [{"kind": "cartesian", "coarse_dims": (4, 3, 2)}], "large"
        else:
            prob, parts, kind = models[r % 3], [{"kind": "cartesian", "coarse_dims": (4, 4, 2)}], "small"
        k = max(min_sources, int(rng.integers(1, 5)))
        reqs.append(Request(r, t, prob, parts, source_sequence(prob, rng, k), kind))
    return reqs


@pytest.mark.parametrize("precision,slots,smoother", [("fp64", 4, "ilu0_rb"), ("fp64", 8, "ilu0_rb"),
                                                      ("mixed", 8, "ilu0_rb"), ("mixed", 8, "ilu0_line")])
def test_alone_equals_mixed(mods, precision, slots, smoother):
    # each request alone on one slot, then all of them at once on `slots`
    # slots: every request has at least three solves, so its last solves run
    # with dynamic stages built from its own increments; every reduction has a
    # fixed order, so each solution is bit for bit the same in the mix
    capi, serve = mods
    a, b = small_requests(n=10, min_sources=3), small_requests(n=10, min_sources=3)
    opt = capi.default_options(smoother=smoother, outer="gmres", precision=precision)
    print(precision, slots, smoother, "requests", [(r.kind, len(r.sources)) for r in a], flush=True)
    serve.Server(slots=1, options=opt, keep_solutions=True).run(a, realtime=False)
    st = serve.Server(slots=slots, options=opt, keep_solutions=True).run(b, realtime=False)
    assert st["completed"] == len(b) and st["all_converged"]
    assert all(len(r.dyn_blocks) >= 1 and all(c > 0 for c in r.dyn_blocks[-1]) for r in b)
    worst = 0.0
    for ra, rb in zip(a, b):
        assert ra.iters == rb.iters and ra.dyn_blocks == rb.dyn_blocks
        for xa, xb in zip(ra.solutions, rb.solutions):
            worst = max(worst, float(np.abs(xa - xb).max() / np.abs(xa).max()))
    print("alone vs mixed: max relative difference", worst, flush=True)
    assert worst == 0.0


def test_tolerance_on_fp64_residual(mods):
    capi, serve = mods
    reqs = small_requests(seed=1)
    st = serve.Server(slots=3, keep_solutions=True, rtol=1e-6).run(reqs, realtime=False)
    assert st["all_converged"]
    for r in reqs:
        o = O.Oracle(r.problem, r.partitions)
        for q, x, rel in zip(r.sources, r.solutions, r.relres):
            true = np.linalg.norm(o.residual(x, source=q)) / np.linalg.norm(O.msrsb.rhs_for(r.problem, o.cells, q))
            assert 0.0 < rel <= 1e-6 and true <= 1.0001e-6, (r.rid, rel, true)
    assert 0.0 < st["max_relres"] <= 1e-6


def test_admission_respects_budget(mods):
    capi, serve = mods
    reqs = small_requests(seed=2)
    opts = capi.default_options(smoother="ilu0_rb", outer="gmres")
    foot = {r.rid: serve.request_footprint(r, opts) for r in reqs}
    budget = max(foot.values()) + min(foot.values()) // 2
    st = serve.Server(slots=4, hbm_budget=budget, options=opts).run(reqs, realtime=False)
    assert st["completed"] == len(reqs)
    events = sorted([(r.admitted, foot[r.rid]) for r in reqs] + [(r.finished, -foot[r.rid]) for r in reqs],
                    key=lambda e: (e[0], e[1]))
    held = 0
    for _, f in events:
        held += f
        assert held <= budget


def test_oversized_request_is_rejected(mods):
    capi, serve = mods
    reqs = small_requests(seed=3)
    opts = capi.default_options(smoother="ilu0_rb", outer="gmres")
    foot = {r.rid: serve.request_footprint(r, opts) for r in reqs}
    small_max = max(f for rid, f in foot.items() if reqs[rid].kind == "small")
    st = serve.Server(slots=2, hbm_budget=small_max, options=opts).run(reqs, realtime=False)
    big = [r for r in reqs if foot[r.rid] > small_max]
    assert big and all(r.error for r in big)
    assert st["rejected"] == len(big) and st["completed"] == len(reqs) - len(big)
