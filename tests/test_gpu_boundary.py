"""C-ABI boundary through the GPU library: contexts whose device memory comes
from PyTorch's caching allocator (msrsb_allocator); transmissibility updates
with local basis updates in msrsb_update_basis (the subsection "Iterative
multiscale multibasis solver": bases brought up to date for changed
properties by a few extra smoothing iterations) against the oracle at fixed
sweep counts: basis entries 1e-12, coarse operators 1e-12 relative, solves
to the tolerance on the oracle's residual of the new operator; and the
asynchronous solve (msrsb_solve_async) against the synchronous Richardson
solve, bit for bit."""
import numpy as np
import pytest

import oracle as O
from workloads import make_config1, make_config2, pressure_increment_pair, rng_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def capi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi as c
    return c


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def scaled_trans(prob, factor):
    nx, ny, nz = prob.dims
    y = (np.arange(prob.n_cells) // nx) % ny
    band = (y >= ny // 3) & (y < ny // 2)
    return tuple(np.where(band, T * factor, T) for T in (prob.tx, prob.ty, prob.tz))


def _request(capi, prob, parts, allocator, precision):
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", outer="gmres", precision=precision),
                    allocator=allocator)
    g.update_basis(max_sweeps=30, tol=1e-3)
    x = torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda")
    its = [g.solve(x, rtol=1e-8, max_iters=500)[0]]
    dp = pressure_increment_pair(prob, rng_for(8, 2))
    g.add_dynamic_basis([dev(d) for d in dp])
    its.append(g.solve(x, source=dev(prob.source * 1.3), rtol=1e-8, max_iters=500)[0])
    ex = [g.export_stage(k) for k in range(g.num_stages())]
    out = host(x)
    return g, its, out, ex


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_torch_allocator_same_results(capi, precision):
    prob = make_config2(dims=(20, 26, 10), seed=5)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "fault_cut", "parent": 0}]
    say(f"torch allocator {precision}")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    g1, its1, x1, ex1 = _request(capi, prob, parts, "torch", precision)
    held = torch.cuda.memory_allocated() - before
    g2, its2, x2, ex2 = _request(capi, prob, parts, None, precision)
    assert held >= capi.footprint_bytes(prob, parts, g1.options) // 2  # the context lives in torch's pool
    assert its1 == its2 and np.array_equal(x1, x2)
    for a, b in zip(ex1, ex2):
        for key in ("block", "slot_block", "values", "Ac"):
            assert np.array_equal(a[key], b[key])
    g1.close()
    g2.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before <= 0  # every block returned


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_transmissibility_update_matches_oracle(capi, precision):
    prob = make_config1(dims=(16, 24, 8), seed=4)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)}, {"kind": "cartesian", "coarse_dims": (4, 4, 1)}]
    say(f"transmissibility update {precision}")
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", precision=precision))
    o = O.Oracle(prob, parts, smoother="ilu0_rb")
    g.update_basis(max_sweeps=12, tol=0.0)
    o.update_basis(max_sweeps=12, tol=0.0)
    dp = pressure_increment_pair(prob, rng_for(8, 3))[0]
    assert g.add_dynamic_basis([dev(dp)]) == o.add_dynamic_basis([dp])
    T = scaled_trans(prob, 20.0)
    # local update: stage 0 smoothed three more times with the new operator; stage 1 and the
    # dynamic stage keep their bases and get new coarse operators
    g.update_basis(stage=0, max_sweeps=3, tol=0.0, warm=True, new_trans=T)
    o.update_basis(stage=0, max_sweeps=3, tol=0.0, warm=True, new_trans=T)
    for k in range(3):
        e = g.export_stage(k)
        st = o.all_stages()[k]
        if precision == "fp64":
            assert np.abs(g.dense_basis(k) - o.export_basis(k)).max() <= 1e-12
            assert relerr(e["Ac"], st.Ac) <= 1e-12
        else:
            # the coarse operator is the Galerkin product of the stored BF16 basis with the new A
            import scipy.sparse as sp

            Pb = sp.csr_matrix(g.dense_basis(k)[o.cells])
            assert relerr(e["Ac"], O.galerkin(Pb, o.A)) <= 1e-12
    # the operator itself: residual of a vector against the oracle's new A
    v = rng_for(8, 4).standard_normal(prob.n_cells) * prob.active
    r = host(g.apply(capi.OP_RESIDUAL, dev(v)))
    assert relerr(r[o.cells], o.b - o.A @ v[o.cells]) <= 1e-13
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-8 if precision == "fp64" else 1e-6, max_iters=2000)
    assert rc == capi.OK
    true = np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b)
    assert true <= (1.0001e-8 if precision == "fp64" else 1.0001e-6)
    if precision == "fp64":
        xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=4)
        q = dev(np.zeros(prob.n_cells))
        g.solve(q, rtol=0.0, max_iters=4)
        assert relerr(host(q), xo) <= 1e-9
    g.close()


def test_transmissibility_update_all_stages_from_scratch(capi):
    prob = make_config2(dims=(14, 18, 8), seed=8)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)}, {"kind": "fault_cut", "parent": 0}]
    say("transmissibility update, all stages from the indicator")
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", outer="gmres"))
    o = O.Oracle(prob, parts, smoother="ilu0_rb")
    g.update_basis(max_sweeps=5, tol=0.0)
    T = scaled_trans(prob, 0.05)
    g.update_basis(max_sweeps=9, tol=0.0, new_trans=T)
    o.update_basis(max_sweeps=9, tol=0.0, new_trans=T)
    for k in (0, 1):
        assert np.abs(g.dense_basis(k) - o.export_basis(k)).max() <= 1e-12
        assert relerr(g.export_stage(k)["Ac"], o.stages[k].Ac) <= 1e-12
    # a rejected update leaves the context as it was
    bad = (T[0] * -1.0, T[1], T[2])
    with pytest.raises(capi.MsrsbError) as ei:
        g.update_basis(max_sweeps=1, tol=0.0, new_trans=bad)
    assert ei.value.code == capi.E_INVAL
    assert np.abs(g.dense_basis(0) - o.export_basis(0)).max() <= 1e-12
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=500)
    assert rc == capi.OK and np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b) <= 1.0001e-10
    g.close()


@pytest.mark.parametrize("outer", ["richardson", "gmres"])
@pytest.mark.parametrize("smoother", ["ilu0_rb", "ilu0_line"])
def test_solve_async_equals_richardson(capi, outer, smoother):
    # msrsb_solve_async enqueues every Richardson cycle at once; its iterates
    # are those of the synchronous Richardson solve bit for bit, also when the
    # context's outer option is GMRES
    prob = make_config1(dims=(20, 24, 8), seed=3)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "cartesian", "coarse_dims": (2, 2, 1)}]
    say(f"async solve, context outer {outer}, smoother {smoother}")
    ref = capi.Solver(prob, parts, capi.default_options(smoother=smoother, outer="richardson"))
    g = capi.Solver(prob, parts, capi.default_options(smoother=smoother, outer=outer))
    for s in (ref, g):
        s.update_basis(max_sweeps=20, tol=0.0)
    p1 = dev(np.zeros(prob.n_cells))
    it, rel, rc = ref.solve(p1, rtol=1e-6, max_iters=400)
    p2 = dev(np.zeros(prob.n_cells))
    res = g.solve_async(p2, rtol=1e-6, max_cycles=400)
    torch.cuda.synchronize()
    st, cyc, rr = g.read_result(res)
    say(f"  Richardson cycles {it}, relres {rel:.3e}; async {cyc}, {rr:.3e}")
    assert st == rc and cyc == it and rr == rel and (rc == capi.OK) == (rel <= 1e-6)
    assert torch.equal(p1, p2)
    # a new source and a cycle cap below the count needed: E_NOCONV, the same iterate
    q = prob.source.copy()
    q[prob.n_cells // 3] += 0.25
    p3, p4 = dev(np.zeros(prob.n_cells)), dev(np.zeros(prob.n_cells))
    it, rel, rc = ref.solve(p3, source=dev(q), rtol=1e-12, max_iters=3)
    res = g.solve_async(p4, source=dev(q), rtol=1e-12, max_cycles=3)
    torch.cuda.synchronize()
    st, cyc, rr = g.read_result(res)
    assert rc == capi.E_NOCONV and st == capi.E_NOCONV and cyc == it == 3 and rr == rel
    assert torch.equal(p3, p4)
    with pytest.raises(capi.MsrsbError) as ei:
        g.solve_async(p4, max_cycles=0)
    assert ei.value.code == capi.E_INVAL
    ref.close()
    g.close()
    h = capi.Solver(prob, parts)
    with pytest.raises(capi.MsrsbError) as ei:
        h.solve_async(p4)
    assert ei.value.code == capi.E_STATE
    h.close()
