// Ensemble batch: the C ABI of msrsb_batch_* and its lockstep drivers.  The
// members are independent contexts; every step of the basis construction and
// of the GMRES solve is one batched launch per kernel (per template key) over
// all members, built from the kernel bodies of the single-context path, with
// the member-wise stop rules of that path (device status flags, host reads at
// the same points), the Galerkin operators and coarse inverses included.
#include <algorithm>
#include <map>
#include <vector>

#include "batch.h"
#include "msrsb_internal.h"

namespace msrsb {

// Launch groups of one kernel from (member, grid, key) triples: members with
// the same key share a launch; their workgroup ranges follow member order.
struct GroupSpec {
    int m, grid, key;
    size_t lds;
};

static void make_groups(const std::vector<GroupSpec> &spec, std::vector<int32_t> &tab, Groups &out,
                        std::vector<std::pair<Groups *, std::vector<size_t>>> &fix) {
    std::map<int, std::vector<GroupSpec>> by;
    for (const GroupSpec &g : spec)
        if (g.grid > 0) by[g.key].push_back(g);  // members without work stay out
    std::vector<size_t> offs;
    for (auto &kv : by) {
        HGroup h;
        h.key = kv.first;
        h.g.n = (int)kv.second.size();
        const size_t o = tab.size();
        int total = 0;
        h.g.direct = 1;
        for (const GroupSpec &g : kv.second) {
            tab.push_back(total);
            total += g.grid;
            h.lds = std::max(h.lds, g.lds);
            if (g.grid != 1) h.g.direct = 0;
        }
        tab.push_back(total);
        for (const GroupSpec &g : kv.second) tab.push_back(g.m);
        h.g.total = total;
        out.push_back(h);
        offs.push_back(o);
    }
    fix.push_back({&out, offs});
}

static int check_member(const Ctx &c, const Ctx &c0, int k) {
    const Stage *s = c.stages.size() == 1 ? &c.stages[0] : nullptr;
    bool dyn = false;
    for (const Stage &d : c.dyn) dyn = dyn || d.M > 0;
    const char *why = nullptr;
    if (!s || s->kind != 0) why = "needs exactly one rectilinear partition";
    else if (dyn) why = "holds dynamic stages";
    else if (c.opt.outer != MSRSB_GMRES || c.opt.restart > kDcgsMax || c.opt.restart < 1)
        why = "needs the GMRES outer loop with restart <= 31";
    else if (c.opt.smoother != MSRSB_SMOOTH_ILU0_LINE || !lilu_reg_chunks(c.nz) || !c.lpack)
        why = "needs the z-line ILU(0) smoother with columns of at most 512 cells";
    else if (c.opt.precision != c0.opt.precision || c.opt.restart != c0.opt.restart || c.opt.omega != c0.opt.omega)
        why = "differs from member 0 in precision, restart or omega";
    else if (c.device != c0.device) why = "is on another device";
    if (why) {
        set_error("batch member %d %s", k, why);
        return MSRSB_E_INVAL;
    }
    return MSRSB_OK;
}

// the member's descriptor (basis pointers as of its current state)
static void fill_member(const Ctx &c, BMember &d) {
    const Stage &s = c.stages[0];
    const bool mixed = c.opt.precision == MSRSB_MIXED;
    d.g = Fine{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    d.cd = s.cart;
    d.M = s.M;
    d.Mp = s.Mp;
    d.ns = s.ns;
    d.wtx = mixed ? (const void *)c.tx32 : (const void *)c.tx;
    d.wty = mixed ? (const void *)c.ty32 : (const void *)c.ty;
    d.wtz = mixed ? (const void *)c.tz32 : (const void *)c.tz;
    d.P[0] = mixed ? (void *)s.P32[0] : (void *)s.P64[0];
    d.P[1] = mixed ? (void *)s.P32[1] : (void *)s.P64[1];
    d.cur = s.cur;
    d.Pt = mixed ? (const void *)s.Pbf : (const void *)s.P64[s.cur];
    d.Pbf = s.Pbf;
    d.rpart = s.rpart;
    d.dvec = s.dvec;
    d.pc = s.pc;
    d.pc_map = s.pc_map;
    d.Ac = s.Ac;
    d.Ainv = s.Ainv;
    d.rap_part = s.rap_part;
    d.cbuf = c.cbuf;
    d.cbuf_n = c.cbuf_n;
    d.bcrhs = c.bcrhs;
    d.b = c.b;
    d.src = c.src;
    d.r = c.r;
    d.tmp = c.tmp;
    d.V = c.V;
    d.Z = c.Z;
    d.Vf = c.Vf;
    d.partial = c.partial;
    d.scal = c.scal;
    d.status = c.status;
    d.maxbits = c.maxbits;
    d.flag = c.flag;
}

static int upload_members(Batch &B) {
    hipError_t e = hipMemcpyAsync(B.d_mem, B.h_mem.data(), sizeof(BMember) * B.n, hipMemcpyHostToDevice, B.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
    return e == hipSuccess ? MSRSB_OK : hip_fail(e, "batch member table");
}

static int set_active(Batch &B) {
    hipError_t e = hipMemcpyAsync(B.d_act, B.h_act, sizeof(int) * B.n, hipMemcpyHostToDevice, B.stream);
    return e == hipSuccess ? MSRSB_OK : hip_fail(e, "batch member mask");
}

// statuses and error flags of the members still taking part, to the host
static int read_statuses(Batch &B) {
    bat_gather_status(B);
    hipError_t e = hipMemcpyAsync(B.h_st, B.d_st, sizeof(Status) * B.n, hipMemcpyDeviceToHost, B.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B.h_flag, B.d_flag, sizeof(int) * B.n, hipMemcpyDeviceToHost, B.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? MSRSB_OK : hip_fail(e, "batch status");
}

__global__ void k_clear_flag_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    D[m].flag[0] = 0;
}

static void free_tables(Batch *B) {
    (void)hipFree(B->d_mem);
    (void)hipFree(B->d_act);
    (void)hipFree(B->d_st);
    (void)hipFree(B->d_flag);
    (void)hipFree(B->d_tab);
    (void)hipHostFree(B->h_act);
    (void)hipHostFree(B->h_st);
    (void)hipHostFree(B->h_flag);
}

}  // namespace msrsb

using namespace msrsb;

struct msrsb_batch : public Batch {};

static void free_batch(msrsb_batch *B) {
    if (!B) return;
    free_tables(B);
    delete B;
}

extern "C" {

int msrsb_batch_create(int n, msrsb_ctx *const *members, void *hip_stream, msrsb_batch **out) {
    clear_error();
    if (!out || !members || n < 1 || n > 65536) {
        set_error("bad batch arguments");
        return MSRSB_E_INVAL;
    }
    *out = nullptr;
    std::vector<Ctx *> mem(n);
    for (int k = 0; k < n; ++k) {
        if (!members[k]) {
            set_error("batch member %d is NULL", k);
            return MSRSB_E_INVAL;
        }
        mem[k] = members[k];
    }
    {
        std::vector<Ctx *> sorted(mem);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
            set_error("a context appears twice in the batch");
            return MSRSB_E_INVAL;
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipGetLastError(), "batch device");
    for (int k = 0; k < n; ++k) {
        int rc = check_member(*mem[k], *mem[0], k);
        if (rc) return rc;
        if (mem[k]->device != dev) {
            set_error("batch member %d is not on the current device", k);
            return MSRSB_E_INVAL;
        }
    }
    msrsb_batch *B = new msrsb_batch();
    B->stream = (hipStream_t)hip_stream;
    B->device = dev;
    B->n = n;
    B->mixed = mem[0]->opt.precision == MSRSB_MIXED;
    B->restart = mem[0]->opt.restart;
    B->mem = mem;
    B->h_mem.resize(n);
    int rc = MSRSB_OK;
    std::vector<hipStream_t> old(n);  // restored if the batch is not made
    for (int k = 0; k < n; ++k) old[k] = mem[k]->stream;
    for (int k = 0; k < n && !rc; ++k) {
        Ctx &c = *mem[k];
        if (c.stream != B->stream) {
            hipError_t e = hipStreamSynchronize(c.stream);
            if (e != hipSuccess) rc = hip_fail(e, "member stream");
            else c.stream = B->stream;
        }
    }
    // launch groups
    std::vector<GroupSpec> one, cells, red, passa, nofuse, lilu, rrows, gather, gemv, prolong, sweep, init, bf16;
    std::vector<GroupSpec> rapbox, rapgather, pad, gjcopy, gjpanel, gjupdate;
    for (int k = 0; k < n && !rc; ++k) {
        const Ctx &c = *mem[k];
        const Stage &s = c.stages[0];
        BMember &d = B->h_mem[k];
        fill_member(c, d);
        const bool fuse = bat_member_fine(c, d);
        one.push_back({k, 1, 0, 0});
        cells.push_back({k, cdiv(c.N, kBlock), 0, 0});
        red.push_back({k, d.G, 0, 0});
        passa.push_back({k, d.GA, 0, 0});
        if (!fuse) nofuse.push_back({k, 1, 0, 0});
        const int gl = bat_member_lilu(c, d);
        lilu.push_back({k, gl, 0, 0});
        int tg[3], tk[3];
        size_t lds = 0;
        bat_member_transfer(c, s, tg, tk, &lds);
        rrows.push_back({k, tg[0], tk[0], lds});
        gather.push_back({k, tg[1], tk[1], 0});
        prolong.push_back({k, tg[2], tk[2], 0});
        int gk = 0;
        const int gg = bat_member_gemv(s, &gk);
        gemv.push_back({k, gg, gk, 0});
        int sk = 0;
        const int sg = bat_member_sweep(c, s, d, &sk);
        sweep.push_back({k, sg, sk, 0});
        const int nsk = s.ns <= 1 ? 1 : (s.ns <= 2 ? 2 : (s.ns <= 4 ? 4 : 8));
        init.push_back({k, cdiv(c.N, kBlock), nsk, 0});
        if (B->mixed) bf16.push_back({k, cdiv((long)s.ns * c.N, kBlock), 0, 0});
        int rg[3], rk = 0, ig[3];
        bat_member_rap(s, rg, &rk);
        rapbox.push_back({k, rg[0], rk, 0});
        rapgather.push_back({k, rg[1], rk, 0});
        pad.push_back({k, rg[2], 0, 0});
        bat_member_inverse(s, ig);
        gjcopy.push_back({k, ig[0], 0, 0});
        gjpanel.push_back({k, ig[1], 0, 0});
        gjupdate.push_back({k, ig[2], 0, 0});
        B->max_tiles = std::max(B->max_tiles, ig[1]);
    }
    std::vector<int32_t> tab;
    std::vector<std::pair<Groups *, std::vector<size_t>>> fix;
    make_groups(one, tab, B->one, fix);
    make_groups(cells, tab, B->cells, fix);
    make_groups(red, tab, B->red, fix);
    make_groups(passa, tab, B->passa, fix);
    make_groups(nofuse, tab, B->nofuse, fix);
    make_groups(lilu, tab, B->lilu, fix);
    make_groups(rrows, tab, B->rrows, fix);
    make_groups(gather, tab, B->gather, fix);
    make_groups(gemv, tab, B->gemv, fix);
    make_groups(prolong, tab, B->prolong, fix);
    make_groups(sweep, tab, B->sweep, fix);
    make_groups(init, tab, B->init, fix);
    make_groups(bf16, tab, B->bf16, fix);
    make_groups(rapbox, tab, B->rapbox, fix);
    make_groups(rapgather, tab, B->rapgather, fix);
    make_groups(pad, tab, B->pad, fix);
    make_groups(gjcopy, tab, B->gjcopy, fix);
    make_groups(gjpanel, tab, B->gjpanel, fix);
    make_groups(gjupdate, tab, B->gjupdate, fix);
    for (const HGroup &h : B->rrows)
        if (h.lds > 65536) {
            set_error("batch rows too long for the restriction's LDS");
            rc = MSRSB_E_INVAL;
        }
    hipError_t e = hipSuccess;
    if (!rc) {
        e = hipMalloc((void **)&B->d_mem, sizeof(BMember) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&B->d_act, sizeof(int) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&B->d_st, sizeof(Status) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&B->d_flag, sizeof(int) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&B->d_tab, sizeof(int32_t) * std::max<size_t>(tab.size(), 1));
        if (e == hipSuccess) e = hipHostMalloc((void **)&B->h_act, sizeof(int) * n);
        if (e == hipSuccess) e = hipHostMalloc((void **)&B->h_st, sizeof(Status) * n);
        if (e == hipSuccess) e = hipHostMalloc((void **)&B->h_flag, sizeof(int) * n);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B->d_tab, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice, B->stream);
        if (e != hipSuccess) rc = hip_fail(e, "batch tables");
    }
    if (!rc) {
        for (auto &f : fix)
            for (size_t q = 0; q < f.first->size(); ++q) {
                HGroup &h = (*f.first)[q];
                h.g.start = B->d_tab + f.second[q];
                h.g.mem = h.g.start + h.g.n + 1;
            }
        for (int k = 0; k < n; ++k) B->h_act[k] = 1;
        B->has_basis = true;
        for (int k = 0; k < n; ++k) B->has_basis = B->has_basis && mem[k]->stages[0].has_basis;
        rc = set_active(*B);
        if (!rc) rc = upload_members(*B);
    }
    if (rc) {
        (void)hipStreamSynchronize(B->stream);
        for (int k = 0; k < n; ++k) mem[k]->stream = old[k];
        free_batch(B);
        return rc;
    }
    *out = B;
    return MSRSB_OK;
}

int msrsb_batch_update_basis(msrsb_batch *B, int max_sweeps, double tol, int32_t *sweeps) {
    clear_error();
    if (!B || max_sweeps < 0 || max_sweeps > 65536 || !(tol >= 0.0)) {
        set_error("bad batch basis arguments");
        return MSRSB_E_INVAL;
    }
    const int n = B->n;
    int rc;
    for (int k = 0; k < n; ++k) B->h_act[k] = 1;
    if ((rc = set_active(*B))) return rc;
    bat_sweep_begin(*B, max_sweeps);
    if (max_sweeps > 0) {
        int k = 0, chunk = 8;
        while (k < max_sweeps) {
            const int kend = std::min(max_sweeps, k + chunk);
            while (k < kend) {
                const int npair = k + 1 < kend ? 2 : 1;
                bat_sweep_pair(*B, k, npair, B->mem[0]->opt.omega, tol, max_sweeps);
                k += npair;
            }
            if ((rc = read_statuses(*B))) return rc;
            bool all = true;
            for (int m = 0; m < n; ++m) all = all && B->h_st[m].done;
            if (all) break;
            chunk = std::min(chunk * 2, 64);
        }
    } else {
        if ((rc = read_statuses(*B))) return rc;
    }
    for (int m = 0; m < n; ++m)
        if (max_sweeps > 0 && (B->h_flag[m] & 2)) {
            set_error("batch member %d: basis row sum not positive", m);
            return MSRSB_E_SINGULAR;
        }
    for (int m = 0; m < n; ++m) {
        Ctx &c = *B->mem[m];
        Stage &s = c.stages[0];
        const int done = max_sweeps > 0 ? B->h_st[m].iters : 0;
        s.cur = done & 1;
        s.sweeps = done;
        s.change = max_sweeps > 0 ? B->h_st[m].relres : nan("");
        if (sweeps) sweeps[m] = done;
        fill_member(c, B->h_mem[m]);
    }
    if ((rc = upload_members(*B))) return rc;
    if (B->mixed) bat_to_bf16(*B);
    // Galerkin operators and their inverses
    for (const HGroup &h : B->one)
        hipLaunchKernelGGL(k_clear_flag_b, dim3(h.g.total), dim3(1), 0, B->stream, B->d_mem, h.g, B->d_act);
    for (int m = 0; m < n; ++m) B->mem[m]->stages[0].version++;
    bat_rap(*B);
    bat_coarse_inverse(*B);
    if ((rc = read_statuses(*B))) return rc;
    for (int m = 0; m < n; ++m) {
        if (B->h_flag[m] & 1) {
            set_error("batch member %d: coarse operator is not symmetric positive definite", m);
            return MSRSB_E_SINGULAR;
        }
        B->mem[m]->stages[0].has_basis = true;
    }
    B->has_basis = true;
    return MSRSB_OK;
}

int msrsb_batch_solve(msrsb_batch *B, const double *const *d_source, double *const *d_p, double rtol, int max_iters,
                      int32_t *iters, double *relres, int32_t *status) {
    clear_error();
    if (!B || !d_p || !(rtol >= 0.0) || max_iters < 0) {
        set_error("bad batch solve arguments");
        return MSRSB_E_INVAL;
    }
    const int n = B->n;
    for (int m = 0; m < n; ++m)
        if (!d_p[m]) {
            set_error("batch member %d has no solution vector", m);
            return MSRSB_E_INVAL;
        }
    if (!B->has_basis) {
        set_error("batch solve called before msrsb_batch_update_basis");
        return MSRSB_E_STATE;
    }
    int rc;
    for (int m = 0; m < n; ++m) {
        fill_member(*B->mem[m], B->h_mem[m]);
        B->h_mem[m].q = d_source ? d_source[m] : nullptr;
        B->h_mem[m].x = d_p[m];
        B->h_act[m] = 1;
    }
    if ((rc = upload_members(*B)) || (rc = set_active(*B))) return rc;
    if (d_source) bat_source_update(*B);
    bat_begin_solve(*B);
    const int mr = std::max(1, std::min(B->restart, kDcgsMax));
    for (;;) {
        // restart: true residual into V(0), the restart test
        bat_restart_residual(*B, rtol, max_iters);
        if ((rc = read_statuses(*B))) return rc;
        int live = 0;
        for (int m = 0; m < n; ++m) {
            if (B->h_act[m] && B->h_st[m].done) B->h_act[m] = 0;  // finished
            live += B->h_act[m];
        }
        if (!live) break;
        if ((rc = set_active(*B))) return rc;
        int j = 0, chunk = 4;
        bool all_done = false;
        while (j < mr) {
            const int jend = std::min(mr, j + chunk);
            for (; j < jend; ++j) {
                const int u = bvsel(BV_U, j), z = bvsel(BV_Z, j);
                // one multistage cycle from zero: z_j = M^-1 u_j
                bat_lilu_assign(*B, u, z);
                bat_residual_restrict(*B, u, z);
                bat_coarse_solve(*B);
                bat_prolong(*B, z);
                bat_dgmres_step(*B, j, rtol, max_iters, false);
            }
            if ((rc = read_statuses(*B))) return rc;
            all_done = true;
            for (int m = 0; m < n; ++m) all_done = all_done && (!B->h_act[m] || B->h_st[m].done);
            if (all_done) break;
            chunk = std::min(chunk * 2, 16);
        }
        // members that ran all mr steps finalise column mr (done ones skip)
        if (j == mr && !all_done) bat_dgmres_step(*B, mr, rtol, max_iters, true);
        bat_solution_update(*B);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch solve kernels");
    int bad = 0;
    for (int m = 0; m < n; ++m) {
        const Status &st = B->h_st[m];
        const int ok = st.relres <= rtol ? MSRSB_OK : MSRSB_E_NOCONV;
        if (iters) iters[m] = st.iters;
        if (relres) relres[m] = st.relres;
        if (status) status[m] = ok;
        if (ok != MSRSB_OK && !bad) {
            bad = 1;
            set_error("batch member %d: tolerance %g not met after %d iterations (relative residual %g)", m, rtol,
                      st.iters, st.relres);
        }
    }
    return bad ? MSRSB_E_NOCONV : MSRSB_OK;
}

void msrsb_batch_destroy(msrsb_batch *B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    free_batch(B);
}

}  // extern "C"
