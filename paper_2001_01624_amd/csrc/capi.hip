// Host side of the library: input validation, setup of the rectilinear
// partitions (integer tables, built once on the host and uploaded), the
// solver drivers and every extern "C" entry point of msrsb.h.
#include <algorithm>
#include <cfloat>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>

#include "dev_util.h"
#include "msrsb_internal.h"

static int finish_coarse(msrsb::Ctx &c, msrsb::Stage &s);

namespace msrsb {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

int hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MSRSB_E_NOMEM : MSRSB_E_DEVICE;
}

// Device memory comes from the device's stream-ordered pool, allocated and
// freed in the order of the context's stream: contexts created and destroyed
// while others run on their own streams never synchronise the device.  The
// pool keeps freed memory for reuse (release threshold raised once per
// device), so a served request does not return memory to the driver.
static void keep_pool_memory(int device) {
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> lock(mu);
    if (std::find(done.begin(), done.end(), device) != done.end()) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    done.push_back(device);
}

// One device allocation of the context: from the caller's allocator when one
// was given at setup, else from the device's stream-ordered pool.
static void *raw_alloc(Ctx &c, size_t bytes) {
    void *p = nullptr;
    if (c.ua.alloc) {
        p = c.ua.alloc(bytes, (void *)c.stream, c.ua.user);
        if (p && ((uintptr_t)p & 255)) {  // the arena carving assumes 256-byte alignment
            c.ua.free(p, bytes, (void *)c.stream, c.ua.user);
            set_error("the caller's allocator returned a pointer not aligned to 256 bytes");
            return nullptr;
        }
    } else {
        keep_pool_memory(c.device);
        if (hipMallocAsync(&p, bytes, c.stream) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    if (!p) {
        set_error("device allocation of %zu bytes failed", bytes);
        return nullptr;
    }
    c.allocs.push_back(p);
    c.alloc_bytes.push_back(bytes);
    return p;
}

static void raw_free(Ctx &c, void *p, size_t bytes) {
    if (c.ua.alloc) c.ua.free(p, bytes, (void *)c.stream, c.ua.user);
    else (void)hipFreeAsync(p, c.stream);
}

// Set-up arenas of destroyed contexts (pool memory only) are kept per device
// for the next set-ups: for contexts of a few MB the pool's own allocation
// and stream-ordered free cost 0.02-0.9 ms each, as much as the rest of the
// set-up.  At most kArenaCacheBytes per device are held (until the process
// ends); an arena is reused by a set-up that needs at least 3/4 of it.
constexpr size_t kArenaCacheBytes = (size_t)4 << 30;
struct CachedArena {
    int device;
    size_t bytes;
    void *p;
};
static std::mutex g_arena_mu;
static std::vector<CachedArena> g_arenas;

static void *arena_take(int device, size_t need, size_t *got) {
    std::lock_guard<std::mutex> lock(g_arena_mu);
    size_t best = g_arenas.size();
    for (size_t k = 0; k < g_arenas.size(); ++k) {
        const CachedArena &a = g_arenas[k];
        if (a.device == device && a.bytes >= need && a.bytes / 4 * 3 <= need &&
            (best == g_arenas.size() || a.bytes < g_arenas[best].bytes))
            best = k;
    }
    if (best == g_arenas.size()) return nullptr;
    void *p = g_arenas[best].p;
    *got = g_arenas[best].bytes;
    g_arenas.erase(g_arenas.begin() + best);
    return p;
}

// true: the cache keeps the (idle) arena
static bool arena_give(int device, void *p, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_arena_mu);
    size_t held = 0;
    for (const CachedArena &a : g_arenas)
        if (a.device == device) held += a.bytes;
    if (held + bytes > kArenaCacheBytes) return false;
    g_arenas.push_back({device, bytes, p});
    return true;
}

void *ctx_alloc(Ctx &c, size_t bytes) {
    if (bytes == 0) bytes = 8;
    const size_t rb = (bytes + 255) & ~(size_t)255;
    if (c.arena_open && c.arena && c.arena_off + rb <= c.arena_size) {
        void *p = c.arena + c.arena_off;
        c.arena_off += rb;
        return p;
    }
    return raw_alloc(c, bytes);
}

// Return a buffer of ctx_alloc in the stream's order.  Buffers carved from
// the set-up arena are left alone (the arena is freed whole).
void ctx_free(Ctx &c, void *p) {
    if (!p) return;
    auto it = std::find(c.allocs.begin(), c.allocs.end(), p);
    if (it == c.allocs.end()) return;
    const size_t k = it - c.allocs.begin();
    raw_free(c, p, c.alloc_bytes[k]);
    c.allocs.erase(it);
    c.alloc_bytes.erase(c.alloc_bytes.begin() + k);
}

// Host -> device copy on the context's stream (the caller keeps the host
// buffer alive until the stream is synchronised).
static bool upload(Ctx &c, void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream) == hipSuccess;
}

// Pinned status mirrors are recycled: freeing pinned memory can wait for the
// whole device.
static std::mutex g_pinned_mu;
static std::vector<Status *> g_pinned_free;

static Status *pinned_status() {
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            Status *p = g_pinned_free.back();
            g_pinned_free.pop_back();
            return p;
        }
    }
    Status *p = nullptr;
    if (hipHostMalloc((void **)&p, sizeof(Status), 0) != hipSuccess) return nullptr;
    return p;
}

static void release_pinned_status(Status *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_pinned_free.push_back(p);
}

// ------------------------------------------------------------ validation ----

// The basis kernels address a stage's slot-major arrays with 32-bit byte
// offsets (buffer resources of at most 2^31 - 1 bytes): ns slots of N cells
// in FP64 must stay below that.
static bool slots_fit(long ns, long N) { return ns * N * (long)sizeof(double) <= 0x7fffffffL; }


struct DSU {
    std::vector<int> p;
    explicit DSU(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int find(int a) {
        while (p[a] != a) a = p[a] = p[p[a]];
        return a;
    }
    void unite(int a, int b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

static int validate(const msrsb_grid *g) {
    if (!g) {
        set_error("grid is NULL");
        return MSRSB_E_INVAL;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || (long)g->nx * g->ny * g->nz > 0x7fffffffL / 8) {
        set_error("bad grid dimensions %d x %d x %d", g->nx, g->ny, g->nz);
        return MSRSB_E_INVAL;
    }
    if (!g->tx || !g->ty || !g->tz) {
        set_error("tx/ty/tz must be given");
        return MSRSB_E_INVAL;
    }
    const int nx = g->nx, ny = g->ny, nz = g->nz, N = nx * ny * nz, nxy = nx * ny;
    auto act = [&](int i) { return g->active ? g->active[i] != 0 : true; };
    const double *T[3] = {g->tx, g->ty, g->tz};
    const int step[3] = {1, nx, nxy};
    // One branch-light pass decides whether the per-cell checks below can find
    // anything, and whether the grid is a full box (every cell active, every
    // interior face with T > 0: one connected component).  Only a grid that
    // fails it is walked again by the checks that name the first error.
    bool bad = false, full = true;
    {
        const uint8_t *A = g->active;
        const double *X = g->tx, *Y = g->ty, *Z = g->tz, *Q = g->source;
        for (int z = 0, i = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x, ++i) {
                    const double t0 = X[i], t1 = Y[i], t2 = Z[i];
                    bad |= !(t0 >= 0.0 && t0 <= DBL_MAX) || !(t1 >= 0.0 && t1 <= DBL_MAX) ||
                           !(t2 >= 0.0 && t2 <= DBL_MAX);
                    if (Q) bad |= !std::isfinite(Q[i]);
                    const bool ai = A ? A[i] != 0 : true;
                    full &= ai;
                    if (x + 1 < nx) {
                        full &= t0 > 0.0;
                        bad |= t0 != 0.0 && !(ai && (A ? A[i + 1] != 0 : true));
                    } else {
                        bad |= t0 != 0.0;
                    }
                    if (y + 1 < ny) {
                        full &= t1 > 0.0;
                        bad |= t1 != 0.0 && !(ai && (A ? A[i + nx] != 0 : true));
                    } else {
                        bad |= t1 != 0.0;
                    }
                    if (z + 1 < nz) {
                        full &= t2 > 0.0;
                        bad |= t2 != 0.0 && !(ai && (A ? A[i + nxy] != 0 : true));
                    } else {
                        bad |= t2 != 0.0;
                    }
                }
    }
    // cells in index order (x fastest), coordinates carried by the loops
    for (int z = 0, i = 0; bad && z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x, ++i) {
                const int c[3] = {x, y, z};
                const int n[3] = {nx, ny, nz};
                for (int a = 0; a < 3; ++a) {
                    const double t = T[a][i];
                    if (!(t >= 0.0) || !std::isfinite(t)) {
                        set_error("transmissibility %c[%d] = %g is negative or not finite", "xyz"[a], i, t);
                        return MSRSB_E_INVAL;
                    }
                    if (t != 0.0) {
                        if (c[a] == n[a] - 1) {
                            set_error("face %c[%d] leaves the grid", "xyz"[a], i);
                            return MSRSB_E_INVAL;
                        }
                        if (!act(i) || !act(i + step[a])) {
                            set_error("face %c[%d] touches an inactive cell", "xyz"[a], i);
                            return MSRSB_E_INVAL;
                        }
                    }
                }
                if (g->source && !std::isfinite(g->source[i])) {
                    set_error("source[%d] not finite", i);
                    return MSRSB_E_INVAL;
                }
            }
    if (g->n_bc < 0 || (g->n_bc > 0 && (!g->bc_cell || !g->bc_trans || !g->bc_value))) {
        set_error("bad boundary-connection arrays");
        return MSRSB_E_INVAL;
    }
    for (int k = 0; k < g->n_bc; ++k) {
        const int i = g->bc_cell[k];
        if (i < 0 || i >= N || !act(i)) {
            set_error("boundary connection %d on a missing or inactive cell %d", k, i);
            return MSRSB_E_INVAL;
        }
        if (!(g->bc_trans[k] >= 0.0) || !std::isfinite(g->bc_trans[k]) || !std::isfinite(g->bc_value[k])) {
            set_error("boundary connection %d: transmissibility/value negative or not finite", k);
            return MSRSB_E_INVAL;
        }
    }
    // every active connected component needs a boundary/well connection:
    // breadth-first search over the faces with T > 0 from every cell with a
    // connection of positive T; the first active cell left unreached (in index
    // order) is reported.  A full box is one component: one connection of
    // positive T anchors it.
    if (full) {
        for (int k = 0; k < g->n_bc; ++k)
            if (g->bc_trans[k] > 0.0) return MSRSB_OK;
        set_error("active cell %d lies in a connected component without boundary or well connection", 0);
        return MSRSB_E_SINGULAR;
    }
    std::vector<uint8_t> seen(N, 0);
    std::vector<int> queue;
    queue.reserve(N);
    for (int k = 0; k < g->n_bc; ++k)
        if (g->bc_trans[k] > 0.0 && !seen[g->bc_cell[k]]) {
            seen[g->bc_cell[k]] = 1;
            queue.push_back(g->bc_cell[k]);
        }
    for (size_t h = 0; h < queue.size(); ++h) {
        const int i = queue[h];
        for (int a = 0; a < 3; ++a) {
            if (T[a][i] != 0.0 && !seen[i + step[a]]) {
                seen[i + step[a]] = 1;
                queue.push_back(i + step[a]);
            }
            if (i >= step[a] && T[a][i - step[a]] != 0.0 && !seen[i - step[a]]) {
                seen[i - step[a]] = 1;
                queue.push_back(i - step[a]);
            }
        }
    }
    for (int i = 0; i < N; ++i)
        if (act(i) && !seen[i]) {
            set_error("active cell %d lies in a connected component without boundary or well connection", i);
            return MSRSB_E_SINGULAR;
        }
    return MSRSB_OK;
}

// Per-axis tables of a rectilinear partition (see CartDev).
static void axis_tables(int n, int m, std::vector<int32_t> &lo, std::vector<int32_t> &nv, std::vector<int32_t> &slo,
                        std::vector<int32_t> &shi, std::vector<int32_t> &be) {
    be.resize(m + 1);
    for (int J = 0; J <= m; ++J) be[J] = (int32_t)(((long)J * n + m - 1) / m);  // ceil(J n / m)
    std::vector<long> c2(m);
    for (int J = 0; J < m; ++J) c2[J] = (long)be[J] + be[J + 1];
    lo.assign(n, 0);
    nv.assign(n, 1);
    slo.assign(m, n);
    shi.assign(m, -1);
    for (int i = 0; i < n; ++i) {
        const int blk = (int)(((long)i * m) / n);
        const long t = 2L * i + 1;
        if (blk > 0 && t < c2[blk]) {
            lo[i] = blk - 1;
            nv[i] = 2;
        } else if (blk < m - 1 && t > c2[blk]) {
            lo[i] = blk;
            nv[i] = 2;
        } else {
            lo[i] = blk;
            nv[i] = 1;
        }
        for (int J = lo[i]; J < lo[i] + nv[i]; ++J) {
            slo[J] = std::min(slo[J], i);
            shi[J] = std::max(shi[J], i);
        }
    }
}

static int build_cart_stage(Ctx &c, const msrsb_partition &p, Stage &s) {
    const int n[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a)
        if (p.coarse_dims[a] < 1 || p.coarse_dims[a] > n[a]) {
            set_error("coarse_dims[%d] = %d outside [1, %d]", a, p.coarse_dims[a], n[a]);
            return MSRSB_E_INVAL;
        }
    s.kind = 0;
    CartDev &cd = s.cart;
    int nbits = 0;
    for (int a = 0; a < 3; ++a) {
        cd.n[a] = n[a];
        cd.m[a] = p.coarse_dims[a];
        cd.bit[a] = cd.m[a] > 1 ? nbits++ : -1;
    }
    cd.ns = s.ns = 1 << nbits;
    std::vector<int32_t> tab;
    for (int a = 0; a < 3; ++a) {
        std::vector<int32_t> lo, nv, slo, shi, be;
        axis_tables(n[a], cd.m[a], lo, nv, slo, shi, be);
        s.tab_off[a][0] = (int)tab.size(); tab.insert(tab.end(), lo.begin(), lo.end());
        s.tab_off[a][1] = (int)tab.size(); tab.insert(tab.end(), nv.begin(), nv.end());
        s.tab_off[a][2] = (int)tab.size(); tab.insert(tab.end(), slo.begin(), slo.end());
        s.tab_off[a][3] = (int)tab.size(); tab.insert(tab.end(), shi.begin(), shi.end());
        s.tab_off[a][4] = (int)tab.size(); tab.insert(tab.end(), be.begin(), be.end());
        // split[J]: first cell of block J whose lo is J (cells before it have lo = J-1)
        std::vector<int32_t> split(cd.m[a]);
        for (int J = 0; J < cd.m[a]; ++J) {
            int sp = be[J + 1];
            for (int i = be[J]; i < be[J + 1]; ++i)
                if (lo[i] == J) {
                    sp = i;
                    break;
                }
            split[J] = sp;
        }
        s.tab_off[a][5] = (int)tab.size(); tab.insert(tab.end(), split.begin(), split.end());
        std::vector<int32_t> pack(n[a]);
        for (int i = 0; i < n[a]; ++i) {
            const int dm = i > 0 ? lo[i] - lo[i - 1] : 0, dp = i + 1 < n[a] ? lo[i + 1] - lo[i] : 0;
            pack[i] = lo[i] | ((nv[i] == 2) << 20) | (dm << 21) | (dp << 22);
        }
        s.tab_off[a][6] = (int)tab.size(); tab.insert(tab.end(), pack.begin(), pack.end());
    }
    // x-axis flags as 64-bit masks per run of 64 cells (bit j: cell 64 t + j):
    // [nv == 2, lo[c] - lo[c-1], lo[c+1] - lo[c]], read by scalar loads
    if (tab.size() & 1) tab.push_back(0);
    const int xmask_off = (int)tab.size();
    {
        const int nxt = cdiv(c.nx, 64);
        const int32_t *px = tab.data() + s.tab_off[0][6];
        std::vector<uint64_t> xm(3 * (size_t)nxt, 0);
        for (int i = 0; i < c.nx; ++i)
            for (int f = 0; f < 3; ++f)
                if ((px[i] >> (20 + f)) & 1) xm[3 * (i / 64) + f] |= 1ull << (i % 64);
        for (uint64_t v : xm) {
            tab.push_back((int32_t)(uint32_t)(v & 0xFFFFFFFFu));
            tab.push_back((int32_t)(uint32_t)(v >> 32));
        }
    }
    // blocks with active cells, compacted in Cartesian order; active cells per block
    const int M0 = cd.m[0] * cd.m[1] * cd.m[2];
    std::vector<int64_t> cnt(M0, 0);
    {
        // block of each coordinate per axis (floor(i m / n)); a full box has
        // the product of the block widths in every block
        std::vector<int32_t> bax[3];
        for (int a = 0; a < 3; ++a) {
            bax[a].resize(n[a]);
            for (int i = 0; i < n[a]; ++i) bax[a][i] = (int32_t)(((long)i * cd.m[a]) / n[a]);
        }
        if (c.n_active == c.N) {
            std::vector<int64_t> w[3];
            for (int a = 0; a < 3; ++a) {
                w[a].assign(cd.m[a], 0);
                for (int i = 0; i < n[a]; ++i) w[a][bax[a][i]]++;
            }
            for (int J2 = 0; J2 < cd.m[2]; ++J2)
                for (int J1 = 0; J1 < cd.m[1]; ++J1)
                    for (int J0 = 0; J0 < cd.m[0]; ++J0)
                        cnt[J0 + cd.m[0] * (J1 + cd.m[1] * J2)] = w[0][J0] * w[1][J1] * w[2][J2];
        } else {
            const uint8_t *act = c.h_active.data();
            for (int z = 0, i = 0; z < c.nz; ++z)
                for (int y = 0; y < c.ny; ++y) {
                    const int Jyz = cd.m[0] * (bax[1][y] + cd.m[1] * bax[2][z]);
                    for (int x = 0; x < c.nx; ++x, ++i)
                        if (act[i]) cnt[bax[0][x] + Jyz]++;
                }
        }
    }
    const int cmap_off = (int)tab.size();
    s.h_present.clear();
    for (int J = 0; J < M0; ++J) {
        tab.push_back(cnt[J] > 0 ? (int32_t)s.h_present.size() : -1);
        if (cnt[J] > 0) s.h_present.push_back(J);
    }
    const int pres_off = (int)tab.size();
    tab.insert(tab.end(), s.h_present.begin(), s.h_present.end());
    const int gbase_off = (int)tab.size();
    int64_t run = 0;
    for (int J = 0; J < M0; ++J) {
        tab.push_back((int32_t)run);
        run += cnt[J];
    }
    tab.push_back((int32_t)run);
    s.M = (int)s.h_present.size();
    s.Mp = cdiv(s.M, kTile) * kTile;
    s.h_tab = tab;
    s.d_tab = (int32_t *)ctx_alloc(c, sizeof(int32_t) * tab.size());
    if (!s.d_tab) return MSRSB_E_NOMEM;
    if (!upload(c, s.d_tab, s.h_tab.data(), sizeof(int32_t) * tab.size()))
        return hip_fail(hipGetLastError(), "upload tables");
    for (int a = 0; a < 3; ++a) {
        cd.lo[a] = s.d_tab + s.tab_off[a][0];
        cd.nv[a] = s.d_tab + s.tab_off[a][1];
        cd.slo[a] = s.d_tab + s.tab_off[a][2];
        cd.shi[a] = s.d_tab + s.tab_off[a][3];
        cd.be[a] = s.d_tab + s.tab_off[a][4];
        cd.split[a] = s.d_tab + s.tab_off[a][5];
        cd.pack[a] = s.d_tab + s.tab_off[a][6];
    }
    cd.xmask = (const uint64_t *)(s.d_tab + xmask_off);
    cd.cmap = s.d_tab + cmap_off;
    cd.present = s.d_tab + pres_off;
    s.gbase = s.d_tab + gbase_off;
    const size_t nsN = (size_t)s.ns * c.N;
    if (c.opt.precision == MSRSB_MIXED) {
        s.P32[0] = (float *)ctx_alloc(c, sizeof(float) * nsN);
        s.P32[1] = (float *)ctx_alloc(c, sizeof(float) * nsN);
        s.Pbf = (uint16_t *)ctx_alloc(c, sizeof(uint16_t) * nsN);
        if (!s.P32[0] || !s.P32[1] || !s.Pbf) return MSRSB_E_NOMEM;
    } else {
        s.P64[0] = (double *)ctx_alloc(c, sizeof(double) * nsN);
        s.P64[1] = (double *)ctx_alloc(c, sizeof(double) * nsN);
        if (!s.P64[0] || !s.P64[1]) return MSRSB_E_NOMEM;
    }
    s.Ac = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    s.Ainv = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    s.dvec = (double *)ctx_alloc(c, sizeof(double) * s.Mp);
    const size_t npc = std::max((size_t)s.Mp, (size_t)cd.m[0] * cd.m[1] * cd.m[2]);
    s.pc = (double *)ctx_alloc(c, sizeof(double) * npc);
    if (!s.Ac || !s.Ainv || !s.dvec || !s.pc) return MSRSB_E_NOMEM;
    if (hipMemsetAsync(s.pc, 0, sizeof(double) * npc, c.stream) != hipSuccess)
        return hip_fail(hipGetLastError(), "clear p_c");
    s.pc_map = cd.present;
    if (c.nx > 64 * 4) {
        set_error("rows longer than 256 cells are not supported by the restriction kernel");
        return MSRSB_E_INVAL;
    }
    if (cd.m[2] > 1024) {
        set_error("more than 1024 coarse blocks along z are not supported by the restriction kernel");
        return MSRSB_E_INVAL;
    }
    {
        // widest dual z-interval: cells of one layer range sharing lo (split to split)
        const int32_t *sp = s.h_tab.data() + s.tab_off[2][5];
        s.zwide = 0;
        for (int L = 0; L < cd.m[2]; ++L) {
            const int z0 = (cd.m[2] > 1 && L > 0) ? sp[L] : 0;
            const int z1 = (cd.m[2] > 1 && L + 1 < cd.m[2]) ? sp[L + 1] : c.nz;
            s.zwide = std::max(s.zwide, z1 - z0);
        }
    }
    s.rpart = (double *)ctx_alloc(c, sizeof(double) * (size_t)c.nz * cd.m[1] * cd.m[0] * s.ns);
    s.rap_part = (double *)ctx_alloc(c, sizeof(double) * rap_part_doubles(s.ns, cd.m[0] * cd.m[1] * cd.m[2]));
    if (!s.rpart || !s.rap_part) return MSRSB_E_NOMEM;
    return MSRSB_OK;
}

// Fault-cut stage: the pieces of every block of the (rectilinear) parent
// stage that stay connected without crossing a fault face, numbered by
// (parent block, smallest cell); the support of a piece is what a breadth-
// first search from it reaches inside the parent block's support box
// without crossing a fault face.  Integer work on the host.
static int explicit_stage_tables(Ctx &c, Stage &s, int M, const std::vector<std::vector<int>> &slots);

static int build_fault_stage(Ctx &c, const msrsb_partition &p, int index, Stage &s, const double *T3[3]) {
    if (p.parent < 0 || p.parent >= index || c.stages[p.parent].kind != 0) {
        set_error("FAULT_CUT partition %d: parent must be an earlier CARTESIAN partition", index);
        return MSRSB_E_INVAL;
    }
    const Stage &par = c.stages[p.parent];
    const int N = c.N, nx = c.nx, ny = c.ny, nz = c.nz, nxy = nx * ny;
    const int step[3] = {1, nx, nxy};
    const int32_t *pt = par.h_tab.data();
    const int cmap_off = (int)(par.cart.cmap - par.d_tab);
    auto pblk = [&](int i) -> int {
        if (!c.h_active[i]) return -1;
        const int cc[3] = {i % nx, (i / nx) % ny, i / nxy};
        int J[3];
        for (int a = 0; a < 3; ++a) J[a] = (int)(((long)cc[a] * par.cart.m[a]) / par.cart.n[a]);
        return pt[cmap_off + J[0] + par.cart.m[0] * (J[1] + par.cart.m[1] * J[2])];
    };
    std::vector<int32_t> pb(N);
    for (int i = 0; i < N; ++i) pb[i] = pblk(i);
    auto open = [&](int i, int a) {
        return T3[a][i] != 0.0 && !(c.h_fault.size() && c.h_fault[(size_t)a * N + i]);
    };
    DSU d(N);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < N; ++i)
            if (open(i, a) && pb[i] == pb[i + step[a]]) d.unite(i, i + step[a]);
    // pieces ordered by (parent block, smallest cell): the DSU root is the smallest cell
    std::vector<std::pair<int64_t, int>> keys;
    std::vector<int> root_id(N, -1);
    for (int i = 0; i < N; ++i)
        if (c.h_active[i] && d.find(i) == i) keys.push_back({(int64_t)pb[i] * N + i, i});
    std::sort(keys.begin(), keys.end());
    for (size_t k = 0; k < keys.size(); ++k) root_id[keys[k].second] = (int)k;
    const int M = (int)keys.size();
    s.h_xpblock.assign(N, -1);
    std::vector<std::vector<int>> members(M);
    for (int i = 0; i < N; ++i)
        if (c.h_active[i]) {
            const int j = root_id[d.find(i)];
            s.h_xpblock[i] = j;
            members[j].push_back(i);
        }
    // supports: BFS inside the parent's support box over open faces
    std::vector<std::vector<int>> slots(N);
    std::vector<int> stamp(N, -1), frontier, next;
    for (int j = 0; j < M; ++j) {
        const int J = pb[members[j][0]];
        const int cid = par.h_present[J];
        const int Jc[3] = {cid % par.cart.m[0], (cid / par.cart.m[0]) % par.cart.m[1],
                           cid / (par.cart.m[0] * par.cart.m[1])};
        int lo3[3], hi3[3];
        for (int a = 0; a < 3; ++a) {
            lo3[a] = pt[par.tab_off[a][2] + Jc[a]];
            hi3[a] = pt[par.tab_off[a][3] + Jc[a]];
        }
        auto inbox = [&](int i) {
            const int cc[3] = {i % nx, (i / nx) % ny, i / nxy};
            for (int a = 0; a < 3; ++a)
                if (cc[a] < lo3[a] || cc[a] > hi3[a]) return false;
            return c.h_active[i] != 0;
        };
        frontier = members[j];
        for (int i : frontier) stamp[i] = j;
        std::vector<int> reached = frontier;
        while (!frontier.empty()) {
            next.clear();
            for (int i : frontier)
                for (int a = 0; a < 3; ++a) {
                    if (open(i, a)) {
                        const int l = i + step[a];
                        if (stamp[l] != j && inbox(l)) {
                            stamp[l] = j;
                            next.push_back(l);
                        }
                    }
                    if (i >= step[a] && open(i - step[a], a)) {
                        const int l = i - step[a];
                        if (stamp[l] != j && inbox(l)) {
                            stamp[l] = j;
                            next.push_back(l);
                        }
                    }
                }
            reached.insert(reached.end(), next.begin(), next.end());
            frontier.swap(next);
        }
        for (int i : reached) slots[i].push_back(j);  // j ascending: lists stay sorted
    }
    s.kind = 2;
    s.parent = p.parent;
    return explicit_stage_tables(c, s, M, slots);
}

// Graph stage (partition types "General" from a graph partitioner and
// "Static" from indicators or wells): the caller's block id per cell, blocks
// renumbered by ascending id (ids without an active cell dropped); the
// support of a block is every active cell within `overlap` face steps of it
// (breadth-first over the faces with T > 0).  Integer work on the host.
static int build_graph_stage(Ctx &c, const msrsb_partition &p, int index, Stage &s, const double *T3[3]) {
    const int N = c.N, nx = c.nx, nxy = c.nx * c.ny;
    const int step[3] = {1, nx, nxy};
    if (!p.block_of_cell || p.overlap < 0) {
        set_error("GRAPH partition %d: block_of_cell is NULL or overlap < 0", index);
        return MSRSB_E_INVAL;
    }
    int maxid = -1;
    for (int i = 0; i < N; ++i) {
        if (!c.h_active[i]) continue;
        const int b = p.block_of_cell[i];
        if (b < 0) {
            set_error("GRAPH partition %d: active cell %d has block %d", index, i, b);
            return MSRSB_E_INVAL;
        }
        maxid = std::max(maxid, b);
    }
    if (maxid < 0) {
        set_error("GRAPH partition %d: no active cell", index);
        return MSRSB_E_INVAL;
    }
    std::vector<int32_t> newid((size_t)maxid + 1, -1);
    for (int i = 0; i < N; ++i)
        if (c.h_active[i]) newid[p.block_of_cell[i]] = 1;
    int M = 0;
    for (auto &v : newid)
        if (v > 0) v = M++;
    s.h_xpblock.assign(N, -1);
    std::vector<std::vector<int>> members(M);
    for (int i = 0; i < N; ++i)
        if (c.h_active[i]) {
            s.h_xpblock[i] = newid[p.block_of_cell[i]];
            members[s.h_xpblock[i]].push_back(i);
        }
    std::vector<std::vector<int>> slots(N);
    std::vector<int> stamp(N, -1), frontier, next;
    for (int j = 0; j < M; ++j) {
        frontier = members[j];
        for (int i : frontier) stamp[i] = j;
        std::vector<int> reached = frontier;
        for (int d = 0; d < p.overlap && !frontier.empty(); ++d) {
            next.clear();
            for (int i : frontier)
                for (int a = 0; a < 3; ++a) {
                    if (T3[a][i] != 0.0 && stamp[i + step[a]] != j) {
                        stamp[i + step[a]] = j;
                        next.push_back(i + step[a]);
                    }
                    if (i >= step[a] && T3[a][i - step[a]] != 0.0 && stamp[i - step[a]] != j) {
                        stamp[i - step[a]] = j;
                        next.push_back(i - step[a]);
                    }
                }
            reached.insert(reached.end(), next.begin(), next.end());
            frontier.swap(next);
        }
        for (int i : reached) slots[i].push_back(j);  // j ascending: lists stay sorted
    }
    s.kind = 2;
    s.graph = true;
    s.parent = -1;
    return explicit_stage_tables(c, s, M, slots);
}

// Slot tables, per-block support lists and basis buffers of an explicit-slot
// stage from the sorted block list of every cell (s.h_xpblock holds the block
// of each cell, -1 inactive).
static int explicit_stage_tables(Ctx &c, Stage &s, int M, const std::vector<std::vector<int>> &slots) {
    const int N = c.N;
    int ns = 1;
    for (int i = 0; i < N; ++i) ns = std::max(ns, (int)slots[i].size());
    if (ns > kMaxXSlots) {
        set_error("explicit-slot stage needs %d slots per cell (limit %d)", ns, kMaxXSlots);
        return MSRSB_E_INVAL;
    }
    if (!slots_fit(ns, N)) {
        set_error("explicit-slot stage: %d basis slots of %d cells exceed the 2^31-byte slot arrays of the kernels", ns,
                  N);
        return MSRSB_E_INVAL;
    }
    if (M > kMaxXBlocks) {
        set_error("explicit-slot stage has %d blocks (limit %d)", M, kMaxXBlocks);
        return MSRSB_E_INVAL;
    }
    s.ns = ns;
    s.M = M;
    s.Mp = cdiv(M, kTile) * kTile;
    s.h_xsb.assign((size_t)ns * N, -1);
    std::vector<int32_t> cnt(M + 1, 0);
    for (int i = 0; i < N; ++i)
        for (size_t t = 0; t < slots[i].size(); ++t) {
            s.h_xsb[t * N + i] = slots[i][t];
            cnt[slots[i][t] + 1]++;
        }
    for (int j = 0; j < M; ++j) cnt[j + 1] += cnt[j];
    std::vector<int32_t> cell(cnt[M]), pos(cnt.begin(), cnt.end() - 1);
    std::vector<uint8_t> slot(cnt[M]);
    for (int i = 0; i < N; ++i)
        for (size_t t = 0; t < slots[i].size(); ++t) {
            const int j = slots[i][t];
            cell[pos[j]] = i;
            slot[pos[j]] = (uint8_t)t;
            pos[j]++;
        }
    auto upi = [&](int32_t *&dst, const std::vector<int32_t> &h) -> bool {
        dst = (int32_t *)ctx_alloc(c, sizeof(int32_t) * std::max<size_t>(h.size(), 1));
        return dst && upload(c, dst, h.data(), sizeof(int32_t) * h.size());
    };
    if (!upi(s.xsb, s.h_xsb) || !upi(s.xpblock, s.h_xpblock) || !upi(s.xptr, cnt) || !upi(s.xcell, cell))
        return MSRSB_E_NOMEM;
    s.xslot = (uint8_t *)ctx_alloc(c, std::max<size_t>(slot.size(), 1));
    if (!s.xslot || !upload(c, s.xslot, slot.data(), slot.size())) return MSRSB_E_NOMEM;
    s.xcnt = (uint8_t *)ctx_alloc(c, (size_t)N);
    if (ns <= kXNibSlots) s.xnib = (uint64_t *)ctx_alloc(c, (size_t)6 * 8 * N);
    else s.xnmap = (uint8_t *)ctx_alloc(c, (size_t)6 * ns * N);
    if (!s.xcnt || !(s.xnmap || s.xnib)) return MSRSB_E_NOMEM;
    launch_xmap_build(c, s);
    // chunk tables of the support lists.  Galerkin rows: the shortest chunk
    // (more wavefronts) whose partial rows fit the stage's partial-row bytes
    int rch = kXRapChunkMin;
    for (; rch < kXRapChunk; rch *= 2) {
        size_t rows = 0;
        for (int j = 0; j < M; ++j) {
            const int nr = cdiv(cnt[j + 1] - cnt[j], rch);
            if (nr > 1) rows += nr;
        }
        if (rows * (size_t)s.Mp * 8 <= xrap_part_bytes((size_t)cnt[M], s.Mp)) break;
    }
    s.xrchunk = rch;
    std::vector<int32_t> cblk, cfirst(M + 1), rcblk, rcfirst(M + 1), rrow;
    int nrow = 0;
    for (int j = 0; j < M; ++j) {
        const int len = cnt[j + 1] - cnt[j];
        cfirst[j] = (int32_t)cblk.size();
        for (int k = 0; k < std::max(1, cdiv(len, kXChunk)); ++k) cblk.push_back(j);
        rcfirst[j] = (int32_t)rcblk.size();
        const int nr = std::max(1, cdiv(len, rch));
        for (int k = 0; k < nr; ++k) {
            rcblk.push_back(j);
            rrow.push_back(nr > 1 ? nrow++ : -1);
        }
    }
    cfirst[M] = (int32_t)cblk.size();
    rcfirst[M] = (int32_t)rcblk.size();
    s.nxch = (int)cblk.size();
    s.nxrch = (int)rcblk.size();
    s.nxrrow = nrow;
    if (!upi(s.xcblk, cblk) || !upi(s.xcfirst, cfirst) || !upi(s.xrcblk, rcblk) || !upi(s.xrcfirst, rcfirst) ||
        !upi(s.xrrow, rrow))
        return MSRSB_E_NOMEM;
    s.nxent = cnt[M];
    s.xplist = ctx_alloc(c, (size_t)std::max(cnt[M], 1) * (c.opt.precision == MSRSB_MIXED ? 2 : 8));
    if (!s.xplist) return MSRSB_E_NOMEM;
    s.xpart = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.nxch);
    s.xrpart = (double *)ctx_alloc(c, sizeof(double) * std::max<size_t>((size_t)nrow * s.Mp, 1));
    if (!s.xpart || !s.xrpart) return MSRSB_E_NOMEM;
    // the host tables above are local: wait for their copies
    if (hipStreamSynchronize(c.stream) != hipSuccess) return hip_fail(hipGetLastError(), "upload fault tables");
    const size_t nsN = (size_t)ns * N;
    if (c.opt.precision == MSRSB_MIXED) {
        s.P32[0] = (float *)ctx_alloc(c, sizeof(float) * nsN);
        s.P32[1] = (float *)ctx_alloc(c, sizeof(float) * nsN);
        s.Pbf = (uint16_t *)ctx_alloc(c, sizeof(uint16_t) * nsN);
        if (!s.P32[0] || !s.P32[1] || !s.Pbf) return MSRSB_E_NOMEM;
    } else {
        s.P64[0] = (double *)ctx_alloc(c, sizeof(double) * nsN);
        s.P64[1] = (double *)ctx_alloc(c, sizeof(double) * nsN);
        if (!s.P64[0] || !s.P64[1]) return MSRSB_E_NOMEM;
    }
    s.Ac = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    s.Ainv = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    s.dvec = (double *)ctx_alloc(c, sizeof(double) * s.Mp);
    s.pc = (double *)ctx_alloc(c, sizeof(double) * s.Mp);
    if (!s.Ac || !s.Ainv || !s.dvec || !s.pc) return MSRSB_E_NOMEM;
    return MSRSB_OK;
}

static size_t cart_bytes(const Ctx &c, const msrsb_partition &p) {
    int nbits = 0;
    long M = 1;
    for (int a = 0; a < 3; ++a) {
        nbits += p.coarse_dims[a] > 1;
        M *= p.coarse_dims[a];
    }
    const long Mp = cdiv(M, kTile) * kTile;
    const size_t nsN = ((size_t)1 << nbits) * c.N;
    size_t b = (c.opt.precision == MSRSB_MIXED) ? nsN * 10 : nsN * 16;
    b += 16 * (size_t)Mp * Mp + 16 * Mp + 4 * (size_t)(c.nx + c.ny + c.nz) * 5 + 12 * (size_t)M;
    b += sizeof(double) * ((size_t)c.nz * p.coarse_dims[1] * p.coarse_dims[0] << nbits);  // restriction partials
    b += sizeof(double) * rap_part_doubles(1 << nbits, (int)M);                          // Galerkin partials
    return b;
}

// ---------------------------------------------------------- solve driver ----

__global__ void k_zero(int N, double *__restrict__ x, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] = 0.0;
}

static void zero_vec(Ctx &c, double *x, const int *done) {
    hipLaunchKernelGGL(k_zero, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, x, done);
}

static std::vector<Stage *> cycle_stages(Ctx &c) {
    std::vector<Stage *> v;
    for (auto &s : c.stages) v.push_back(&s);
    for (auto &s : c.dyn)
        if (s.M > 0) v.push_back(&s);
    return v;
}

// One cycle of eq. multiscale-multibasis on (b, x).  If r_valid, c.r already
// holds b - A x on entry; if x_zero, the cycle starts from x = 0 (x need not
// be initialised: the first smoother step assigns x = S b).
static void cycle(Ctx &c, const double *b, double *x, bool r_valid, const int *done, bool x_zero = false) {
    auto st = cycle_stages(c);
    for (size_t k = 0; k < st.size(); ++k) {
        Stage &s = *st[k];
        if (k == 0 && x_zero) {
            launch_smooth(c, b, x, done, true);
        } else {
            if (!(k == 0 && r_valid)) launch_residual(c, b, x, c.r, false, done);
            launch_smooth(c, c.r, x, done);
        }
        if (s.kind == 0) {
            launch_residual_restrict(c, s, b, x, done);
        } else {
            launch_residual(c, b, x, c.r, false, done);
            if (s.kind == 3) launch_dyn_restrict(c, s, c.r, done);
            else launch_restrict(c, s, c.r, done);
        }
        launch_coarse_solve(c, s, done);
        if (s.kind == 3) launch_dyn_prolong(c, s, x, done);
        else launch_prolong(c, s, x, done);
    }
}

static int read_status(Ctx &c) {
    hipError_t e = hipMemcpyAsync(c.h_status, c.status, sizeof(Status), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "status read");
    return MSRSB_OK;
}

static void begin_solve(Ctx &c, const double *b, double *x) { launch_begin_solve(c, b, x); }

static int solve_richardson(Ctx &c, const double *b, double *x, double rtol, int max_iters) {
    launch_residual(c, b, x, c.r, true, nullptr);
    launch_norm_finish(c, c.scal, nullptr);
    launch_check(c, rtol, max_iters, 0);
    int chunk = 2;
    int rc;
    for (;;) {
        if ((rc = read_status(c))) return rc;
        if (c.h_status->done) break;
        for (int k = 0; k < chunk; ++k) {
            const int *done = &c.status->done;
            cycle(c, b, x, true, done);
            launch_residual(c, b, x, c.r, true, done);
            launch_norm_finish(c, c.scal, done);
            launch_check(c, rtol, max_iters, 1);
        }
        chunk = std::min(chunk * 2, 16);
    }
    return MSRSB_OK;
}

// Mixed precision keeps the GMRES basis in FP32 on the DCGS2 path (dots,
// Hessenberg and candidate vectors stay FP64; the restart residual is FP64).
static bool fp32_basis(const msrsb_options &o) { return o.precision == MSRSB_MIXED && o.restart <= kDcgsMax; }

static int solve_gmres(Ctx &c, const double *b, double *x, double rtol, int max_iters) {
    const int m = std::max(1, std::min(c.opt.restart, kMaxRestart));
    const long N = c.N;
    double *w = c.tmp;
    const bool dcgs = m <= kDcgsMax;
    int rc;
    for (;;) {
        // restart: true residual of the current iterate (DCGS2: into V(0),
        // which holds u_0 = r; the cycle overwrites c.r)
        launch_residual(c, b, x, dcgs ? c.V : c.r, true, nullptr);
        launch_norm_finish(c, c.scal, nullptr);
        launch_gmres_begin(c, rtol, max_iters);
        if ((rc = read_status(c))) return rc;
        if (c.h_status->done) break;
        if (!dcgs) launch_gmres_start(c, c.r, c.V, m);
        int j = 0;
        int chunk = 4;
        while (j < m) {
            const int jend = std::min(m, j + chunk);
            for (; j < jend; ++j) {
                const int *done = &c.status->done;
                if (dcgs) {
                    // column j from u_j = V(j) (u_0 = r); q_j and u_{j+1} land in V
                    const double *uj = c.V + (c.Vf ? (long)(j & 1) : (long)j) * N;
                    double *zj = c.Z + (long)j * N;  // kept for the solution update
                    cycle(c, uj, zj, false, done, true);
                    launch_dgmres_step(c, zj, w, uj, j, rtol, max_iters, false);
                } else {
                    double *vj = c.V + (long)j * N;
                    cycle(c, vj, c.z, false, done, true);
                    launch_arnoldi(c, c.z, w, j, rtol, max_iters, m);
                }
            }
            if ((rc = read_status(c))) return rc;
            if (c.h_status->done) break;
            chunk = std::min(chunk * 2, 16);
        }
        int k;
        if (dcgs && j == m && !c.h_status->done) {
            // finalise the last column from u_m; the step sets jcur = m, so the
            // host need not wait for it (the restart's status read follows)
            launch_dgmres_step(c, nullptr, w, c.V + (c.Vf ? (long)(m & 1) : (long)m) * N, m, rtol, max_iters, true);
            k = m;
        } else {
            k = c.h_status->jcur;
        }
        // x += M^{-1} V y.  DCGS2: M^-1 Q = Z T^-1 from the stored candidates,
        // so x += Z (T^-1 y) without another application of the cycle
        if (k > 0 && dcgs) {
            launch_gmres_solve_small(c, m, true);
            launch_multiaxpy(c, c.Z, k, c.scal + kScalW, x, 1.0, false, nullptr);
        } else if (k > 0) {
            launch_gmres_solve_small(c, m);
            zero_vec(c, c.u, nullptr);
            if (c.Vf) launch_multiaxpy(c, c.Vf, k, c.scal + 4608, c.u, 1.0, false, nullptr);
            else launch_multiaxpy(c, c.V, k, c.scal + 4608, c.u, 1.0, false, nullptr);
            cycle(c, c.u, c.z, false, nullptr, true);
            launch_axpy(c, x, c.z, nullptr);
        }
    }
    return MSRSB_OK;
}

// ---- hooks for the two-phase CPR preconditioner (tp_capi.hip) ----

// One multistage cycle from zero: x = M^{-1} r (the multiscale multibasis
// preconditioner of the pressure system).
void ms_precondition(Ctx &c, const double *r, double *x) { cycle(c, r, x, false, nullptr, true); }

__global__ void k_to_f32(long n, const double *__restrict__ a, float *__restrict__ b) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Per-cell sums of the connection terms in a fixed order (the connections of
// a cell in list order).
__global__ void k_bc_sums(int N, const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                          const double *__restrict__ bct, const double *__restrict__ bcv, double *__restrict__ bcd,
                          double *__restrict__ bcr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double d = 0.0, r = 0.0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        d += bct[idx[k]];
        r += bct[idx[k]] * bcv[idx[k]];
    }
    bcd[i] = d;
    bcr[i] = r;
}

// Replace the operator from device arrays (face coefficients [3N] and
// connection coefficients [n_bc], either may be null) with the same
// connectivity: no host validation, so the caller guarantees T >= 0 exactly
// where the set-up faces had T > 0.  Rebuilds A, b, FP32 copies and pivots.
int set_operator_device(Ctx &c, const double *d_t3, const double *d_bc) {
    const size_t N = c.N;
    if (d_t3) {
        double *d64[3] = {c.tx, c.ty, c.tz};
        float *d32[3] = {c.tx32, c.ty32, c.tz32};
        for (int a = 0; a < 3; ++a) {
            if (hipMemcpyAsync(d64[a], d_t3 + a * N, 8 * N, hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
                return hip_fail(hipGetLastError(), "operator copy");
            hipLaunchKernelGGL(k_to_f32, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, c.stream, (long)N, d64[a], d32[a]);
        }
    }
    if (d_bc && c.n_bc > 0) {
        if (hipMemcpyAsync(c.bc_trans, d_bc, 8 * (size_t)c.n_bc, hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
            return hip_fail(hipGetLastError(), "connection copy");
        hipLaunchKernelGGL(k_bc_sums, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, c.stream, (int)N, c.bcptr, c.bcidx,
                           c.bc_trans, c.bc_value, c.bcdiag, c.bcrhs);
    }
    launch_assemble(c);
    launch_ilu_factor(c);
    return MSRSB_OK;
}

// After an operator change: `sweeps` more smoothing sweeps of every general
// and static basis from its current state (the local updates), then new
// Galerkin operators and inverses for every stage, dynamic ones included.
int refresh_bases(Ctx &c, int sweeps) {
    int rc;
    for (auto &s : c.stages) {
        if (!s.has_basis) continue;
        if (sweeps > 0 && (rc = launch_sweeps(c, s, sweeps, 0.0, true, nullptr, nullptr))) return rc;
        s.version++;
        launch_rap(c, s);
        if ((rc = finish_coarse(c, s))) return rc;
    }
    for (auto &s : c.dyn)
        if (s.M > 0) {
            launch_dyn_rap(c, s);
            if ((rc = finish_coarse(c, s))) return rc;
        }
    return MSRSB_OK;
}

}  // namespace msrsb

using namespace msrsb;


extern "C" {

const char *msrsb_last_error(void) { return g_err.c_str(); }

void msrsb_default_options(msrsb_options *o) {
    if (!o) return;
    o->omega = 2.0 / 3.0;
    o->omega_s = 2.0 / 3.0;
    o->smoother = MSRSB_SMOOTH_JACOBI;
    o->precision = MSRSB_FP64;
    o->n_bins = 4;
    o->max_dyn_blocks = 4096;
    o->outer = MSRSB_RICHARDSON;
    o->restart = 30;
}

static int check_options(const msrsb_options *o) {
    if (!(o->omega > 0.0 && o->omega < 2.0) || !(o->omega_s > 0.0 && o->omega_s < 2.0)) {
        set_error("omega and omega_s must lie in (0, 2)");
        return MSRSB_E_INVAL;
    }
    if (o->smoother != MSRSB_SMOOTH_JACOBI && o->smoother != MSRSB_SMOOTH_ILU0_RB &&
        o->smoother != MSRSB_SMOOTH_ILU0_LINE) {
        set_error("unknown smoother %d", o->smoother);
        return MSRSB_E_INVAL;
    }
    if (o->precision != MSRSB_FP64 && o->precision != MSRSB_MIXED) {
        set_error("unknown precision %d", o->precision);
        return MSRSB_E_INVAL;
    }
    if (o->n_bins < 1 || o->n_bins > 8 || o->max_dyn_blocks < 1) {
        set_error("n_bins must lie in [1, 8] and max_dyn_blocks >= 1");
        return MSRSB_E_INVAL;
    }
    if (o->outer != MSRSB_RICHARDSON && o->outer != MSRSB_GMRES) {
        set_error("unknown outer solver %d", o->outer);
        return MSRSB_E_INVAL;
    }
    if (o->restart < 1 || o->restart > kMaxRestart) {
        set_error("restart must lie in [1, %d]", kMaxRestart);
        return MSRSB_E_INVAL;
    }
    return MSRSB_OK;
}

static int check_parts(const msrsb_grid *g, int n_part, const msrsb_partition *parts) {
    if (n_part < 1 || !parts || parts[0].kind != MSRSB_PART_CARTESIAN) {
        set_error("at least one partition is needed and the first must be CARTESIAN");
        return MSRSB_E_INVAL;
    }
    for (int k = 0; k < n_part; ++k) {
        if (parts[k].kind == MSRSB_PART_FAULT_CUT) {
            if (parts[k].parent < 0 || parts[k].parent >= k || parts[parts[k].parent].kind != MSRSB_PART_CARTESIAN) {
                set_error("partition %d: FAULT_CUT needs an earlier CARTESIAN parent", k);
                return MSRSB_E_INVAL;
            }
            continue;
        }
        if (parts[k].kind == MSRSB_PART_GRAPH) {
            if (!parts[k].block_of_cell || parts[k].overlap < 0) {
                set_error("partition %d: GRAPH needs block_of_cell and overlap >= 0", k);
                return MSRSB_E_INVAL;
            }
            continue;
        }
        if (parts[k].kind != MSRSB_PART_CARTESIAN) {
            set_error("partition %d: unknown kind %d", k, parts[k].kind);
            return MSRSB_E_INVAL;
        }
        const int n[3] = {g->nx, g->ny, g->nz};
        int nbits = 0;
        for (int a = 0; a < 3; ++a) {
            if (parts[k].coarse_dims[a] < 1 || parts[k].coarse_dims[a] > n[a]) {
                set_error("partition %d: coarse_dims[%d] = %d outside [1, %d]", k, a, parts[k].coarse_dims[a], n[a]);
                return MSRSB_E_INVAL;
            }
            nbits += parts[k].coarse_dims[a] > 1;
        }
        if (!slots_fit(1 << nbits, (long)g->nx * g->ny * g->nz)) {
            set_error("partition %d: %d basis slots of %ld cells exceed the 2^31-byte slot arrays of the kernels", k,
                      1 << nbits, (long)g->nx * g->ny * g->nz);
            return MSRSB_E_INVAL;
        }
    }
    return MSRSB_OK;
}

// ---------------------------------------------- static partition builders ----

// Face neighbours (T > 0) of cell i, written to nb; returns the count.
static int face_nbrs(const msrsb_grid *g, int i, int nb[6]) {
    const int nxy = g->nx * g->ny, N = nxy * g->nz;
    const int step[3] = {1, g->nx, nxy};
    const double *T[3] = {g->tx, g->ty, g->tz};
    int n = 0;
    for (int a = 0; a < 3; ++a) {
        if (T[a][i] > 0.0 && i + step[a] < N) nb[n++] = i + step[a];
        if (i >= step[a] && T[a][i - step[a]] > 0.0) nb[n++] = i - step[a];
    }
    return n;
}

int msrsb_partition_wells(const msrsb_grid *g, int n_wells, const int32_t *well_ptr, const int32_t *well_cells,
                          int radius, int32_t *block) {
    g_err.clear();
    int rc = validate(g);
    if (rc) return rc;
    if (n_wells < 1 || !well_ptr || !well_cells || radius < 0 || !block) {
        set_error("need n_wells >= 1, well lists, radius >= 0 and an output array");
        return MSRSB_E_INVAL;
    }
    const int N = g->nx * g->ny * g->nz;
    auto act = [&](int i) { return !g->active || g->active[i]; };
    std::vector<int32_t> lab(N, -1);
    std::vector<int> frontier;
    // layer 0: the wells' own cells (a cell listed by two wells goes to the lower index)
    for (int w = 0; w < n_wells; ++w) {
        if (well_ptr[w + 1] <= well_ptr[w]) {
            set_error("well %d has no cells", w);
            return MSRSB_E_INVAL;
        }
        for (int k = well_ptr[w]; k < well_ptr[w + 1]; ++k) {
            const int i = well_cells[k];
            if (i < 0 || i >= N || !act(i)) {
                set_error("well %d: cell %d is not an active cell of the grid", w, i);
                return MSRSB_E_INVAL;
            }
            if (lab[i] < 0) {
                lab[i] = w;
                frontier.push_back(i);
            }
        }
    }
    // layer d + 1: unlabelled neighbours of layer d take the lowest label among
    // the layer-d cells next to them (smallest distance, ties to the lower well)
    std::vector<int> next;
    std::vector<int32_t> cand(N, INT32_MAX);
    int nb[6];
    for (int d = 0; d < radius && !frontier.empty(); ++d) {
        next.clear();
        for (int i : frontier) {
            const int n = face_nbrs(g, i, nb);
            for (int t = 0; t < n; ++t) {
                const int l = nb[t];
                if (lab[l] >= 0) continue;
                if (cand[l] == INT32_MAX) next.push_back(l);
                cand[l] = std::min(cand[l], lab[i]);
            }
        }
        for (int l : next) {
            lab[l] = cand[l];
            cand[l] = INT32_MAX;
        }
        frontier.swap(next);
    }
    for (int i = 0; i < N; ++i) block[i] = act(i) ? (lab[i] >= 0 ? lab[i] : n_wells) : -1;
    return MSRSB_OK;
}

int msrsb_partition_indicator(const msrsb_grid *g, const double *ind, int n_bins, const int32_t coarse_dims[3],
                              int min_cells, int32_t *block) {
    g_err.clear();
    int rc = validate(g);
    if (rc) return rc;
    const int n3[3] = {g->nx, g->ny, g->nz};
    if (!ind || n_bins < 1 || min_cells < 0 || !coarse_dims || !block) {
        set_error("need an indicator, n_bins >= 1, min_cells >= 0, coarse_dims and an output array");
        return MSRSB_E_INVAL;
    }
    for (int a = 0; a < 3; ++a)
        if (coarse_dims[a] < 1 || coarse_dims[a] > n3[a]) {
            set_error("coarse_dims[%d] = %d outside [1, %d]", a, coarse_dims[a], n3[a]);
            return MSRSB_E_INVAL;
        }
    const int N = g->nx * g->ny * g->nz, nx = g->nx, nxy = g->nx * g->ny;
    auto act = [&](int i) { return !g->active || g->active[i]; };
    std::vector<int> cells;
    for (int i = 0; i < N; ++i)
        if (act(i)) {
            if (!std::isfinite(ind[i])) {
                set_error("indicator not finite at active cell %d", i);
                return MSRSB_E_INVAL;
            }
            cells.push_back(i);
        }
    const long na = (long)cells.size();
    // 1. equal-count bins over the ranking by (indicator, cell)
    std::vector<int> ord(cells);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return ind[a] < ind[b]; });
    std::vector<int32_t> key(N, -1);
    auto parent = [&](int i) {
        const int c3[3] = {i % nx, (i / nx) % g->ny, i / nxy};
        int J[3];
        for (int a = 0; a < 3; ++a) J[a] = (int)(((long)c3[a] * coarse_dims[a]) / n3[a]);
        return J[0] + coarse_dims[0] * (J[1] + coarse_dims[1] * J[2]);
    };
    std::vector<int32_t> bin(N, -1), par(N, -1);
    for (long r = 0; r < na; ++r) bin[ord[r]] = (int32_t)(r * n_bins / na);
    for (int i : cells) par[i] = parent(i);
    // 2. pieces: face-connected cells with equal (parent, bin); root = smallest cell
    DSU d(N);
    int nb[6];
    for (int i : cells) {
        const int n = face_nbrs(g, i, nb);
        for (int t = 0; t < n; ++t)
            if (nb[t] > i && bin[nb[t]] == bin[i] && par[nb[t]] == par[i]) d.unite(i, nb[t]);
    }
    // pieces keyed by their smallest cell; member lists
    std::vector<int32_t> own(N, -1);
    std::vector<std::vector<int>> mem(N);
    for (int i : cells) {
        own[i] = d.find(i);
        mem[own[i]].push_back(i);
    }
    // 3. merging, smallest (size, key) first, through a lazy min-heap
    typedef std::pair<long, int> Item;  // (size, key)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int i : cells)
        if (own[i] == i && (long)mem[i].size() < min_cells) heap.push({(long)mem[i].size(), i});
    std::vector<int> cnt_key;
    std::vector<int32_t> cnt(N, 0);
    while (!heap.empty()) {
        const Item it = heap.top();
        heap.pop();
        const int k = it.second;
        if (mem[k].empty() || (long)mem[k].size() != it.first) continue;  // stale entry
        // shared faces with each same-parent neighbour piece
        cnt_key.clear();
        for (int i : mem[k]) {
            const int n = face_nbrs(g, i, nb);
            for (int t = 0; t < n; ++t) {
                const int l = nb[t];
                if (own[l] == k || par[l] != par[i]) continue;
                if (cnt[own[l]]++ == 0) cnt_key.push_back(own[l]);
            }
        }
        if (cnt_key.empty()) continue;  // no neighbour in its parent block: stays as it is
        int tgt = -1;
        for (int q : cnt_key)
            if (tgt < 0 || cnt[q] > cnt[tgt] || (cnt[q] == cnt[tgt] && q < tgt)) tgt = q;
        for (int q : cnt_key) cnt[q] = 0;
        // merge: the merged piece is keyed by the smaller key
        const int keep = std::min(k, tgt), gone = std::max(k, tgt);
        for (int i : mem[gone]) own[i] = keep;
        mem[keep].insert(mem[keep].end(), mem[gone].begin(), mem[gone].end());
        std::vector<int>().swap(mem[gone]);
        if ((long)mem[keep].size() < min_cells) heap.push({(long)mem[keep].size(), keep});
    }
    // 4. blocks numbered by their smallest cell
    std::vector<int32_t> id(N, -1);
    int M = 0;
    for (int i : cells)
        if (own[i] == i && !mem[i].empty()) id[i] = M++;
    for (int i = 0; i < N; ++i) block[i] = act(i) ? id[own[i]] : -1;
    return MSRSB_OK;
}

int msrsb_validate_grid(const msrsb_grid *grid) {
    g_err.clear();
    return validate(grid);
}

int msrsb_axis_support(int n, int m, int32_t *lo, int32_t *nv, int32_t *slo, int32_t *shi) {
    if (n < 1 || m < 1 || m > n) {
        set_error("need 1 <= m <= n");
        return MSRSB_E_INVAL;
    }
    std::vector<int32_t> a, b, c, d, e;
    axis_tables(n, m, a, b, c, d, e);
    if (lo) memcpy(lo, a.data(), sizeof(int32_t) * n);
    if (nv) memcpy(nv, b.data(), sizeof(int32_t) * n);
    if (slo) memcpy(slo, c.data(), sizeof(int32_t) * m);
    if (shi) memcpy(shi, d.data(), sizeof(int32_t) * m);
    return MSRSB_OK;
}

size_t msrsb_footprint_bytes(const msrsb_grid *g, int n_part, const msrsb_partition *parts, const msrsb_options *opt) {
    msrsb_options o;
    if (opt) o = *opt;
    else msrsb_default_options(&o);
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || (long)g->nx * g->ny * g->nz > 0x7fffffffL / 8 ||
        check_options(&o) || check_parts(g, n_part, parts))
        return 0;
    Ctx c;
    c.opt = o;
    c.nx = g->nx; c.ny = g->ny; c.nz = g->nz;
    c.N = g->nx * g->ny * g->nz;
    const size_t N = c.N;
    size_t b = N * 8 * 3 + N * 4 * 3 + N * 8 * 6 + N * 4 * 2;  // T, T32, diag/b/src/bcdiag/bcrhs/dtil, f32 copies
    b += N * 8 * 5;                                          // work vectors
    if (o.smoother == MSRSB_SMOOTH_ILU0_LINE) {             // z-line ILU(0) factors, packed copies
        b += N * 24;
        if (lilu_reg_chunks(c.nz)) b += 8 * lilu_slots(c.nx, c.ny, c.nz) * (o.precision == MSRSB_MIXED ? 4 : 8);
    }
    b += (size_t)kRedBlocks * (2 * kMaxRestart + 2) * 8 + 8192 * 8 + 65536 * 8;
    if (o.outer == MSRSB_GMRES) b += fp32_basis(o) ? N * 8 * 2 + (size_t)o.restart * N * 4 : (size_t)(o.restart + 1) * N * 8;
    if (o.outer == MSRSB_GMRES && o.restart <= kDcgsMax) b += (size_t)o.restart * N * 8;  // candidates M^-1 u_j
    b += (size_t)g->n_bc * 24;
    long cb = 0;
    for (int k = 0; k < n_part; ++k) {
        if (parts[k].kind == MSRSB_PART_GRAPH) {
            // blocks and slots from the block vector (supports as in build_graph_stage would need the
            // faces: estimated at 8 slots per cell)
            long M = 0;
            for (size_t i = 0; i < N; ++i)
                if (!g->active || g->active[i]) M = std::max(M, (long)parts[k].block_of_cell[i] + 1);
            const long Mp = cdiv(M, kTile) * kTile;
            const size_t nsN = (size_t)8 * N;
            b += (o.precision == MSRSB_MIXED ? nsN * 10 : nsN * 16) + nsN * 9 + N * 4 + 16 * (size_t)Mp * Mp + 16 * Mp;
            b += 6 * nsN + N;  // neighbour slot maps
            b += xrap_part_bytes(nsN, Mp) + (nsN / kXChunk + M) * 8;  // chunk partials
            b += nsN * 8;  // basis values in list order
            cb = std::max(cb, Mp);
            continue;
        }
        const msrsb_partition &pk = parts[k].kind == MSRSB_PART_FAULT_CUT ? parts[parts[k].parent] : parts[k];
        b += cart_bytes(c, pk);
        if (parts[k].kind == MSRSB_PART_FAULT_CUT) {
            const long Mf = 2L * pk.coarse_dims[0] * pk.coarse_dims[1] * pk.coarse_dims[2];
            b += (size_t)16 * 8 * N;  // slot tables, lists (16 slots)
            b += (size_t)6 * 16 * N + N;  // neighbour slot maps
            b += (size_t)16 * N * 8;      // basis values in list order
            b += xrap_part_bytes((size_t)16 * N, (long)cdiv(Mf, kTile) * kTile) + (16 * N / kXChunk + Mf) * 8;
        }
        long M = (long)pk.coarse_dims[0] * pk.coarse_dims[1] * pk.coarse_dims[2];
        if (parts[k].kind == MSRSB_PART_FAULT_CUT) M *= 2;
        cb = std::max(cb, (long)cdiv(M, kTile) * kTile);
    }
    cb = std::max(cb, (long)cdiv(o.max_dyn_blocks, kTile) * kTile);
    b += (size_t)(cb + 2 * kTile) * kTile * 8;
    return b;
}

int msrsb_setup(const msrsb_grid *g, int n_part, const msrsb_partition *parts, const msrsb_options *opt,
                const msrsb_allocator *alloc, void *hip_stream, msrsb_ctx **out) {
    g_err.clear();
    if (!out) {
        set_error("out is NULL");
        return MSRSB_E_INVAL;
    }
    *out = nullptr;
    int rc = validate(g);
    if (rc) return rc;
    msrsb_options o;
    if (opt) o = *opt;
    else msrsb_default_options(&o);
    if ((rc = check_options(&o)) || (rc = check_parts(g, n_part, parts))) return rc;
    if (alloc && (!alloc->alloc || !alloc->free)) {
        set_error("an allocator needs both alloc and free");
        return MSRSB_E_INVAL;
    }
    msrsb_ctx *c = new msrsb_ctx();
    c->opt = o;
    c->stream = (hipStream_t)hip_stream;
    if (alloc) c->ua = *alloc;
    (void)hipGetDevice(&c->device);
    c->nx = g->nx; c->ny = g->ny; c->nz = g->nz;
    const int N = c->N = g->nx * g->ny * g->nz;
    if (g->fault) c->h_fault.assign(g->fault, g->fault + (size_t)3 * N);
    c->h_active.assign(N, 1);
    if (g->active)
        for (int i = 0; i < N; ++i) c->h_active[i] = g->active[i] ? 1 : 0;
    c->n_active = 0;
    for (int i = 0; i < N; ++i) c->n_active += c->h_active[i];
    c->n_bc = g->n_bc;
    c->h_bc_cell.assign(g->bc_cell, g->bc_cell + g->n_bc);
    c->h_bc_trans.assign(g->bc_trans, g->bc_trans + g->n_bc);
    c->h_bc_value.assign(g->bc_value, g->bc_value + g->n_bc);
    // per-cell sums of the boundary connections
    std::vector<double> bcd(N, 0.0), bcr(N, 0.0);
    for (int k = 0; k < g->n_bc; ++k) {
        bcd[g->bc_cell[k]] += g->bc_trans[k];
        bcr[g->bc_cell[k]] += g->bc_trans[k] * g->bc_value[k];
    }
    std::vector<double> src(N, 0.0);
    if (g->source)
        for (int i = 0; i < N; ++i) src[i] = c->h_active[i] ? g->source[i] : 0.0;
    auto fail = [&](int code) {
        msrsb_destroy(c);
        return code;
    };
    auto up = [&](double *&dst, const double *h) -> bool {
        dst = (double *)ctx_alloc(*c, sizeof(double) * N);
        return dst && upload(*c, dst, h, sizeof(double) * N);
    };
    // FP32 copies converted on the device (round to nearest, as on the host)
    auto dev32 = [&](float *&dst, const double *d) -> bool {
        dst = (float *)ctx_alloc(*c, sizeof(float) * N);
        if (!dst) return false;
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, c->stream, (long)N, d, dst);
        return true;
    };
    // the set-up's buffers come from one arena of the estimated set-up size
    {
        const size_t est = msrsb_footprint_bytes(g, n_part, parts, &o);
        if (est > 0) {
            const size_t sz = est + est / 32 + ((size_t)1 << 20);
            size_t got = 0;
            void *a = c->ua.alloc ? nullptr : arena_take(c->device, sz, &got);
            if (a) {
                c->allocs.push_back(a);
                c->alloc_bytes.push_back(got);
            } else {
                got = sz;
                a = raw_alloc(*c, sz);  // on failure the buffers are allocated one by one
            }
            if (a) {
                c->arena = (char *)a;
                c->arena_size = got;
            }
            g_err.clear();
        }
        c->arena_open = true;
    }
    if (!up(c->tx, g->tx) || !up(c->ty, g->ty) || !up(c->tz, g->tz) || !up(c->bcdiag, bcd.data()) ||
        !up(c->bcrhs, bcr.data()) || !up(c->src, src.data()) || !dev32(c->tx32, c->tx) || !dev32(c->ty32, c->ty) ||
        !dev32(c->tz32, c->tz))
        return fail(MSRSB_E_NOMEM);
    auto dalloc = [&](size_t bytes) { return ctx_alloc(*c, bytes); };
    c->diag = (double *)dalloc(8 * (size_t)N);
    c->b = (double *)dalloc(8 * (size_t)N);
    c->dtil = (double *)dalloc(8 * (size_t)N);
    c->dtil32 = (float *)dalloc(4 * (size_t)N);
    c->diag32 = (float *)dalloc(4 * (size_t)N);
    if (o.smoother == MSRSB_SMOOTH_ILU0_LINE) {
        c->ldinv = (double *)dalloc(8 * (size_t)N);
        c->lcz = (double *)dalloc(8 * (size_t)N);
        c->ldinv32 = (float *)dalloc(4 * (size_t)N);
        c->lcz32 = (float *)dalloc(4 * (size_t)N);
        if (!c->ldinv || !c->lcz || !c->ldinv32 || !c->lcz32) return fail(MSRSB_E_NOMEM);
        if (lilu_reg_chunks(c->nz)) {
            const size_t S = lilu_slots(c->nx, c->ny, c->nz), w = o.precision == MSRSB_MIXED ? 4 : 8;
            c->lpack = dalloc(6 * S * w);
            c->lpe = dalloc(2 * S * w);
            if (!c->lpack || !c->lpe) return fail(MSRSB_E_NOMEM);
        }
    }
    c->r = (double *)dalloc(8 * (size_t)N);
    c->e = (double *)dalloc(8 * (size_t)N);
    c->tmp = (double *)dalloc(8 * (size_t)N);
    c->z = (double *)dalloc(8 * (size_t)N);
    c->u = (double *)dalloc(8 * (size_t)N);
    // reduction partials: dot/norm kernels, and one maximum per sweep workgroup
    const size_t npart = std::max({(size_t)kRedBlocks * (2 * kMaxRestart + 2),
                                   (size_t)cdiv(g->nx, 64) * cdiv((long)g->ny * g->nz, 4),
                                   (size_t)cdiv(N, kBlock)});
    c->partial = (double *)dalloc(8 * npart);
    c->scal = (double *)dalloc(8 * 16384);
    c->status = (Status *)dalloc(sizeof(Status));
    c->maxbits = (unsigned long long *)dalloc(8 * 65536);
    c->flag = (int *)dalloc(2 * sizeof(int));  // [1]: the second sweep of a stop-rule pair
    if (!c->diag || !c->b || !c->dtil || !c->dtil32 || !c->diag32 || !c->r || !c->e || !c->tmp || !c->z || !c->u ||
        !c->partial || !c->scal || !c->status || !c->maxbits || !c->flag)
        return fail(MSRSB_E_NOMEM);
    if (!(c->h_status = pinned_status())) return fail(MSRSB_E_NOMEM);
    // connections grouped by cell (list order kept) for device-side updates
    std::vector<int32_t> bcptr(N + 1, 0), bcidx(std::max(g->n_bc, 1));
    for (int k = 0; k < g->n_bc; ++k) bcptr[g->bc_cell[k] + 1]++;
    for (int i = 0; i < N; ++i) bcptr[i + 1] += bcptr[i];
    {
        std::vector<int32_t> pos(bcptr.begin(), bcptr.end() - 1);
        for (int k = 0; k < g->n_bc; ++k) bcidx[pos[g->bc_cell[k]]++] = k;
    }
    c->bcptr = (int32_t *)dalloc(4 * (size_t)(N + 1));
    c->bcidx = (int32_t *)dalloc(4 * bcidx.size());
    if (!c->bcptr || !c->bcidx) return fail(MSRSB_E_NOMEM);
    upload(*c, c->bcptr, bcptr.data(), 4 * (size_t)(N + 1));
    upload(*c, c->bcidx, bcidx.data(), 4 * bcidx.size());
    if (g->n_bc > 0) {
        c->bc_cell = (int32_t *)dalloc(4 * (size_t)g->n_bc);
        c->bc_trans = (double *)dalloc(8 * (size_t)g->n_bc);
        c->bc_value = (double *)dalloc(8 * (size_t)g->n_bc);
        if (!c->bc_cell || !c->bc_trans || !c->bc_value) return fail(MSRSB_E_NOMEM);
        upload(*c, c->bc_cell, g->bc_cell, 4 * (size_t)g->n_bc);
        upload(*c, c->bc_trans, g->bc_trans, 8 * (size_t)g->n_bc);
        upload(*c, c->bc_value, g->bc_value, 8 * (size_t)g->n_bc);
    }
    if (o.outer == MSRSB_GMRES) {
        if (fp32_basis(o)) {
            c->V = (double *)dalloc(8 * 2 * (size_t)N);
            c->Vf = (float *)dalloc(4 * (size_t)o.restart * N);
            if (!c->V || !c->Vf) return fail(MSRSB_E_NOMEM);
            if (hipMemsetAsync(c->Vf, 0, 4 * (size_t)o.restart * N, c->stream) != hipSuccess)
                return fail(MSRSB_E_DEVICE);
        } else {
            c->V = (double *)dalloc(8 * (size_t)(o.restart + 1) * N);
            if (!c->V) return fail(MSRSB_E_NOMEM);
        }
        if (o.restart <= kDcgsMax) {
            c->Z = (double *)dalloc(8 * (size_t)o.restart * N);
            if (!c->Z) return fail(MSRSB_E_NOMEM);
        }
    }
    c->stages.resize(n_part);
    long cb = cdiv(o.max_dyn_blocks, kTile) * kTile;
    const double *T3[3] = {g->tx, g->ty, g->tz};
    for (int k = 0; k < n_part; ++k) {
        if (parts[k].kind == MSRSB_PART_FAULT_CUT) rc = build_fault_stage(*c, parts[k], k, c->stages[k], T3);
        else if (parts[k].kind == MSRSB_PART_GRAPH) rc = build_graph_stage(*c, parts[k], k, c->stages[k], T3);
        else rc = build_cart_stage(*c, parts[k], c->stages[k]);
        if (rc) return fail(rc);
        cb = std::max(cb, (long)c->stages[k].Mp);
    }
    c->cbuf = (double *)dalloc(8 * (size_t)(cb + 2 * kTile) * kTile);  // + two diagonal-block inverses
    c->cbuf_n = cb;
    if (!c->cbuf) return fail(MSRSB_E_NOMEM);
    hipMemsetAsync(c->tmp, 0, 8 * (size_t)N, c->stream);
    launch_assemble(*c);
    launch_ilu_factor(*c);
    c->arena_open = false;  // later allocations (dynamic stages, exports) are freed on their own
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(hip_fail(e, "setup kernels"));
    *out = c;
    return MSRSB_OK;
}

static int finish_coarse(Ctx &c, Stage &s) {
    hipMemsetAsync(c.flag, 0, sizeof(int), c.stream);
    launch_coarse_inverse(c, s);
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, c.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse inverse");
    if (flag & 1) {
        set_error("coarse operator is not symmetric positive definite");
        return MSRSB_E_SINGULAR;
    }
    return MSRSB_OK;
}

// Replace the face transmissibilities (host [3N]: tx, ty, tz) and rebuild
// what depends on them on the device: diagonal, right-hand side, FP32 copies
// and the smoother's pivots.  Partitions and supports keep their set-up
// structure.
static int set_transmissibility(Ctx &c, const double *T, const double *bct) {
    const int N = c.N;
    std::vector<double> tcur;
    if (!T) {  // only the connections change: validate with the current faces
        tcur.resize((size_t)3 * N);
        const double *d64[3] = {c.tx, c.ty, c.tz};
        for (int a = 0; a < 3; ++a)
            if (hipMemcpy(tcur.data() + (size_t)a * N, d64[a], 8 * (size_t)N, hipMemcpyDeviceToHost) != hipSuccess)
                return hip_fail(hipGetLastError(), "transmissibility read");
        T = tcur.data();
    }
    msrsb_grid g{};
    g.nx = c.nx; g.ny = c.ny; g.nz = c.nz;
    g.active = c.h_active.data();
    g.tx = T; g.ty = T + N; g.tz = T + 2 * (size_t)N;
    g.n_bc = c.n_bc;
    g.bc_cell = c.h_bc_cell.data();
    g.bc_trans = bct ? bct : c.h_bc_trans.data();
    g.bc_value = c.h_bc_value.data();
    int rc = validate(&g);
    if (rc) return rc;
    std::vector<float> t32((size_t)3 * N);
    for (size_t i = 0; i < (size_t)3 * N; ++i) t32[i] = (float)T[i];
    double *d64[3] = {c.tx, c.ty, c.tz};
    float *d32[3] = {c.tx32, c.ty32, c.tz32};
    for (int a = 0; a < 3; ++a)
        if (!upload(c, d64[a], T + (size_t)a * N, 8 * (size_t)N) || !upload(c, d32[a], t32.data() + (size_t)a * N, 4 * (size_t)N))
            return hip_fail(hipGetLastError(), "transmissibility upload");
    std::vector<double> bcd, bcr;
    if (bct && c.n_bc > 0) {
        c.h_bc_trans.assign(bct, bct + c.n_bc);
        bcd.assign(N, 0.0);
        bcr.assign(N, 0.0);
        for (int k = 0; k < c.n_bc; ++k) {
            bcd[c.h_bc_cell[k]] += bct[k];
            bcr[c.h_bc_cell[k]] += bct[k] * c.h_bc_value[k];
        }
        if (!upload(c, c.bc_trans, bct, 8 * (size_t)c.n_bc) || !upload(c, c.bcdiag, bcd.data(), 8 * (size_t)N) ||
            !upload(c, c.bcrhs, bcr.data(), 8 * (size_t)N))
            return hip_fail(hipGetLastError(), "connection upload");
    }
    launch_assemble(c);
    launch_ilu_factor(c);
    hipError_t e = hipStreamSynchronize(c.stream);  // the host copies above are local
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transmissibility update");
    return MSRSB_OK;
}

int msrsb_update_basis(msrsb_ctx *c, int stage, const double *new_trans, const double *new_bc_trans, int max_sweeps,
                       double tol, int warm, int *sweeps_done, double *last_change) {
    g_err.clear();
    if (!c) {
        set_error("ctx is NULL");
        return MSRSB_E_INVAL;
    }
    if (stage < -1 || stage >= (int)c->stages.size() || max_sweeps < 0 || max_sweeps > 65536 || !(tol >= 0.0)) {
        set_error("bad stage/max_sweeps/tol");
        return MSRSB_E_INVAL;
    }
    const int s0 = stage < 0 ? 0 : stage, s1 = stage < 0 ? (int)c->stages.size() : stage + 1;
    for (int k = s0; k < s1; ++k)
        if (warm && !c->stages[k].has_basis) {
            set_error("warm start of stage %d before its basis exists", k);
            return MSRSB_E_STATE;
        }
    int rc;
    const bool changed = new_trans || new_bc_trans;
    if (changed && (rc = set_transmissibility(*c, new_trans, new_bc_trans))) return rc;
    for (int k = s0; k < s1; ++k) {
        Stage &s = c->stages[k];
        rc = launch_sweeps(*c, s, max_sweeps, tol, warm != 0, sweeps_done, last_change);
        if (rc) return rc;
        s.version++;
        launch_rap(*c, s);
        if ((rc = finish_coarse(*c, s))) return rc;
        s.has_basis = true;
    }
    if (changed) {
        for (auto &s : c->stages) s.version++;
        // every other stage keeps its basis; its coarse operator follows the new A
        for (int k = 0; k < (int)c->stages.size(); ++k) {
            Stage &s = c->stages[k];
            if ((k >= s0 && k < s1) || !s.has_basis) continue;
            launch_rap(*c, s);
            if ((rc = finish_coarse(*c, s))) return rc;
        }
        for (auto &s : c->dyn)
            if (s.M > 0) {
                launch_dyn_rap(*c, s);
                if ((rc = finish_coarse(*c, s))) return rc;
            }
    }
    return MSRSB_OK;
}

// ------------------------------------------------------ finite volume ----

// Host tables of a stage's own blocks for the finite-volume mode (once per
// stage): block per cell, cell lists, list positions, an explicit slot table
// for rectilinear stages, chunk tables over the lists, operator buffers.
static int fv_prepare(Ctx &c, Stage &s) {
    const int N = c.N, M = s.M;
    std::vector<int32_t> blk(N, -1), sbv;
    if (s.kind == 2) {
        blk = s.h_xpblock;
    } else {
        sbv.assign((size_t)s.ns * N, -1);
        const CartDev &cd = s.cart;
        const int32_t *T = s.h_tab.data();
        const int cmap_off = (int)(cd.cmap - s.d_tab);
        for (int i = 0; i < N; ++i) {
            if (!c.h_active[i]) continue;
            const int c3[3] = {i % c.nx, (i / c.nx) % c.ny, i / (c.nx * c.ny)};
            int J[3], lo[3], nv[3];
            for (int a = 0; a < 3; ++a) {
                J[a] = (int)(((long)c3[a] * cd.m[a]) / cd.n[a]);
                lo[a] = T[s.tab_off[a][0] + c3[a]];
                nv[a] = T[s.tab_off[a][1] + c3[a]];
            }
            blk[i] = T[cmap_off + J[0] + cd.m[0] * (J[1] + cd.m[1] * J[2])];
            for (int sl = 0; sl < s.ns; ++sl) {
                int K[3];
                bool ok = true;
                for (int a = 0; a < 3; ++a) {
                    const int bit = cd.bit[a] >= 0 ? (sl >> cd.bit[a]) & 1 : 0;
                    if (bit >= nv[a]) ok = false;
                    K[a] = lo[a] + bit;
                }
                if (ok) sbv[(size_t)sl * N + i] = T[cmap_off + K[0] + cd.m[0] * (K[1] + cd.m[1] * K[2])];
            }
        }
    }
    std::vector<int32_t> ptr(M + 1, 0), loc(N, -1);
    for (int i = 0; i < N; ++i)
        if (blk[i] >= 0) ptr[blk[i] + 1]++;
    int maxc = 0;
    for (int j = 0; j < M; ++j) {
        maxc = std::max(maxc, ptr[j + 1]);
        ptr[j + 1] += ptr[j];
    }
    if (maxc > kFvMaxCells) {
        set_error("finite-volume mode: a block of %d cells exceeds the %d-cell limit of the local solves", maxc,
                  kFvMaxCells);
        return MSRSB_E_INVAL;
    }
    std::vector<int32_t> cells(std::max(ptr[M], 1)), pos(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < N; ++i)
        if (blk[i] >= 0) {
            loc[i] = pos[blk[i]] - ptr[blk[i]];
            cells[pos[blk[i]]++] = i;
        }
    std::vector<int32_t> rcblk, rcfirst(M + 1), rrow;
    int nrow = 0;
    for (int j = 0; j < M; ++j) {
        const int nr = std::max(1, cdiv(ptr[j + 1] - ptr[j], kXRapChunk));
        rcfirst[j] = (int32_t)rcblk.size();
        for (int k = 0; k < nr; ++k) {
            rcblk.push_back(j);
            rrow.push_back(nr > 1 ? nrow++ : -1);
        }
    }
    rcfirst[M] = (int32_t)rcblk.size();
    auto upi = [&](int32_t *&dst, const std::vector<int32_t> &h) -> bool {
        dst = (int32_t *)ctx_alloc(c, sizeof(int32_t) * std::max<size_t>(h.size(), 1));
        return dst && upload(c, dst, h.data(), sizeof(int32_t) * h.size());
    };
    if (!upi(s.fvblock, blk) || !upi(s.fvptr, ptr) || !upi(s.fvcells, cells) || !upi(s.fvloc, loc) ||
        !upi(s.fvrcblk, rcblk) || !upi(s.fvrcfirst, rcfirst) || !upi(s.fvrrow, rrow) ||
        (s.kind != 2 && !upi(s.fvsb, sbv)))
        return MSRSB_E_NOMEM;
    s.nfvrch = (int)rcblk.size();
    s.nfvrrow = nrow;
    s.fvrpart = (double *)ctx_alloc(c, sizeof(double) * std::max<size_t>((size_t)nrow * s.Mp, 1));
    s.Afv = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    s.Afvinv = (double *)ctx_alloc(c, sizeof(double) * (size_t)s.Mp * s.Mp);
    if (!s.fvrpart || !s.Afv || !s.Afvinv) return MSRSB_E_NOMEM;
    hipError_t e = hipStreamSynchronize(c.stream);  // the host tables above are local
    if (e != hipSuccess) return hip_fail(e, "finite-volume tables");
    s.fv_maxcells = maxc;
    s.fv_ready = true;
    return MSRSB_OK;
}

int msrsb_solve_fv(msrsb_ctx *c, int stage, const double *d_source, double *d_p, double *d_p_fine,
                   double *d_face_flux, double *d_bc_flux, double local_rtol, int max_local_iters, int *local_iters,
                   double *max_imbalance) {
    g_err.clear();
    if (!c || !d_p || !d_face_flux || !(local_rtol >= 0.0) || max_local_iters < 0) {
        set_error("bad finite-volume solve arguments");
        return MSRSB_E_INVAL;
    }
    if (stage < 0 || stage >= (int)c->stages.size()) {
        set_error("finite-volume mode needs a general or static stage (0..%d)", (int)c->stages.size() - 1);
        return MSRSB_E_INVAL;
    }
    Stage &s = c->stages[stage];
    if (!s.has_basis) {
        set_error("stage %d has no basis yet", stage);
        return MSRSB_E_STATE;
    }
    int rc;
    if (!s.fv_ready && (rc = fv_prepare(*c, s))) return rc;
    if (s.fv_version != s.version) {
        launch_fv_rap(*c, s);
        hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
        launch_coarse_inverse_of(*c, s.Afv, s.Afvinv, s.Mp, true);
        int flag = 0;
        hipError_t e = hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "finite-volume coarse operator");
        if (flag & 1) {
            set_error("finite-volume coarse operator of stage %d has a zero pivot", stage);
            return MSRSB_E_SINGULAR;
        }
        s.fv_version = s.version;
    }
    if (d_source) launch_source_update(*c, d_source);
    launch_fv_restrict(*c, s, c->b);
    launch_coarse_solve_with(*c, s, s.Afvinv, nullptr);
    zero_vec(*c, d_p, nullptr);
    launch_prolong(*c, s, d_p, nullptr);
    double *pf = d_p_fine ? d_p_fine : c->e;
    zero_vec(*c, pf, nullptr);
    int *iters_dev = (int *)(c->maxbits + 1);
    hipMemsetAsync(c->maxbits, 0, 2 * sizeof(unsigned long long), c->stream);
    if ((rc = launch_fv_local(*c, s, d_p, pf, local_rtol, max_local_iters, iters_dev))) {
        set_error("finite-volume local solves: block size not supported");
        return rc;
    }
    launch_fv_faces(*c, s, d_p, pf, d_face_flux);
    if (d_bc_flux) launch_fluxes(*c, pf, nullptr, d_bc_flux);
    launch_fv_imbalance(*c, d_face_flux, pf, c->maxbits);
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(h, c->maxbits, sizeof h, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "finite-volume solve");
    if (local_iters) *local_iters = (int)(h[1] & 0xffffffffu);
    if (max_imbalance) memcpy(max_imbalance, &h[0], sizeof(double));
    return MSRSB_OK;
}

int msrsb_add_dynamic_basis(msrsb_ctx *c, int n_incr, const double *const *d_dp, int *n_dyn_blocks) {
    g_err.clear();
    if (!c || n_incr < 1 || n_incr > 2 || !d_dp) {
        set_error("need 1 or 2 increments");
        return MSRSB_E_INVAL;
    }
    {
        const Stage &s0 = c->stages[0];
        for (int J = 0; J < s0.cart.m[0] * s0.cart.m[1] * s0.cart.m[2]; ++J) {
            const int Jx = J % s0.cart.m[0], Jy = (J / s0.cart.m[0]) % s0.cart.m[1],
                      Jz = J / (s0.cart.m[0] * s0.cart.m[1]);
            const int *be0 = s0.h_tab.data() + s0.tab_off[0][4], *be1 = s0.h_tab.data() + s0.tab_off[1][4],
                      *be2 = s0.h_tab.data() + s0.tab_off[2][4];
            const long vol = (long)(be0[Jx + 1] - be0[Jx]) * (be1[Jy + 1] - be1[Jy]) * (be2[Jz + 1] - be2[Jz]);
            if (vol > 6144) {
                set_error("general blocks of %ld cells exceed the 6144-cell limit of dynamic partitioning", vol);
                return MSRSB_E_INVAL;
            }
        }
    }
    if ((int)c->dyn.size() < 2) c->dyn.resize(2);
    for (int k = 0; k < 2; ++k) c->dyn[k].M = 0;
    int slot = 0;
    // on any failure no dynamic stage of this call stays in the cycle
    auto fail = [&](int rc) {
        for (int k = 0; k < 2; ++k) c->dyn[k].M = 0;
        return rc;
    };
    for (int k = 0; k < n_incr; ++k) {
        int count = 0;
        Stage &s = c->dyn[slot];
        int rc = build_dynamic_stage(*c, d_dp[k], s, &count);
        if (rc) return fail(rc);
        if (n_dyn_blocks) n_dyn_blocks[k] = count;
        if (count == 0) continue;
        if (s.Mp > c->cbuf_n) {
            ctx_free(*c, c->cbuf);
            c->cbuf = (double *)ctx_alloc(*c, 8 * (size_t)(s.Mp + 2 * kTile) * kTile);
            c->cbuf_n = c->cbuf ? s.Mp : 0;
            if (!c->cbuf) return fail(MSRSB_E_NOMEM);
        }
        launch_dyn_rap(*c, s);
        if ((rc = finish_coarse(*c, s))) return fail(rc);
        s.has_basis = true;
        ++slot;
    }
    return MSRSB_OK;
}

int msrsb_clear_dynamic_basis(msrsb_ctx *c) {
    if (!c) return MSRSB_E_INVAL;
    for (auto &s : c->dyn) s.M = 0;
    return MSRSB_OK;
}

static bool ready(msrsb_ctx *c) {
    for (auto &s : c->stages)
        if (!s.has_basis) return false;
    return true;
}

int msrsb_solve(msrsb_ctx *c, const double *d_source, double *d_p, double rtol, int max_iters, int *iters,
                double *relres) {
    g_err.clear();
    if (!c || !d_p || !(rtol >= 0.0) || max_iters < 0) {
        set_error("bad solve arguments");
        return MSRSB_E_INVAL;
    }
    if (!ready(c)) {
        set_error("solve called before update_basis");
        return MSRSB_E_STATE;
    }
    if (d_source) launch_source_update(*c, d_source);
    begin_solve(*c, c->b, d_p);
    int rc = c->opt.outer == MSRSB_GMRES ? solve_gmres(*c, c->b, d_p, rtol, max_iters)
                                         : solve_richardson(*c, c->b, d_p, rtol, max_iters);
    if (rc) return rc;
    if ((rc = read_status(*c))) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "solve kernels");
    if (iters) *iters = c->h_status->iters;
    if (relres) *relres = c->h_status->relres;
    if (!(c->h_status->relres <= rtol)) {
        set_error("tolerance %g not met after %d iterations (relative residual %g)", rtol, c->h_status->iters,
                  c->h_status->relres);
        return MSRSB_E_NOCONV;
    }
    return MSRSB_OK;
}

__global__ void k_write_result(const Status *st, double rtol, msrsb_result *out) {
    out->cycles = st->iters;
    out->relres = st->relres;
    out->status = st->relres <= rtol ? MSRSB_OK : MSRSB_E_NOCONV;
}

int msrsb_solve_async(msrsb_ctx *c, const double *d_source, double *d_p, double rtol, int max_cycles,
                      msrsb_result *d_result) {
    g_err.clear();
    if (!c || !d_p || !(rtol >= 0.0) || max_cycles < 1 || max_cycles > 100000) {
        set_error("bad asynchronous solve arguments");
        return MSRSB_E_INVAL;
    }
    if (!ready(c)) {
        set_error("solve called before update_basis");
        return MSRSB_E_STATE;
    }
    Ctx &x = *c;
    if (d_source) launch_source_update(x, d_source);
    begin_solve(x, x.b, d_p);
    // the Richardson loop of solve_richardson, every cycle enqueued at once:
    // after the test is met, `done` turns each later kernel into a no-op
    launch_residual(x, x.b, d_p, x.r, true, nullptr);
    launch_norm_finish(x, x.scal, nullptr);
    launch_check(x, rtol, max_cycles, 0);
    const int *done = &x.status->done;
    for (int k = 0; k < max_cycles; ++k) {
        cycle(x, x.b, d_p, true, done);
        launch_residual(x, x.b, d_p, x.r, true, done);
        launch_norm_finish(x, x.scal, done);
        launch_check(x, rtol, max_cycles, 1);
    }
    if (d_result) hipLaunchKernelGGL(k_write_result, dim3(1), dim3(1), 0, x.stream, x.status, rtol, d_result);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "asynchronous solve launches");
    return MSRSB_OK;
}

int msrsb_faces_to_box(int32_t nx, int32_t ny, int32_t nz, int32_t n_faces, const int32_t *face_cells,
                       const double *face_trans, double *tx, double *ty, double *tz) {
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1 || (long)nx * ny * nz > 0x7fffffffL / 8 || n_faces < 0 ||
        (n_faces > 0 && (!face_cells || !face_trans)) || !tx || !ty || !tz) {
        set_error("bad box or face arrays");
        return MSRSB_E_INVAL;
    }
    const long N = (long)nx * ny * nz, nxy = (long)nx * ny;
    double *T[3] = {tx, ty, tz};
    for (int a = 0; a < 3; ++a) std::fill(T[a], T[a] + N, 0.0);
    std::vector<uint8_t> seen((size_t)3 * N, 0);
    for (int f = 0; f < n_faces; ++f) {
        const long a = face_cells[2 * (long)f], b = face_cells[2 * (long)f + 1];
        const double t = face_trans[f];
        if (a < 0 || b >= N || a >= b) {
            set_error("face %d: cells (%ld, %ld) not an ascending pair inside the box", f, a, b);
            return MSRSB_E_INVAL;
        }
        int ax = -1;
        if (b - a == 1 && a % nx + 1 < nx) ax = 0;
        else if (b - a == nx && (a / nx) % ny + 1 < ny) ax = 1;
        else if (b - a == nxy) ax = 2;
        if (ax < 0) {
            set_error("face %d: cells %ld and %ld are not box neighbours (only box grids are supported)", f, a, b);
            return MSRSB_E_INVAL;
        }
        if (!(t >= 0.0) || !std::isfinite(t)) {
            set_error("face %d: transmissibility %g is negative or not finite", f, t);
            return MSRSB_E_INVAL;
        }
        if (seen[(size_t)ax * N + a]++) {
            set_error("face %d: cells %ld and %ld are joined twice", f, a, b);
            return MSRSB_E_INVAL;
        }
        T[ax][a] = t;
    }
    return MSRSB_OK;
}

int msrsb_apply(msrsb_ctx *c, int op, const double *d_in, double *d_out) {
    g_err.clear();
    if (!c || !d_in || !d_out || d_in == d_out) {
        set_error("bad apply arguments");
        return MSRSB_E_INVAL;
    }
    switch (op) {
    case MSRSB_OP_RESIDUAL: launch_residual(*c, c->b, d_in, d_out, false, nullptr); break;
    case MSRSB_OP_SMOOTH: launch_smooth(*c, d_in, d_out, nullptr, true); break;
    case MSRSB_OP_PRECOND:
        if (!ready(c)) {
            set_error("precondition before update_basis");
            return MSRSB_E_STATE;
        }
        cycle(*c, d_in, d_out, false, nullptr, true);
        break;
    case MSRSB_OP_MATVEC: launch_matvec(*c, d_in, d_out, false, nullptr); break;
    default: set_error("unknown op %d", op); return MSRSB_E_INVAL;
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "apply");
    return MSRSB_OK;
}

int msrsb_fluxes(msrsb_ctx *c, const double *d_p, double *d_face_flux, double *d_bc_flux) {
    g_err.clear();
    if (!c || !d_p) {
        set_error("bad flux arguments");
        return MSRSB_E_INVAL;
    }
    launch_fluxes(*c, d_p, d_face_flux, d_bc_flux);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fluxes");
    return MSRSB_OK;
}

int msrsb_num_stages(msrsb_ctx *c) {
    if (!c) return MSRSB_E_INVAL;
    int n = (int)c->stages.size();
    for (auto &s : c->dyn) n += s.M > 0;
    return n;
}

static Stage *stage_at(msrsb_ctx *c, int k) {
    auto v = cycle_stages(*c);
    if (k < 0 || k >= (int)v.size()) return nullptr;
    return v[k];
}

int msrsb_stage_info(msrsb_ctx *c, int stage, int *M, int *kind, int *n_slots) {
    g_err.clear();
    if (!c) return MSRSB_E_INVAL;
    Stage *s = stage_at(c, stage);
    if (!s) {
        set_error("no stage %d", stage);
        return MSRSB_E_INVAL;
    }
    if (M) *M = s->M;
    if (kind) *kind = s->graph ? MSRSB_PART_GRAPH : s->kind;
    if (n_slots) *n_slots = s->ns;
    return MSRSB_OK;
}

int msrsb_export_stage(msrsb_ctx *c, int stage, int32_t *h_block, int32_t *h_slot_block, double *h_vals,
                       double *h_Ac) {
    g_err.clear();
    if (!c) return MSRSB_E_INVAL;
    Stage *s = stage_at(c, stage);
    if (!s) {
        set_error("no stage %d", stage);
        return MSRSB_E_INVAL;
    }
    const int N = c->N;
    hipError_t e = hipSuccess;
    if (s->kind == 2) {
        if (h_block) memcpy(h_block, s->h_xpblock.data(), 4 * (size_t)N);
        if (h_slot_block) memcpy(h_slot_block, s->h_xsb.data(), 4 * (size_t)s->ns * N);
        if (h_vals) {
            double *dv = (double *)ctx_alloc(*c, 8 * (size_t)s->ns * N);
            if (!dv) return MSRSB_E_NOMEM;
            launch_export_cart(*c, *s, dv);
            e = hipStreamSynchronize(c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(h_vals, dv, 8 * (size_t)s->ns * N, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            ctx_free(*c, dv);
            if (e != hipSuccess) return hip_fail(e, "export");
        }
    } else if (s->kind == 3) {
        std::vector<int32_t> blk(N);
        e = hipMemcpyAsync(blk.data(), s->dblock, 4 * (size_t)N, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "export");
        if (h_block) memcpy(h_block, blk.data(), 4 * (size_t)N);
        if (h_slot_block) memcpy(h_slot_block, blk.data(), 4 * (size_t)N);
        if (h_vals)
            for (int i = 0; i < N; ++i) h_vals[i] = blk[i] >= 0 ? 1.0 : 0.0;
    } else {
        const CartDev &cd = s->cart;
        const int32_t *T = s->h_tab.data();
        const int cmap_off = (int)(cd.cmap - s->d_tab);
        for (int i = 0; i < N; ++i) {
            const int c3[3] = {i % c->nx, (i / c->nx) % c->ny, i / (c->nx * c->ny)};
            int J[3], lo[3], nv[3];
            for (int a = 0; a < 3; ++a) {
                J[a] = (int)(((long)c3[a] * cd.m[a]) / cd.n[a]);
                lo[a] = T[s->tab_off[a][0] + c3[a]];
                nv[a] = T[s->tab_off[a][1] + c3[a]];
            }
            const bool act = c->h_active[i] != 0;
            if (h_block) h_block[i] = act ? T[cmap_off + J[0] + cd.m[0] * (J[1] + cd.m[1] * J[2])] : -1;
            if (h_slot_block)
                for (int sl = 0; sl < s->ns; ++sl) {
                    int K[3];
                    bool ok = act;
                    for (int a = 0; a < 3; ++a) {
                        const int bit = cd.bit[a] >= 0 ? (sl >> cd.bit[a]) & 1 : 0;
                        if (bit >= nv[a]) ok = false;
                        K[a] = lo[a] + bit;
                    }
                    h_slot_block[(long)sl * N + i] =
                        ok ? T[cmap_off + K[0] + cd.m[0] * (K[1] + cd.m[1] * K[2])] : -1;
                }
        }
        if (h_vals) {
            double *dv = (double *)ctx_alloc(*c, 8 * (size_t)s->ns * N);
            if (!dv) return MSRSB_E_NOMEM;
            launch_export_cart(*c, *s, dv);
            e = hipStreamSynchronize(c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(h_vals, dv, 8 * (size_t)s->ns * N, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            ctx_free(*c, dv);
            if (e != hipSuccess) return hip_fail(e, "export");
        }
    }
    if (h_Ac) {
        e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy2D(h_Ac, 8 * (size_t)s->M, s->Ac, 8 * (size_t)s->Mp, 8 * (size_t)s->M, s->M,
                            hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "export A_c");
    }
    return MSRSB_OK;
}

// ------------------------------------------------ allocation-free export ----
// Staging array of msrsb_export_stage_noalloc: one slot column of a BF16
// basis widened to FP64.  Each device holds its own copy until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy: the
// name is a host-side stand-in, the device address comes from
// hipGetSymbolAddress (once per device, with that device current).
static __device__ __align__(256) double scratch[MSRSB_NOALLOC_MAX_CELLS];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_ptr;  // per device; null until resolved

static int scratch_address(int device, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        double *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return MSRSB_OK;
}

int msrsb_export_stage_noalloc(msrsb_ctx *c, int stage, int32_t *h_block, int32_t *h_slot_block, double *h_vals,
                               double *h_Ac) {
    g_err.clear();
    if (!c) return MSRSB_E_INVAL;
    Stage *s = stage_at(c, stage);
    if (!s) {
        set_error("no stage %d", stage);
        return MSRSB_E_INVAL;
    }
    const int N = c->N;
    if (N > MSRSB_NOALLOC_MAX_CELLS) {
        set_error("allocation-free export handles at most %d cells per slot (grid has %d)", MSRSB_NOALLOC_MAX_CELLS,
                  N);
        return MSRSB_E_INVAL;
    }
    hipError_t e = hipSuccess;
    if (s->kind == 3) {
        // constant basis: block per cell straight from the device, slots and
        // values derived from it on the host
        int32_t *dst = h_block ? h_block : h_slot_block;
        if (dst) {
            e = hipMemcpyAsync(dst, s->dblock, 4 * (size_t)N, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(e, "export");
            if (h_block && h_slot_block) memcpy(h_slot_block, h_block, 4 * (size_t)N);
            if (h_vals)
                for (int i = 0; i < N; ++i) h_vals[i] = dst[i] >= 0 ? 1.0 : 0.0;
        } else if (h_vals) {
            // no integer output to stage through: the values are 1 on blocks, 0 off them
            e = hipMemcpyAsync(h_vals, s->dblock, 4 * (size_t)N, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(e, "export");
            const int32_t *blk = (const int32_t *)h_vals;
            for (int i = N - 1; i >= 0; --i) h_vals[i] = blk[i] >= 0 ? 1.0 : 0.0;  // widen in place, last first
        }
    } else {
        // integer tables come from the host copies, exactly as msrsb_export_stage
        if (h_block || h_slot_block) {
            int rc = msrsb_export_stage(c, stage, h_block, h_slot_block, nullptr, nullptr);
            if (rc) return rc;
        }
        if (h_vals) {
            if (c->opt.precision == MSRSB_MIXED) {
                double *sp = nullptr;
                int rc = scratch_address(c->device, &sp);
                if (rc) return rc;
                // one slot column at a time through the staging array
                for (int sl = 0; sl < s->ns && e == hipSuccess; ++sl) {
                    launch_export_bf16(*c, s->Pbf + (size_t)sl * N, N, sp);
                    e = hipMemcpyAsync(h_vals + (size_t)sl * N, sp, 8 * (size_t)N, hipMemcpyDeviceToHost, c->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
                }
            } else {
                e = hipMemcpyAsync(h_vals, s->P64[s->cur], 8 * (size_t)s->ns * N, hipMemcpyDeviceToHost, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
            if (e == hipSuccess) e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "export");
        }
    }
    if (h_Ac) {
        e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(h_Ac, 8 * (size_t)s->M, s->Ac, 8 * (size_t)s->Mp, 8 * (size_t)s->M, s->M,
                                 hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "export A_c");
    }
    return MSRSB_OK;
}

int msrsb_coarse_apply(msrsb_ctx *c, int stage, const double *h_d, double *h_pc) {
    g_err.clear();
    if (!c || !h_d || !h_pc) {
        set_error("bad coarse-apply arguments");
        return MSRSB_E_INVAL;
    }
    Stage *s = stage_at(c, stage);
    if (!s) {
        set_error("no stage %d", stage);
        return MSRSB_E_INVAL;
    }
    if (!s->has_basis) {
        set_error("stage %d has no coarse operator yet", stage);
        return MSRSB_E_STATE;
    }
    const int M = s->M;
    hipError_t e = hipMemcpyAsync(s->dvec, h_d, 8 * (size_t)M, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "coarse apply upload");
    launch_coarse_solve(*c, *s, nullptr);
    // rectilinear stages keep p_c per Cartesian block (entry j at present[j])
    const size_t n = s->pc_map ? (size_t)s->cart.m[0] * s->cart.m[1] * s->cart.m[2] : (size_t)M;
    std::vector<double> pc(n);
    e = hipMemcpyAsync(pc.data(), s->pc, 8 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse apply");
    for (int j = 0; j < M; ++j) h_pc[j] = s->pc_map ? pc[s->h_present[j]] : pc[j];
    return MSRSB_OK;
}

int msrsb_profile_begin(msrsb_ctx *c, int kernel_class, int max_launches) {
    g_err.clear();
    if (!c || kernel_class < 1 || kernel_class > MSRSB_K_RESTRICT_ROWS || max_launches < 1 || max_launches > 1000000) {
        set_error("bad profile arguments");
        return MSRSB_E_INVAL;
    }
    const int need = 2 * max_launches;
    while ((int)c->prof_ev.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventCreate");
        c->prof_ev.push_back(e);
    }
    c->prof_used = 0;
    c->prof_class = kernel_class;
    return MSRSB_OK;
}

int msrsb_profile_end(msrsb_ctx *c, double *total_ms, int *launches) {
    g_err.clear();
    if (!c) return MSRSB_E_INVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "profile sync");
    double tot = 0.0;
    for (int k = 0; k + 1 < c->prof_used; k += 2) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->prof_ev[k], c->prof_ev[k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = c->prof_used / 2;
    c->prof_class = -1;
    c->prof_used = 0;
    return MSRSB_OK;
}

int msrsb_set_stream(msrsb_ctx *c, void *hip_stream) {
    if (!c) return MSRSB_E_INVAL;
    // work and pool allocations of the old stream complete before the switch
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set stream");
    c->stream = (hipStream_t)hip_stream;
    return MSRSB_OK;
}

void msrsb_destroy(msrsb_ctx *c) {
    if (!c) return;
    hipStreamSynchronize(c->stream);
    for (size_t k = 0; k < c->allocs.size(); ++k) {
        if (!c->ua.alloc && c->allocs[k] == (void *)c->arena &&
            arena_give(c->device, c->allocs[k], c->alloc_bytes[k]))
            continue;  // idle after the synchronisation: kept for the next set-up
        raw_free(*c, c->allocs[k], c->alloc_bytes[k]);
    }
    for (hipEvent_t e : c->prof_ev) hipEventDestroy(e);
    release_pinned_status(c->h_status);
    delete c;
}

}  // extern "C"
