// Dynamic partitions with constant basis functions (subsection "Iterative
// multiscale multibasis solver", type "Dynamic": cells are put into bins by
// the magnitude of their pressure update and agglomerated into blocks; the
// work is a few comparisons and an integer per cell).
//
// Binning: a = |dp|, thresholds ldexp(max a, -2k) for k = 1..n_bins-1 (exact
// scalings, so the bins do not depend on rounding), bin = number of
// thresholds a does not exceed.  Blocks: face-connected cells with the same
// bin inside one block of the general (stage-0) partition.  Because every
// dynamic block lies inside one general block, the connected components are
// found inside one workgroup per general block, in LDS, by min-label
// propagation with pointer jumping (the fixed point is the smallest local
// index of the component, whatever the update order).  Blocks are numbered by
// (general block, smallest cell index); the per-block cell lists are written
// in ascending cell order.
#include <algorithm>
#include <cstring>

#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

constexpr int kDynMaxBox = 6144;  // cells of one general block handled in LDS

__global__ __launch_bounds__(kBlock) void k_absmax(int N, const double *__restrict__ diag, const double *__restrict__ dp,
                                                   unsigned long long *bits, int *flag) {
    __shared__ double lds[kBlock / 64];
    double m = 0.0;
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        if (!(diag[i] > 0.0)) continue;
        const double a = fabs(dp[i]);
        if (!(a <= 1.7976931348623157e308)) bad = true;
        else m = fmax(m, a);
    }
    if (bad) atomicOr(flag, 4);
    m = block_max(m, lds);
    if (threadIdx.x == 0 && m > 0.0) atomicMax(bits, (unsigned long long)__double_as_longlong(m));
}

struct DynGeom {
    int nx, ny, nz, nxy;
    int m[3];
    const int32_t *be[3];      // general-partition block starts per axis (m+1)
    const double *tx, *ty, *tz, *diag;
};

__device__ inline void gblock_box(const DynGeom &G, int g, int b0[3], int sz[3]) {
    const int J[3] = {g % G.m[0], (g / G.m[0]) % G.m[1], g / (G.m[0] * G.m[1])};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b0[a] = G.be[a][J[a]];
        sz[a] = G.be[a][J[a] + 1] - b0[a];
    }
}

// One workgroup per Cartesian general block g (index in the full coarse box;
// blocks without active cells produce no dynamic blocks).
__global__ __launch_bounds__(kBlock) void k_dyn_label(DynGeom G, const double *__restrict__ dp, double amax, int nb,
                                                      int32_t *__restrict__ local_id, int32_t *__restrict__ count) {
    __shared__ int32_t lab[kDynMaxBox];
    __shared__ int8_t key[kDynMaxBox];
    __shared__ int32_t wsum[kBlock / 64 + 1];
    const int g = blockIdx.x;
    int b0[3], sz[3];
    gblock_box(G, g, b0, sz);
    const int V = sz[0] * sz[1] * sz[2];
    double thr[8];
    for (int k = 1; k < nb; ++k) thr[k] = ldexp(amax, -2 * k);
    for (int t = threadIdx.x; t < V; t += blockDim.x) {
        const int cx = b0[0] + t % sz[0], rem = t / sz[0];
        const int cy = b0[1] + rem % sz[1], cz = b0[2] + rem / sz[1];
        const int i = cx + G.nx * (cy + G.ny * cz);
        int8_t kk = -1;
        if (G.diag[i] > 0.0) {
            const double a = fabs(dp[i]);
            int bin = 0;
            for (int k = 1; k < nb; ++k) bin += (a <= thr[k]);
            kk = (int8_t)bin;
        }
        key[t] = kk;
        lab[t] = t;
    }
    __syncthreads();
    // min-label propagation over same-key faces inside the box
    for (;;) {
        int changed = 0;
        for (int t = threadIdx.x; t < V; t += blockDim.x) {
            const int8_t kk = key[t];
            if (kk < 0) continue;
            const int lx = t % sz[0], rem = t / sz[0];
            const int ly = rem % sz[1], lz = rem / sz[1];
            const int i = (b0[0] + lx) + G.nx * ((b0[1] + ly) + G.ny * (b0[2] + lz));
            int m = lab[t];
            if (lx + 1 < sz[0] && G.tx[i] != 0.0 && key[t + 1] == kk) m = min(m, lab[t + 1]);
            if (lx > 0 && G.tx[i - 1] != 0.0 && key[t - 1] == kk) m = min(m, lab[t - 1]);
            const int sy = sz[0], szz = sz[0] * sz[1];
            if (ly + 1 < sz[1] && G.ty[i] != 0.0 && key[t + sy] == kk) m = min(m, lab[t + sy]);
            if (ly > 0 && G.ty[i - G.nx] != 0.0 && key[t - sy] == kk) m = min(m, lab[t - sy]);
            if (lz + 1 < sz[2] && G.tz[i] != 0.0 && key[t + szz] == kk) m = min(m, lab[t + szz]);
            if (lz > 0 && G.tz[i - G.nxy] != 0.0 && key[t - szz] == kk) m = min(m, lab[t - szz]);
            m = min(m, lab[m]);  // pointer jump: lab[m] is a member of the same component
            if (m < lab[t]) {
                lab[t] = m;
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    // roots (lab[t] == t) numbered in ascending local index = ascending cell index
    const int per = (V + blockDim.x - 1) / blockDim.x;
    const int t0 = threadIdx.x * per, t1 = min(V, t0 + per);
    int cnt = 0;
    for (int t = t0; t < t1; ++t) cnt += (key[t] >= 0 && lab[t] == t);
    // exclusive scan of cnt over threads (fixed order)
    __shared__ int32_t tc[kBlock];
    tc[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < (int)blockDim.x; ++k) {
            const int v = tc[k];
            tc[k] = run;
            run += v;
        }
        wsum[0] = run;
    }
    __syncthreads();
    // rank roots: store the id in lab of the root as a negative marker
    int run = tc[threadIdx.x];
    __shared__ int32_t rid[kDynMaxBox];
    for (int t = t0; t < t1; ++t) {
        rid[t] = -1;
        if (key[t] >= 0 && lab[t] == t) rid[t] = run++;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < V; t += blockDim.x) {
        const int cx = b0[0] + t % sz[0], rem = t / sz[0];
        const int cy = b0[1] + rem % sz[1], cz = b0[2] + rem / sz[1];
        const int i = cx + G.nx * (cy + G.ny * cz);
        local_id[i] = key[t] >= 0 ? rid[lab[t]] : -1;
    }
    if (threadIdx.x == 0) count[g] = wsum[0];
}

// Exclusive scan of the per-general-block counts (single workgroup, fixed order).
__global__ void k_dyn_scan(int M0, const int32_t *__restrict__ count, int32_t *__restrict__ off, Status *st) {
    if (threadIdx.x != 0) return;
    int run = 0;
    for (int g = 0; g < M0; ++g) {
        off[g] = run;
        run += count[g];
    }
    off[M0] = run;
    st->iters = run;
}

// Final block ids, per-block cell lists (ascending cell order) and CSR offsets.
// One 64-lane workgroup per general block; gbase[g] = active cells before g.
__global__ __launch_bounds__(64) void k_dyn_place(DynGeom G, const int32_t *__restrict__ local_id,
                                                  const int32_t *__restrict__ off, const int32_t *__restrict__ gbase,
                                                  int32_t *__restrict__ block, int32_t *__restrict__ cells,
                                                  int32_t *__restrict__ ptr, int M0) {
    __shared__ int32_t cnt[kDynMaxBox];
    const int g = blockIdx.x, lane = threadIdx.x;
    int b0[3], sz[3];
    gblock_box(G, g, b0, sz);
    const int V = sz[0] * sz[1] * sz[2];
    const int nid = off[g + 1] - off[g];
    for (int k = lane; k < nid; k += 64) cnt[k] = 0;
    __syncthreads();
    for (int t = lane; t < V; t += 64) {
        const int cx = b0[0] + t % sz[0], rem = t / sz[0];
        const int cy = b0[1] + rem % sz[1], cz = b0[2] + rem / sz[1];
        const int i = cx + G.nx * (cy + G.ny * cz);
        const int id = local_id[i];
        if (id >= 0) atomicAdd(&cnt[id], 1);
    }
    __syncthreads();
    if (lane == 0) {
        int run = 0;
        for (int k = 0; k < nid; ++k) {
            const int v = cnt[k];
            cnt[k] = run;
            ptr[off[g] + k] = gbase[g] + run;
            run += v;
        }
        if (g == M0 - 1) ptr[off[M0]] = gbase[M0];
    }
    __syncthreads();
    // stable placement in chunks of 64 cells
    for (int base = 0; base < V; base += 64) {
        const int t = base + lane;
        int id = -1, i = 0;
        if (t < V) {
            const int cx = b0[0] + t % sz[0], rem = t / sz[0];
            const int cy = b0[1] + rem % sz[1], cz = b0[2] + rem / sz[1];
            i = cx + G.nx * (cy + G.ny * cz);
            id = local_id[i];
            if (id >= 0) block[i] = off[g] + id;
        }
        unsigned long long pending = __ballot(id >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int lid = __shfl(id, leader, 64);
            const unsigned long long same = __ballot(id == lid);
            const unsigned long long lower = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            if (id == lid) cells[gbase[g] + cnt[lid] + __popcll(same & lower)] = i;
            __syncthreads();
            if (lane == leader) cnt[lid] += __popcll(same);
            __syncthreads();
            pending &= ~same;
        }
    }
}

__global__ void k_fill_i32(long n, int32_t *p, int32_t v) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Row j of the coarse two-point operator of a constant basis:
//   A_c[j,k] = -sum of T over faces between blocks j and k (k != j),
//   A_c[j,j] = sum of T over faces leaving j + sum of bc on j.
// One wavefront per row walks the row's cells in order; every sum is a
// fixed-shape wave reduction added in a fixed sequence.
__global__ __launch_bounds__(64) void k_dyn_rap(DynGeom G, const int32_t *__restrict__ block,
                                                const int32_t *__restrict__ cells, const int32_t *__restrict__ ptr,
                                                const double *__restrict__ bcdiag, double *__restrict__ Ac, int Mp) {
    const int j = blockIdx.x, lane = threadIdx.x;
    const int c0 = ptr[j], c1 = ptr[j + 1];
    double dsum = 0.0;  // lane 0 only
    for (int base = c0; base < c1; base += 64) {
        const int p = base + lane;
        int i = -1;
        if (p < c1) i = cells[p];
        double di = 0.0;
        int nk[6];
        double nt[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            nk[q] = -1;
            nt[q] = 0.0;
        }
        if (i >= 0) {
            di = bcdiag[i];
            const int step[3] = {1, G.nx, G.nxy};
            const double *Ta[3] = {G.tx, G.ty, G.tz};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int a = q >> 1;
                int l;
                double T;
                if (q & 1) {
                    T = Ta[a][i];
                    l = i + step[a];
                } else {
                    if (i < step[a]) continue;
                    l = i - step[a];
                    T = Ta[a][l];
                }
                if (T == 0.0) continue;
                const int k = block[l];
                if (k != j) {
                    di += T;
                    nk[q] = k;
                    nt[q] = T;
                }
            }
        }
        const double ds = wave_sum(di);
        if (lane == 0) dsum += ds;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            int mine = nk[q];
            unsigned long long pending = __ballot(mine >= 0);
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const int kk = __shfl(mine, leader, 64);
                const unsigned long long same = __ballot(mine == kk);
                const double s = wave_sum(mine == kk ? nt[q] : 0.0);
                if (lane == 0) Ac[(long)j * Mp + kk] -= s;
                pending &= ~same;
            }
        }
    }
    if (lane == 0) Ac[(long)j * Mp + j] = dsum;
}

__global__ __launch_bounds__(kBlock) void k_dyn_restrict(const int32_t *__restrict__ cells, const int32_t *__restrict__ ptr,
                                                         const double *__restrict__ r, double *__restrict__ d,
                                                         const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    const int j = blockIdx.x;
    const int p0 = ptr[j], p1 = ptr[j + 1];
    // thread t adds the cells p0 + t, p0 + t + 256, ... in order, eight at a
    // time with all index loads, then all value loads, in flight (entries past
    // the block repeat the first one of the batch and are multiplied by zero)
    double acc = 0.0;
    for (int pb = p0 + threadIdx.x; pb < p1; pb += 8 * blockDim.x) {
        int ci[8];
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = pb + q * blockDim.x;
            ci[q] = cells[p < p1 ? p : pb];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = r[ci[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q] * (pb + q * (int)blockDim.x < p1 ? 1.0 : 0.0);
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) d[j] = s;
}

__global__ void k_dyn_prolong(int N, const int32_t *__restrict__ block, const double *__restrict__ pc,
                              double *__restrict__ x, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = block[i];
    if (b >= 0) x[i] += pc[b];
}

void launch_dyn_restrict(Ctx &c, Stage &s, const double *r, const int *done) {
    hipLaunchKernelGGL(k_dyn_restrict, dim3(s.M), dim3(kBlock), 0, c.stream, s.dcells, s.dptr, r, s.dvec, done);
}

void launch_dyn_prolong(Ctx &c, Stage &s, double *x, const int *done) {
    hipLaunchKernelGGL(k_dyn_prolong, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, s.dblock, s.pc, x,
                       done);
}

static DynGeom geom_of(Ctx &c) {
    const Stage &s0 = c.stages[0];
    DynGeom G;
    G.nx = c.nx; G.ny = c.ny; G.nz = c.nz; G.nxy = c.nx * c.ny;
    for (int a = 0; a < 3; ++a) {
        G.m[a] = s0.cart.m[a];
        G.be[a] = s0.cart.be[a];
    }
    G.tx = c.tx; G.ty = c.ty; G.tz = c.tz; G.diag = c.diag;
    return G;
}

void launch_dyn_rap(Ctx &c, Stage &s) {
    DynGeom G = geom_of(c);
    hipMemsetAsync(s.Ac, 0, sizeof(double) * (size_t)s.Mp * s.Mp, c.stream);
    hipLaunchKernelGGL(k_dyn_rap, dim3(s.M), dim3(64), 0, c.stream, G, s.dblock, s.dcells, s.dptr, c.bcdiag, s.Ac,
                       s.Mp);
    launch_symmetrize(c, s.Ac, s.M, s.Mp);
}

static int sync_read(Ctx &c, void *dst, const void *src, size_t n) {
    hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "device read");
    return MSRSB_OK;
}


// Build the partition of one dynamic stage into `out` (buffers grown as
// needed).  *count = number of blocks (0: no stage).
int build_dynamic_stage(Ctx &c, const double *dp, Stage &out, int *count) {
    Stage &s0 = c.stages[0];
    const int M0 = s0.cart.m[0] * s0.cart.m[1] * s0.cart.m[2];
    DynGeom G = geom_of(c);
    // workspace: local ids [N] in c.u (reinterpret), counts/offsets in c.tmp
    int32_t *local_id = (int32_t *)c.u;
    int32_t *counts = (int32_t *)c.z;
    int32_t *offs = counts + M0 + 1;
    hipMemsetAsync(c.maxbits, 0, sizeof(unsigned long long), c.stream);
    hipMemsetAsync(c.flag, 0, sizeof(int), c.stream);
    hipLaunchKernelGGL(k_absmax, dim3(std::min(kRedBlocks, cdiv(c.N, kBlock))), dim3(kBlock), 0, c.stream, c.N, c.diag,
                       dp, c.maxbits, c.flag);
    unsigned long long bits = 0;
    int flag = 0, rc;
    if ((rc = sync_read(c, &bits, c.maxbits, sizeof(bits)))) return rc;
    if ((rc = sync_read(c, &flag, c.flag, sizeof(flag)))) return rc;
    double amax;
    memcpy(&amax, &bits, sizeof(double));
    *count = 0;
    if ((flag & 4) || !(amax > 0.0)) return MSRSB_OK;
    int nb = c.opt.n_bins;
    int total = 0;
    for (;;) {
        hipLaunchKernelGGL(k_dyn_label, dim3(M0), dim3(kBlock), 0, c.stream, G, dp, amax, nb, local_id, counts);
        hipLaunchKernelGGL(k_dyn_scan, dim3(1), dim3(1), 0, c.stream, M0, counts, offs, c.status);
        Status st;
        if ((rc = sync_read(c, &st, c.status, sizeof(Status)))) return rc;
        total = st.iters;
        if (total <= c.opt.max_dyn_blocks) break;
        if (nb == 1) {
            set_error("dynamic partition has %d blocks with one bin, more than max_dyn_blocks = %d", total,
                      c.opt.max_dyn_blocks);
            return MSRSB_E_INVAL;
        }
        nb /= 2;
    }
    // (re)allocate the stage buffers
    const int Mp = cdiv(total, kTile) * kTile;
    if (!out.dblock) {
        out.dblock = (int32_t *)ctx_alloc(c, sizeof(int32_t) * (size_t)c.N);
        out.dcells = (int32_t *)ctx_alloc(c, sizeof(int32_t) * (size_t)std::max(c.n_active, 1));
        if (!out.dblock || !out.dcells) return MSRSB_E_NOMEM;
    }
    if (Mp > out.Mp) {
        // the smaller buffers of an earlier increment go back to the pool
        for (void *p : {(void *)out.dptr, (void *)out.Ac, (void *)out.Ainv, (void *)out.dvec, (void *)out.pc})
            ctx_free(c, p);
        out.dptr = (int32_t *)ctx_alloc(c, sizeof(int32_t) * (size_t)(Mp + 1));
        out.Ac = (double *)ctx_alloc(c, sizeof(double) * (size_t)Mp * Mp);
        out.Ainv = (double *)ctx_alloc(c, sizeof(double) * (size_t)Mp * Mp);
        out.dvec = (double *)ctx_alloc(c, sizeof(double) * (size_t)Mp);
        out.pc = (double *)ctx_alloc(c, sizeof(double) * (size_t)Mp);
        if (!out.dptr || !out.Ac || !out.Ainv || !out.dvec || !out.pc) return MSRSB_E_NOMEM;
        out.Mp = Mp;
    }
    out.kind = 3;
    out.M = total;
    out.ns = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, (long)c.N, out.dblock, -1);
    hipLaunchKernelGGL(k_dyn_place, dim3(M0), dim3(64), 0, c.stream, G, local_id, offs, s0.gbase, out.dblock,
                       out.dcells, out.dptr, M0);
    *count = total;
    return MSRSB_OK;
}

}  // namespace msrsb
