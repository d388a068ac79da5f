// Finite-volume restriction and conservative flux reconstruction (section
// "Multiscale methods": for fine-scale fluxes, a restriction that sums the
// cells of each block instead of R = P^T).
//
//   A_fv = R_fv A P     R_fv[j, i] = 1 for i in block j
//   p_ms = P A_fv^{-1} R_fv b
// Summed over a block, b - A p_ms vanishes, so the fluxes of p_ms across block
// boundaries balance each block.  Inside every block the fine pressure p' then
// solves the block's own problem with those boundary fluxes imposed (a
// Neumann problem: faces to other blocks carry T (p_ms,i - p_ms,l)):
//   sum_{l in block} T_il (p'_i - p'_l) + bc_i p'_i = b_i - sum_{l not in block} T_il (p_ms,i - p_ms,l)
// and the fluxes T (p'_a - p'_b) inside blocks, T (p_ms,a - p_ms,b) between
// blocks and bc (p'_i - p_bc) balance every cell.
#include <algorithm>

#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

// Row j of A_fv: over the block's own cells a, sum_k of bc_a P_ak plus, for
// every face (a, l) leaving the block, T (P_ak - P_lk).  (Faces inside the
// block add T (P_ak - P_lk) from a and the opposite from l, so they cancel.)
// One wavefront per chunk of the block's cell list; contributions of a
// wavefront step are summed per column by fixed-shape wave reductions in a
// fixed order; blocks of several chunks write partial rows.
template <typename PS>
__global__ __launch_bounds__(64) void k_fv_rap(Fine g, int ns, const int32_t *__restrict__ sb,
                                               const int32_t *__restrict__ fvblock, const int32_t *__restrict__ ptr,
                                               const int32_t *__restrict__ rcblk, const int32_t *__restrict__ rcfirst,
                                               const int32_t *__restrict__ rrow, const int32_t *__restrict__ cells,
                                               const PS *__restrict__ P, const double *__restrict__ bcdiag,
                                               double *__restrict__ A, double *__restrict__ rpart, int Mp) {
    const int ch = blockIdx.x, j = rcblk[ch], lane = threadIdx.x;
    const long N = g.N;
    double *row = rrow[ch] >= 0 ? rpart + (long)rrow[ch] * Mp : A + (long)j * Mp;
    const int k0 = ptr[j] + (ch - rcfirst[j]) * kXRapChunk, k1 = min(k0 + kXRapChunk, ptr[j + 1]);
    auto commit = [&](int kb, double v) {
        unsigned long long pending = __ballot(kb >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int kk = __shfl(kb, leader, 64);
            const unsigned long long same = __ballot(kb == kk);
            const double sum = wave_sum(kb == kk ? v : 0.0);
            if (lane == 0) row[kk] += sum;
            pending &= ~same;
        }
    };
    for (int base = k0; base < k1; base += 64) {
        const int k = base + lane;
        const bool live = k < k1;
        const int a = live ? cells[k] : 0;
        const double bc = live ? bcdiag[a] : 0.0;
        for (int t = 0; t < ns; ++t) {
            const int kb = live && bc > 0.0 ? sb[(long)t * N + a] : -1;
            commit(kb, kb >= 0 ? bc * ld_basis(P, (long)t * N + a) : 0.0);
        }
        for (int q = 0; q < 6; ++q) {
            const int ax = q >> 1;
            const int step = ax == 0 ? 1 : (ax == 1 ? g.nx : g.nxy);
            const double *Ta = ax == 0 ? g.tx : (ax == 1 ? g.ty : g.tz);
            int l = -1;
            double T = 0.0;
            if (live) {
                if (q & 1) {
                    T = Ta[a];
                    l = a + step;
                } else if (a >= step) {
                    l = a - step;
                    T = Ta[l];
                }
            }
            const bool out = T != 0.0 && fvblock[l] != j;
            for (int t = 0; t < ns; ++t) {
                const int kb = out ? sb[(long)t * N + a] : -1;
                commit(kb, kb >= 0 ? T * ld_basis(P, (long)t * N + a) : 0.0);
            }
            for (int t = 0; t < ns; ++t) {
                const int kb = out ? sb[(long)t * N + l] : -1;
                commit(kb, kb >= 0 ? -T * ld_basis(P, (long)t * N + l) : 0.0);
            }
        }
    }
}

// d_j = sum of b over block j's cells (one wavefront per block, fixed order).
__global__ __launch_bounds__(64) void k_fv_restrict(int M, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ cells, const double *__restrict__ b,
                                                    double *__restrict__ d) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int k = ptr[j] + threadIdx.x; k < ptr[j + 1]; k += 64) s += b[cells[k]];
    s = wave_sum(s);
    if (threadIdx.x == 0) d[j] = s;
}

// Sum over the workgroup, the same value returned to every thread (waves
// added in index order).  lds: blockDim/64 doubles.
__device__ inline double block_allsum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) s += lds[k];
    return s;
}

constexpr int kFvThreads = 1024;

// The block's Neumann problem by Jacobi-preconditioned conjugate gradients,
// one workgroup per block, from p' = p_ms.  The search direction lives in LDS
// by list position, so neighbours inside the block are read there (their
// position from loc); the iterate, residual and A p of a cell live in global
// vectors that only the thread owning the cell (list positions t, t + 1024,
// ...) reads and writes.  Stops when ||r|| <= rtol ||rhs|| (every thread
// takes the same decision from the same sums) or after max_iters.  Cells
// with neither an in-block face nor a boundary term keep p_ms.
__global__ __launch_bounds__(kFvThreads) void k_fv_local(Fine g, const int32_t *__restrict__ fvblock,
                                                         const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ cells,
                                                         const int32_t *__restrict__ loc,
                                                         const double *__restrict__ bcdiag,
                                                         const double *__restrict__ b, const double *__restrict__ pms,
                                                         double *__restrict__ x, double *__restrict__ r,
                                                         double *__restrict__ q, double rtol, int max_iters,
                                                         int *iters_max) {
    extern __shared__ double pl[];  // [n] by list position
    __shared__ double red[kFvThreads / 64];
    const int j = blockIdx.x;
    const int c0 = ptr[j], n = ptr[j + 1] - c0;
    const int step[3] = {1, g.nx, g.nxy};
    const double *Ta[3] = {g.tx, g.ty, g.tz};
    // diagonal of the block's operator (in-block faces and boundary terms)
    // and, with `ext`, the flux of p_ms through the faces leaving the block
    auto diag_of = [&](int i, double *ext) {
        double d = bcdiag[i], e = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double tu = Ta[a][i];
            if (tu != 0.0) {
                if (fvblock[i + step[a]] == j) d += tu;
                else e += tu * (pms[i] - pms[i + step[a]]);
            }
            if (i >= step[a]) {
                const double td = Ta[a][i - step[a]];
                if (td != 0.0) {
                    if (fvblock[i - step[a]] == j) d += td;
                    else e += td * (pms[i] - pms[i - step[a]]);
                }
            }
        }
        if (ext) *ext = e;
        return d;
    };
    // (A_block v)_i with v held in pl
    auto apply = [&](int i, double d, double own) {
        double y = d * own;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double tu = Ta[a][i];
            if (tu != 0.0 && fvblock[i + step[a]] == j) y -= tu * pl[loc[i + step[a]]];
            if (i >= step[a]) {
                const double td = Ta[a][i - step[a]];
                if (td != 0.0 && fvblock[i - step[a]] == j) y -= td * pl[loc[i - step[a]]];
            }
        }
        return y;
    };
    // x = p_ms, r = rhs (for now), pl = x
    double rhs2 = 0.0;
    for (int k = threadIdx.x; k < n; k += kFvThreads) {
        const int i = cells[c0 + k];
        double ext;
        (void)diag_of(i, &ext);
        const double rh = b[i] - ext;
        x[i] = pms[i];
        r[i] = rh;
        rhs2 += rh * rh;
        pl[k] = pms[i];
    }
    rhs2 = block_allsum(rhs2, red);  // its leading barrier publishes pl
    // A block without boundary or well terms has a singular operator whose
    // null space is the constant (blocks are face-connected): its residuals
    // are kept at zero sum (the range of the operator), which removes the
    // rounding-level inconsistency a recomputed residual would carry along
    // the null space.
    double nb = 0.0;
    for (int k = threadIdx.x; k < n; k += kFvThreads) nb += bcdiag[cells[c0 + k]] > 0.0 ? 1.0 : 0.0;
    const bool anchored = block_allsum(nb, red) > 0.0;
    double rz = 0.0, rr = 0.0;
    // after r is written: zero block sum if unanchored, then rz = (r, D^-1 r), rr = (r, r)
    auto finish_residual = [&]() {
        if (!anchored) {
            double sum = 0.0;
            for (int k = threadIdx.x; k < n; k += kFvThreads) sum += r[cells[c0 + k]];
            const double mean = block_allsum(sum, red) / n;
            for (int k = threadIdx.x; k < n; k += kFvThreads) r[cells[c0 + k]] -= mean;
        }
        double rzt = 0.0, rrt = 0.0;
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            const double d = diag_of(i, nullptr);
            const double rv = r[i];
            rzt += rv * (d > 0.0 ? rv / d : 0.0);
            rrt += rv * rv;
        }
        rz = block_allsum(rzt, red);
        rr = block_allsum(rrt, red);
    };
    // r = rhs - A x
    for (int k = threadIdx.x; k < n; k += kFvThreads) {
        const int i = cells[c0 + k];
        const double d = diag_of(i, nullptr);
        r[i] -= apply(i, d, pl[k]);
    }
    finish_residual();  // every read of pl above came before its barriers
    for (int k = threadIdx.x; k < n; k += kFvThreads) {
        const int i = cells[c0 + k];
        const double d = diag_of(i, nullptr);
        pl[k] = d > 0.0 ? r[i] / d : 0.0;  // p = z
    }
    __syncthreads();
    const double stop2 = rtol * rtol * rhs2;
    // When the updated residual meets the tolerance, the true residual
    // rhs - A x is formed (pl holds x meanwhile) and, unless it meets the
    // tolerance too or fell by less than half since the last such check (the
    // attainable accuracy is reached), conjugate gradients restart from x
    // with it.  Continuing with the old direction after replacing the
    // residual is unstable once the updated residual has run far below the
    // true one.
    auto true_residual = [&]() {
        __syncthreads();  // every read of pl of the step is done
        for (int k = threadIdx.x; k < n; k += kFvThreads) pl[k] = x[cells[c0 + k]];
        __syncthreads();
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            double ext;
            const double d = diag_of(i, &ext);
            r[i] = (b[i] - ext) - apply(i, d, pl[k]);
        }
        finish_residual();  // every read of pl above came before its barriers
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            const double d = diag_of(i, nullptr);
            pl[k] = d > 0.0 ? r[i] / d : 0.0;  // restart: p = z
        }
        __syncthreads();
    };
    int it = 0;
    double prev = INFINITY;
    for (;;) {
        if (rr <= stop2) {
            true_residual();
            if (rr <= stop2 || rr > 0.25 * prev) break;
            prev = rr;
        }
        if (!(it < max_iters && rz > 0.0)) break;
        double pq = 0.0;
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            const double pv = pl[k];
            const double qv = apply(i, diag_of(i, nullptr), pv);
            q[i] = qv;
            pq += pv * qv;
        }
        pq = block_allsum(pq, red);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        double rzn = 0.0, rrn = 0.0;
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            const double d = diag_of(i, nullptr);
            x[i] += alpha * pl[k];
            const double rv = r[i] - alpha * q[i];
            r[i] = rv;
            const double zv = d > 0.0 ? rv / d : 0.0;
            rzn += rv * zv;
            rrn += rv * rv;
        }
        rzn = block_allsum(rzn, red);
        rr = block_allsum(rrn, red);  // every read of pl in this step came before these barriers
        const double beta = rzn / rz;
        rz = rzn;
        for (int k = threadIdx.x; k < n; k += kFvThreads) {
            const int i = cells[c0 + k];
            const double d = diag_of(i, nullptr);
            pl[k] = (d > 0.0 ? r[i] / d : 0.0) + beta * pl[k];
        }
        __syncthreads();  // the new direction is visible before the next step reads it
        ++it;
    }
    if (threadIdx.x == 0) atomicMax(iters_max, it);
}

// The same Neumann problems for blocks of at most kFvLineCells cells, by
// conjugate gradients preconditioned with the block's z lines: M = D - L_z -
// U_z (D the block operator's diagonal, L_z, U_z its couplings along z), whose
// inverse is a tridiagonal solve per chain of cells linked along +z inside
// the block.  The strong vertical coupling of layered models then sits in the
// preconditioner.  Chains are factored once per launch (pivots p_k = (1 +
// 2^-10) d_k - t_{k-1}^2 / p_{k-1}: the slightly raised diagonal keeps every
// pivot positive, also on a chain that is a whole singular Neumann block);
// 1/p and t/p are kept in FP32 (a fixed preconditioner; its application runs
// in FP64).  Each thread owns the list positions t, t + 1024, t + 2048 and
// keeps their diagonal, right-hand side, iterate and residual in registers;
// LDS holds the search direction, the preconditioner's work vector, the
// factors and the chain links (next and previous position, head flag), 28
// bytes per cell.  The owner of a chain's lowest cell walks it forward and
// back.  Stopping, restarts and the zero-sum treatment of unanchored blocks
// are those of k_fv_local.
constexpr int kFvLineCells = 2304;
constexpr int kFvOwn = (kFvLineCells + kFvThreads - 1) / kFvThreads;

__global__ __launch_bounds__(kFvThreads) void k_fv_local_line(Fine g, const int32_t *__restrict__ fvblock,
                                                              const int32_t *__restrict__ ptr,
                                                              const int32_t *__restrict__ cells,
                                                              const int32_t *__restrict__ loc,
                                                              const double *__restrict__ bcdiag,
                                                              const double *__restrict__ b,
                                                              const double *__restrict__ pms, double *__restrict__ xout,
                                                              double rtol, int max_iters, int *iters_max) {
    extern __shared__ double smem[];
    __shared__ double red[kFvThreads / 64];
    const int j = blockIdx.x;
    const int c0 = ptr[j], n = ptr[j + 1] - c0;
    double *pl = smem, *zl = smem + n;
    float *fip = (float *)(smem + 2 * n), *fe = fip + n;
    int32_t *lnk = (int32_t *)(fe + n);  // next + 1 | (prev + 1) << 12 | head << 24
    const int step[3] = {1, g.nx, g.nxy};
    const double *Ta[3] = {g.tx, g.ty, g.tz};
    auto diag_of = [&](int i, double *ext) {
        double d = bcdiag[i], e = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double tu = Ta[a][i];
            if (tu != 0.0) {
                if (fvblock[i + step[a]] == j) d += tu;
                else e += tu * (pms[i] - pms[i + step[a]]);
            }
            if (i >= step[a]) {
                const double td = Ta[a][i - step[a]];
                if (td != 0.0) {
                    if (fvblock[i - step[a]] == j) d += td;
                    else e += td * (pms[i] - pms[i - step[a]]);
                }
            }
        }
        *ext = e;
        return d;
    };
    auto apply = [&](int i, double d, double own) {
        double y = d * own;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double tu = Ta[a][i];
            if (tu != 0.0 && fvblock[i + step[a]] == j) y -= tu * pl[loc[i + step[a]]];
            if (i >= step[a]) {
                const double td = Ta[a][i - step[a]];
                if (td != 0.0 && fvblock[i - step[a]] == j) y -= td * pl[loc[i - step[a]]];
            }
        }
        return y;
    };
    int ci[kFvOwn];
    double dg[kFvOwn], rh[kFvOwn], xr[kFvOwn], rv[kFvOwn];
    double rhs2 = 0.0, nb = 0.0;
#pragma unroll
    for (int u = 0; u < kFvOwn; ++u) {
        const int k = threadIdx.x + u * kFvThreads;
        ci[u] = 0;
        dg[u] = rh[u] = xr[u] = rv[u] = 0.0;
        if (k >= n) continue;
        const int i = cells[c0 + k];
        ci[u] = i;
        double ext;
        dg[u] = diag_of(i, &ext);
        rh[u] = b[i] - ext;
        xr[u] = pms[i];
        rhs2 += rh[u] * rh[u];
        nb += bcdiag[i] > 0.0 ? 1.0 : 0.0;
        pl[k] = pms[i];
        // the chain link along +z and the head flag (no link from below)
        int nx = -1, pv = -1;
        double t = 0.0;
        if (g.tz[i] != 0.0 && fvblock[i + g.nxy] == j) {
            nx = loc[i + g.nxy];
            t = g.tz[i];
        }
        if (i >= g.nxy && g.tz[i - g.nxy] != 0.0 && fvblock[i - g.nxy] == j) pv = loc[i - g.nxy];
        lnk[k] = (nx + 1) | ((pv + 1) << 12) | (pv < 0 ? 1 << 24 : 0);
        zl[k] = dg[u];
        fe[k] = (float)t;  // the link's T until the factorisation replaces it by t / p
    }
    rhs2 = block_allsum(rhs2, red);  // its barriers publish pl, zl, fe and lnk
    const bool anchored = block_allsum(nb, red) > 0.0;
    auto next_of = [&](int k) { return (lnk[k] & 0xfff) - 1; };
    auto prev_of = [&](int k) { return ((lnk[k] >> 12) & 0xfff) - 1; };
    // factor every chain (zl holds d, fe the link T)
#pragma unroll
    for (int u = 0; u < kFvOwn; ++u) {
        const int k = threadIdx.x + u * kFvThreads;
        if (k >= n || !(lnk[k] >> 24)) continue;
        double pprev = 0.0, tprev = 0.0;
        for (int kk = k; kk >= 0; kk = next_of(kk)) {
            const double d = zl[kk], t = fe[kk];
            const double p = (1.0 + 0x1p-10) * d - (pprev > 0.0 ? tprev * tprev / pprev : 0.0);
            const double ip = p > 0.0 ? 1.0 / p : 0.0;
            fip[kk] = (float)ip;
            fe[kk] = (float)(t * ip);
            pprev = p;
            tprev = t;
        }
    }
    __syncthreads();
    // z = M^-1 r in zl (the owners wrote r there): forward y_k = r_k +
    // (t/p)_{k-1} y_{k-1}, w_k = y_k / p_k; backward z_k = w_k + (t/p)_k z_{k+1}
    auto precond = [&]() {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k >= n || !(lnk[k] >> 24)) continue;
            double y = 0.0, eprev = 0.0;
            int tail = k;
            for (int kk = k; kk >= 0; kk = next_of(kk)) {
                y = zl[kk] + eprev * y;
                zl[kk] = y * (double)fip[kk];
                eprev = (double)fe[kk];
                tail = kk;
            }
            double z = 0.0;
            for (int kk = tail; kk >= 0; kk = prev_of(kk)) {
                z = zl[kk] + (double)fe[kk] * z;
                zl[kk] = z;
            }
        }
        __syncthreads();
    };
    double rz = 0.0, rr = 0.0;
    // after rv holds a residual: zero block sum if unanchored, z = M^-1 r,
    // rz = (r, z), rr = (r, r)
    auto finish_residual = [&]() {
        if (!anchored) {
            double sum = 0.0;
#pragma unroll
            for (int u = 0; u < kFvOwn; ++u) sum += threadIdx.x + u * kFvThreads < n ? rv[u] : 0.0;
            const double mean = block_allsum(sum, red) / n;
#pragma unroll
            for (int u = 0; u < kFvOwn; ++u) rv[u] -= mean;
        }
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k < n) zl[k] = rv[u];
        }
        precond();
        double rzt = 0.0, rrt = 0.0;
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k >= n) continue;
            rzt += rv[u] * zl[k];
            rrt += rv[u] * rv[u];
        }
        rz = block_allsum(rzt, red);
        rr = block_allsum(rrt, red);
    };
    // r = rhs - A x, p = z (pl holds x = p_ms)
    auto true_residual = [&]() {
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k < n) rv[u] = rh[u] - apply(ci[u], dg[u], pl[k]);
        }
        finish_residual();  // every read of pl above came before its barriers
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k < n) pl[k] = zl[k];
        }
        __syncthreads();
    };
    true_residual();
    const double stop2 = rtol * rtol * rhs2;
    int it = 0;
    double prev = INFINITY;
    for (;;) {
        if (rr <= stop2) {
            __syncthreads();  // every read of pl of the step is done
#pragma unroll
            for (int u = 0; u < kFvOwn; ++u) {
                const int k = threadIdx.x + u * kFvThreads;
                if (k < n) pl[k] = xr[u];
            }
            __syncthreads();
            true_residual();
            if (rr <= stop2 || rr > 0.25 * prev) break;
            prev = rr;
        }
        if (!(it < max_iters && rz > 0.0)) break;
        double pq = 0.0, qv[kFvOwn];
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            qv[u] = 0.0;
            if (k >= n) continue;
            qv[u] = apply(ci[u], dg[u], pl[k]);
            pq += pl[k] * qv[u];
        }
        pq = block_allsum(pq, red);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        double rrn = 0.0;
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k >= n) continue;
            xr[u] += alpha * pl[k];
            rv[u] -= alpha * qv[u];
            rrn += rv[u] * rv[u];
            zl[k] = rv[u];
        }
        rr = block_allsum(rrn, red);  // every read of pl in this step came before these barriers
        precond();
        double rzn = 0.0;
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k < n) rzn += rv[u] * zl[k];
        }
        rzn = block_allsum(rzn, red);
        const double beta = rzn / rz;
        rz = rzn;
#pragma unroll
        for (int u = 0; u < kFvOwn; ++u) {
            const int k = threadIdx.x + u * kFvThreads;
            if (k < n) pl[k] = zl[k] + beta * pl[k];
        }
        __syncthreads();  // the new direction is visible before the next step reads it
        ++it;
    }
#pragma unroll
    for (int u = 0; u < kFvOwn; ++u)
        if (threadIdx.x + u * kFvThreads < n) xout[ci[u]] = xr[u];
    if (threadIdx.x == 0) atomicMax(iters_max, it);
}

// Face fluxes of the reconstruction (layout of msrsb_fluxes): inside a block
// from p', between blocks from p_ms.
__global__ void k_fv_faces(Fine g, const int32_t *__restrict__ fvblock, const double *__restrict__ pms,
                           const double *__restrict__ pf, double *__restrict__ face) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    const int step[3] = {1, g.nx, g.nxy};
    const double *Ta[3] = {g.tx, g.ty, g.tz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double T = Ta[a][i];
        double v = 0.0;
        if (T != 0.0) {
            const int l = i + step[a];
            v = fvblock[i] == fvblock[l] ? T * (pf[i] - pf[l]) : T * (pms[i] - pms[l]);
        }
        face[(long)a * g.N + i] = v;
    }
}

// Largest per-cell imbalance |out-flow - q_i| of the fluxes (face fluxes,
// boundary/well terms from p'), as the bit pattern of a non-negative double
// (order-independent maximum).
__global__ void k_fv_imbalance(Fine g, const double *__restrict__ face, const double *__restrict__ pf,
                               const double *__restrict__ bcdiag, const double *__restrict__ bcrhs,
                               const double *__restrict__ src, unsigned long long *maxbits) {
    __shared__ double lds[kBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < g.N && g.diag[i] > 0.0) {
        const int step[3] = {1, g.nx, g.nxy};
        double out = bcdiag[i] * pf[i] - bcrhs[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out += face[(long)a * g.N + i];
            if (i >= step[a]) out -= face[(long)a * g.N + i - step[a]];
        }
        e = fabs(out - src[i]);
    }
    const double m = block_max(e, lds);
    if (threadIdx.x == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
}

void launch_partial_rows_finish(Ctx &c, int M, int Mp, const int32_t *rcfirst, const int32_t *rrow,
                                const double *rpart, double *A);
void launch_pad_identity(Ctx &c, double *A, int M, int Mp);

void launch_fv_rap(Ctx &c, Stage &s) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    hipMemsetAsync(s.Afv, 0, sizeof(double) * (size_t)s.Mp * s.Mp, c.stream);
    if (s.nfvrrow > 0) hipMemsetAsync(s.fvrpart, 0, sizeof(double) * (size_t)s.nfvrrow * s.Mp, c.stream);
    const int32_t *sb = s.kind == 2 ? s.xsb : s.fvsb;
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_fv_rap<uint16_t>, dim3(s.nfvrch), dim3(64), 0, c.stream, g, s.ns, sb, s.fvblock, s.fvptr,
                           s.fvrcblk, s.fvrcfirst, s.fvrrow, s.fvcells, s.Pbf, c.bcdiag, s.Afv, s.fvrpart, s.Mp);
    else
        hipLaunchKernelGGL(k_fv_rap<double>, dim3(s.nfvrch), dim3(64), 0, c.stream, g, s.ns, sb, s.fvblock, s.fvptr,
                           s.fvrcblk, s.fvrcfirst, s.fvrrow, s.fvcells, s.P64[s.cur], c.bcdiag, s.Afv, s.fvrpart,
                           s.Mp);
    if (s.nfvrrow > 0) launch_partial_rows_finish(c, s.M, s.Mp, s.fvrcfirst, s.fvrrow, s.fvrpart, s.Afv);
    launch_pad_identity(c, s.Afv, s.M, s.Mp);
}

void launch_fv_restrict(Ctx &c, Stage &s, const double *b) {
    hipLaunchKernelGGL(k_fv_restrict, dim3(s.M), dim3(64), 0, c.stream, s.M, s.fvptr, s.fvcells, b, s.dvec);
}

int launch_fv_local(Ctx &c, Stage &s, const double *pms, double *pf, double rtol, int max_iters, int *iters_max) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    if (s.fv_maxcells > kFvMaxCells) return MSRSB_E_INVAL;
    if (s.fv_maxcells <= kFvLineCells) {
        const size_t lds = 28 * (size_t)std::max(s.fv_maxcells, 1);
        hipLaunchKernelGGL(k_fv_local_line, dim3(s.M), dim3(kFvThreads), lds, c.stream, g, s.fvblock, s.fvptr,
                           s.fvcells, s.fvloc, c.bcdiag, c.b, pms, pf, rtol, max_iters, iters_max);
        return MSRSB_OK;
    }
    const size_t lds = sizeof(double) * (size_t)std::max(s.fv_maxcells, 1);
    hipLaunchKernelGGL(k_fv_local, dim3(s.M), dim3(kFvThreads), lds, c.stream, g, s.fvblock, s.fvptr, s.fvcells,
                       s.fvloc, c.bcdiag, c.b, pms, pf, c.r, c.tmp, rtol, max_iters, iters_max);
    return MSRSB_OK;
}

void launch_fv_faces(Ctx &c, Stage &s, const double *pms, const double *pf, double *face) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    hipLaunchKernelGGL(k_fv_faces, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, s.fvblock, pms, pf, face);
}

void launch_fv_imbalance(Ctx &c, const double *face, const double *pf, unsigned long long *maxbits) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    hipLaunchKernelGGL(k_fv_imbalance, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, face, pf, c.bcdiag,
                       c.bcrhs, c.src, maxbits);
}

}  // namespace msrsb
