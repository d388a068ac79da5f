// ILU(0) in z-line red-black order (the smoother of section "Computational
// efficiency" is ILU(0); the paper leaves its ordering open).  Columns (x, y)
// are coloured by the parity of x + y, red (even) columns first, each
// column's cells in ascending z.  Two columns of one colour are never
// coupled, and inside a column the operator is tridiagonal, so ILU(0) in this
// order is:
//   red column:   p_k = a_kk - Tz_{k-1}^2 / p_{k-1}            (exact LU)
//   black column: p_k = a_kk - sum_{red m in x, y} T_km^2 / p_m - Tz_{k-1}^2 / p_{k-1}
// with p the pivots (dinv = 1/p, cz_k = Tz_{k-1} / p_{k-1} stored), and its
// application (LU)^{-1} r is
//   red forward:   y_k = r_k + cz_k y_{k-1},               w_k = y_k / p_k
//   black forward: y_k = r_k + sum_{red m} T_km w_m + cz_k y_{k-1}
//   black back:    z_k = (y_k + Tz_k z_{k+1}) / p_k
//   red back:      z_k = w_k + (Tz_k z_{k+1} + sum_{black j} T_kj z_j) / p_k
// (with nz = 1 this is the red-black ILU(0) of k_fine.hip).  Strong vertical
// coupling (T_z / T_x ~ 100 on the benchmark model) is inside the columns.
//
// Each recurrence along a column is a linear recurrence, computed by a
// chunked scan: z is cut into chunks of at most kLineLMax cells; a thread
// loads its chunk's coefficients into registers, composes the chunk's affine
// map y_out = A + B y_in, the maps of one column are combined in LDS in chunk
// order, and the thread walks its chunk again from the incoming value out of
// registers.  Threads take only columns of the phase's colour (packed: the
// p-th column of a colour in row-major order), so no lane idles on the other
// colour, and the black phase keeps its forward result in registers for the
// backward sweep.  Columns taller than kLineLMax * 64 cells use a second
// kernel that walks each chunk twice from memory.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

constexpr int kLineChunks = 8;

// Pivots, column by column (one thread per column of the colour).
template <int COLOUR>
__global__ void k_lilu_factor(Fine g, double *__restrict__ dinv, double *__restrict__ cz, float *__restrict__ dinv32,
                              float *__restrict__ cz32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nxy) return;
    const int x = t % g.nx, y = t / g.nx;
    if (((x + y) & 1) != COLOUR) return;
    double dprev = 0.0;
    for (int k = 0; k < g.nz; ++k) {
        const int i = t + g.nxy * k;
        double p = g.diag[i];
        double c = 0.0;
        if (k > 0) {
            const double tz = g.tz[i - g.nxy];
            if (tz != 0.0) {
                p -= tz * tz * dprev;
                c = tz * dprev;
            }
        }
        if (COLOUR == 1 && g.diag[i] > 0.0) {
            double tq;
            if (x > 0 && (tq = g.tx[i - 1]) != 0.0) p -= tq * tq * dinv[i - 1];
            if (x + 1 < g.nx && (tq = g.tx[i]) != 0.0) p -= tq * tq * dinv[i + 1];
            if (y > 0 && (tq = g.ty[i - g.nx]) != 0.0) p -= tq * tq * dinv[i - g.nx];
            if (y + 1 < g.ny && (tq = g.ty[i]) != 0.0) p -= tq * tq * dinv[i + g.nx];
        }
        const double di = g.diag[i] > 0.0 && p > 0.0 ? 1.0 / p : 0.0;
        dinv[i] = di;
        cz[i] = c;
        dinv32[i] = (float)di;
        cz32[i] = (float)c;
        dprev = di;
    }
}

void launch_lilu_factor(Ctx &c) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const int nb = cdiv(g.nxy, kBlock);
    hipLaunchKernelGGL(k_lilu_factor<0>, dim3(nb), dim3(kBlock), 0, c.stream, g, c.ldinv, c.lcz, c.ldinv32, c.lcz32);
    hipLaunchKernelGGL(k_lilu_factor<1>, dim3(nb), dim3(kBlock), 0, c.stream, g, c.ldinv, c.lcz, c.ldinv32, c.lcz32);
}

template <typename TT>
struct LineArgs {
    Fine g;
    const TT *tx, *ty, *tz, *dinv, *cz;
    const double *r;
    double *e;   // red cells: w = y / p; black cells: y, then z
    double *x;
    int nseg, nch, L;
};

// Sum over the x/y neighbours m of cell i (column x, y) of T_im v_m.
template <typename TT>
__device__ inline TT xy_sum(const LineArgs<TT> &a, int i, int x, int y, const double *__restrict__ v) {
    TT s = (TT)0, t;
    if (x > 0 && (t = a.tx[i - 1]) != (TT)0) s += t * (TT)v[i - 1];
    if (x + 1 < a.g.nx && (t = a.tx[i]) != (TT)0) s += t * (TT)v[i + 1];
    if (y > 0 && (t = a.ty[i - a.g.nx]) != (TT)0) s += t * (TT)v[i - a.g.nx];
    if (y + 1 < a.g.ny && (t = a.ty[i]) != (TT)0) s += t * (TT)v[i + a.g.nx];
    return s;
}

// Combine the chunk maps (A, B) of this lane in chunk order (forward: chunks
// before `ch`; backward: chunks after it) into the incoming value.
template <typename TT>
__device__ inline TT incoming(TT (*sA)[64], TT (*sB)[64], int ch, int nch, int lane, bool fwd) {
    TT v = (TT)0;
    if (fwd) {
        for (int c = 0; c < ch; ++c) v = sA[c][lane] + sB[c][lane] * v;
    } else {
        for (int c = nch - 1; c > ch; --c) v = sA[c][lane] + sB[c][lane] * v;
    }
    return v;
}

// PHASE 0: red forward (writes w to e); 1: black forward + backward (writes y,
// then z to e, and x); 2: red backward (writes x).
template <typename TT, int PHASE, bool ASSIGN>
__global__ __launch_bounds__(64 * kLineChunks) void k_lilu_apply(LineArgs<TT> a, const int *done) {
    __shared__ TT sA[kLineChunks][64], sB[kLineChunks][64];
    if (done && *done) return;
    const int b = xcd_block();
    if (b >= a.nseg * a.g.ny) return;
    const int lane = threadIdx.x & 63, ch = threadIdx.x >> 6;
    const int y = b / a.nseg, x = (b % a.nseg) * 64 + lane;
    const int colour = PHASE == 1 ? 1 : 0;
    const bool mine = x < a.g.nx && ch < a.nch && ((x + y) & 1) == colour;
    const int col = x + a.g.nx * y, nxy = a.g.nxy;
    const int z0 = ch * a.L, z1 = min(a.g.nz, z0 + a.L);
    if (PHASE <= 1) {
        // forward: y_k = alpha_k + cz_k y_{k-1}
        auto alpha_f = [&](int i) -> TT {
            TT v = (TT)a.r[i];
            if (PHASE == 1) v += xy_sum(a, i, x, y, a.e);
            return v;
        };
        TT A = (TT)0, B = (TT)1;
        if (mine)
            for (int k = z0; k < z1; ++k) {
                const int i = col + nxy * k;
                const TT be = a.cz[i];
                A = alpha_f(i) + be * A;
                B = be * B;
            }
        sA[ch][lane] = A;
        sB[ch][lane] = B;
        __syncthreads();
        if (mine) {
            TT v = incoming(sA, sB, ch, a.nch, lane, true);
            for (int k = z0; k < z1; ++k) {
                const int i = col + nxy * k;
                v = alpha_f(i) + a.cz[i] * v;
                a.e[i] = PHASE == 0 ? (double)(v * a.dinv[i]) : (double)v;
            }
        }
        if (PHASE == 0) return;
        __syncthreads();  // LDS reuse
    }
    // backward: z_k = alpha_k + (Tz_k / p_k) z_{k+1}
    auto alpha_b = [&](int i) -> TT {
        if (PHASE == 1) return (TT)a.e[i] * a.dinv[i];
        return (TT)a.e[i] + a.dinv[i] * xy_sum(a, i, x, y, a.e);
    };
    auto beta_b = [&](int i, int k) -> TT { return k + 1 < a.g.nz ? a.tz[i] * a.dinv[i] : (TT)0; };
    TT A = (TT)0, B = (TT)1;
    if (mine)
        for (int k = z1 - 1; k >= z0; --k) {
            const int i = col + nxy * k;
            const TT be = beta_b(i, k);
            A = alpha_b(i) + be * A;
            B = be * B;
        }
    sA[ch][lane] = A;
    sB[ch][lane] = B;
    __syncthreads();
    if (!mine) return;
    TT v = incoming(sA, sB, ch, a.nch, lane, false);
    for (int k = z1 - 1; k >= z0; --k) {
        const int i = col + nxy * k;
        v = alpha_b(i) + beta_b(i, k) * v;
        if (PHASE == 1) a.e[i] = (double)v;
        if (a.g.diag[i] > 0.0) a.x[i] = ASSIGN ? (double)v : a.x[i] + (double)v;
        else if (ASSIGN) a.x[i] = 0.0;
    }
}

constexpr int kLineLMax = 8;      // cells per chunk held in registers
constexpr int kLineThreads = 256;  // threads per workgroup: columns x chunks (power of 2)

template <typename TT>
struct LineRegArgs {
    Fine g;
    const TT *tx, *ty, *tz, *dinv, *cz;
    const double *r;
    double *e, *x;
    int hx, ncol;    // columns of one colour per row, ceil(nx / 2), and hx * ny
    int cw, nch, L;  // columns per workgroup, chunks per column, cells per chunk (<= kLineLMax)
};

// Branch-free: every load is issued at an in-bounds index (the cell itself
// where the neighbour does not exist) and the product is dropped afterwards,
// so the loads of all cells of a chunk can be in flight together; a dropped
// product never reaches the sum, whatever the value read.
template <typename TT>
__device__ inline TT xy_sum_r(const LineRegArgs<TT> &a, int i, int x, int y, const double *__restrict__ v) {
    const bool hxm = x > 0, hxp = x + 1 < a.g.nx, hym = y > 0, hyp = y + 1 < a.g.ny;
    const int ixm = hxm ? i - 1 : i, iym = hym ? i - a.g.nx : i;
    const int ixp = hxp ? i + 1 : i, iyp = hyp ? i + a.g.nx : i;
    const TT pxm = a.tx[ixm] * (TT)v[ixm], pxp = a.tx[i] * (TT)v[ixp];
    const TT pym = a.ty[iym] * (TT)v[iym], pyp = a.ty[i] * (TT)v[iyp];
    TT s = hxm ? pxm : (TT)0;
    s += hxp ? pxp : (TT)0;
    s += hym ? pym : (TT)0;
    s += hyp ? pyp : (TT)0;
    return s;
}

// PHASE 0: red forward (writes w = y / p to e); 1: black forward and backward
// (writes z to e and x); 2: red backward (writes x).  Thread layout: column
// slot cl = threadIdx % cw, chunk ch = threadIdx / cw.
template <typename TT, int PHASE, bool ASSIGN>
__global__ __launch_bounds__(kLineThreads) void k_lilu_reg(LineRegArgs<TT> a, const int *done) {
    __shared__ TT sA[kLineThreads], sB[kLineThreads];
    if (done && *done) return;
    const int b = xcd_block();
    if (b * a.cw >= a.ncol) return;
    const int cl = threadIdx.x % a.cw, ch = threadIdx.x / a.cw;
    const int p = b * a.cw + cl;
    const int colour = PHASE == 1 ? 1 : 0;
    int y = p / a.hx, x = 2 * (p % a.hx) + ((colour + y) & 1);
    const bool mine = p < a.ncol && x < a.g.nx && ch < a.nch;
    const int z0 = ch * a.L;
    const int n = mine ? min(a.L, a.g.nz - z0) : 0;
    if (!mine) x = y = 0;  // loads below stay in bounds; nothing is written
    const int col = x + a.g.nx * y, nxy = a.g.nxy, nz = a.g.nz;
    auto cell = [&](int t) { return col + nxy * min(z0 + min(t, max(n - 1, 0)), nz - 1); };
    TT al[kLineLMax], be[kLineLMax], dv[kLineLMax];
    bool act[kLineLMax];
    TT v;
    if (PHASE <= 1) {
        // forward: y_k = al_k + be_k y_{k-1}
#pragma unroll
        for (int t = 0; t < kLineLMax; ++t) {
            const int i = cell(t);
            TT s = (TT)a.r[i];
            if (PHASE == 1) s += xy_sum_r(a, i, x, y, a.e);
            al[t] = s;
            be[t] = a.cz[i];
            dv[t] = a.dinv[i];
        }
        TT A = (TT)0, B = (TT)1;
#pragma unroll
        for (int t = 0; t < kLineLMax; ++t)
            if (t < n) {
                A = al[t] + be[t] * A;
                B = be[t] * B;
            }
        sA[threadIdx.x] = A;
        sB[threadIdx.x] = B;
        __syncthreads();
        v = (TT)0;
        for (int c = 0; c < ch; ++c) v = sA[c * a.cw + cl] + sB[c * a.cw + cl] * v;
#pragma unroll
        for (int t = 0; t < kLineLMax; ++t)
            if (t < n) {
                v = al[t] + be[t] * v;
                if (PHASE == 0) a.e[col + nxy * (z0 + t)] = (double)(v * dv[t]);
                else al[t] = v;  // y, kept for the backward sweep
            }
        if (PHASE == 0) return;
        __syncthreads();  // LDS reuse
    }
    // backward: z_k = al_k + be_k z_{k+1}, be_k = Tz_k / p_k
#pragma unroll
    for (int t = 0; t < kLineLMax; ++t) {
        const int i = cell(t);
        if (PHASE == 2) {
            dv[t] = a.dinv[i];
            al[t] = (TT)a.e[i] + dv[t] * xy_sum_r(a, i, x, y, a.e);
        } else {
            al[t] = al[t] * dv[t];
        }
        be[t] = z0 + t + 1 < nz ? a.tz[i] * dv[t] : (TT)0;
        act[t] = a.g.diag[i] > 0.0;
    }
    TT A = (TT)0, B = (TT)1;
#pragma unroll
    for (int t = kLineLMax - 1; t >= 0; --t)
        if (t < n) {
            A = al[t] + be[t] * A;
            B = be[t] * B;
        }
    sA[threadIdx.x] = A;
    sB[threadIdx.x] = B;
    __syncthreads();
    if (!mine) return;
    v = (TT)0;
    for (int c = a.nch - 1; c > ch; --c) v = sA[c * a.cw + cl] + sB[c * a.cw + cl] * v;
#pragma unroll
    for (int t = kLineLMax - 1; t >= 0; --t)
        if (t < n) {
            v = al[t] + be[t] * v;
            const int i = col + nxy * (z0 + t);
            if (PHASE == 1) a.e[i] = (double)v;
            if (act[t]) a.x[i] = ASSIGN ? (double)v : a.x[i] + (double)v;
            else if (ASSIGN) a.x[i] = 0.0;
        }
}

template <typename TT, bool ASSIGN>
static void lilu_dispatch(Ctx &c, const TT *tx, const TT *ty, const TT *tz, const TT *dinv, const TT *cz,
                          const double *r, double *x, const int *done) {
    const Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    int nchp = 1;  // chunks per column rounded up to a power of two
    while (nchp * kLineLMax < c.nz) nchp *= 2;
    if (nchp <= kLineThreads / 4) {
        LineRegArgs<TT> q;
        q.g = g;
        q.tx = tx; q.ty = ty; q.tz = tz; q.dinv = dinv; q.cz = cz;
        q.r = r; q.e = c.e; q.x = x;
        q.hx = (c.nx + 1) / 2;
        q.ncol = q.hx * c.ny;
        q.cw = kLineThreads / nchp;
        q.L = cdiv(c.nz, nchp);
        q.nch = cdiv(c.nz, q.L);
        const dim3 grid(xcd_grid(cdiv(q.ncol, q.cw))), blk(kLineThreads);
        hipLaunchKernelGGL((k_lilu_reg<TT, 0, ASSIGN>), grid, blk, 0, c.stream, q, done);
        hipLaunchKernelGGL((k_lilu_reg<TT, 1, ASSIGN>), grid, blk, 0, c.stream, q, done);
        hipLaunchKernelGGL((k_lilu_reg<TT, 2, ASSIGN>), grid, blk, 0, c.stream, q, done);
        return;
    }
    LineArgs<TT> a;
    a.g = g;
    a.tx = tx; a.ty = ty; a.tz = tz; a.dinv = dinv; a.cz = cz;
    a.r = r; a.e = c.e; a.x = x;
    a.nseg = cdiv(c.nx, 64);
    a.nch = std::min(kLineChunks, c.nz);
    a.L = cdiv(c.nz, a.nch);
    a.nch = cdiv(c.nz, a.L);
    const dim3 grid(xcd_grid(a.nseg * c.ny)), blk(64 * kLineChunks);
    hipLaunchKernelGGL((k_lilu_apply<TT, 0, ASSIGN>), grid, blk, 0, c.stream, a, done);
    hipLaunchKernelGGL((k_lilu_apply<TT, 1, ASSIGN>), grid, blk, 0, c.stream, a, done);
    hipLaunchKernelGGL((k_lilu_apply<TT, 2, ASSIGN>), grid, blk, 0, c.stream, a, done);
}

void launch_lilu_apply(Ctx &c, const double *r, double *x, const int *done, bool assign) {
    if (c.opt.precision == MSRSB_MIXED) {
        if (assign) lilu_dispatch<float, true>(c, c.tx32, c.ty32, c.tz32, c.ldinv32, c.lcz32, r, x, done);
        else lilu_dispatch<float, false>(c, c.tx32, c.ty32, c.tz32, c.ldinv32, c.lcz32, r, x, done);
    } else {
        if (assign) lilu_dispatch<double, true>(c, c.tx, c.ty, c.tz, c.ldinv, c.lcz, r, x, done);
        else lilu_dispatch<double, false>(c, c.tx, c.ty, c.tz, c.ldinv, c.lcz, r, x, done);
    }
}

}  // namespace msrsb
