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
// registers.  Threads take only columns of the phase's colour (the p-th
// column of a colour in row-major order), so no lane idles on the other
// colour, and the black phase keeps its forward result in registers for the
// backward sweep.  The factors and the corrections are stored per colour in
// that packed order, so each pass reads only its own colour's factors and
// the other colour's corrections, contiguously; r, x and the face
// coefficients keep the natural layout.  Columns taller than kLineLMax * 64
// cells use a second kernel that walks each chunk twice from memory over the
// natural layout.
#include <hip/hip_runtime.h>

#include "batch.h"
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

// forward declarations of the register path's layout (defined below)
int lilu_reg_chunks(int nz);
template <typename TT>
__global__ void k_lilu_pack(Fine g, int hx, int ncol, const double *__restrict__ dinv,
                            const double *__restrict__ cz, const TT *__restrict__ tz, TT *__restrict__ out);

void launch_lilu_factor(Ctx &c) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const int nb = cdiv(g.nxy, kBlock);
    hipLaunchKernelGGL(k_lilu_factor<0>, dim3(nb), dim3(kBlock), 0, c.stream, g, c.ldinv, c.lcz, c.ldinv32, c.lcz32);
    hipLaunchKernelGGL(k_lilu_factor<1>, dim3(nb), dim3(kBlock), 0, c.stream, g, c.ldinv, c.lcz, c.ldinv32, c.lcz32);
    if (!c.lpack) return;
    const int hx = (c.nx + 1) / 2, ncol = hx * c.ny;
    const size_t S2 = 2 * (size_t)ncol * c.nz;
    const dim3 grid((unsigned)((S2 + kBlock - 1) / kBlock)), blk(kBlock);
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_lilu_pack<float>, grid, blk, 0, c.stream, g, hx, ncol, c.ldinv, c.lcz, c.tz32,
                           (float *)c.lpack);
    else
        hipLaunchKernelGGL(k_lilu_pack<double>, grid, blk, 0, c.stream, g, hx, ncol, c.ldinv, c.lcz, c.tz,
                           (double *)c.lpack);
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

// Chunks per column (a power of two) of the register path; 0 if the columns
// are too tall for it.
int lilu_reg_chunks(int nz) {
    int nchp = 1;
    while (nchp * kLineLMax < nz) nchp *= 2;
    return nchp <= kLineThreads / 4 ? nchp : 0;
}

// Colour-packed layout of the register path: slot p of colour c is column
// (x, y) with y = p / hx, x = 2 (p % hx) + ((c + y) & 1), hx = ceil(nx / 2)
// (slots with x >= nx are padding), and entry (k, p) sits at k * ncol + p,
// ncol = hx * ny.  Per colour three factor arrays (1/p, cz, Tz/p) and one
// correction array (w for red, z for black), so that every pass reads and
// writes only its own colour's entries, contiguously.
size_t lilu_slots(int nx, int ny, int nz) { return (size_t)((nx + 1) / 2) * ny * nz; }

template <typename TT>
__global__ void k_lilu_pack(Fine g, int hx, int ncol, const double *__restrict__ dinv,
                            const double *__restrict__ cz, const TT *__restrict__ tz, TT *__restrict__ out) {
    const size_t S = (size_t)ncol * g.nz;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * S) return;
    const int c = q >= S;
    const size_t rem = q - c * S;
    const int k = (int)(rem / ncol), p = (int)(rem % ncol);
    const int y = p / hx, x = 2 * (p % hx) + ((c + y) & 1);
    TT d = (TT)0, cc = (TT)0, t = (TT)0;
    if (x < g.nx) {
        const int i = x + g.nx * y + g.nxy * k;
        d = (TT)dinv[i];
        cc = (TT)cz[i];
        if (k + 1 < g.nz) t = tz[i] * d;
    }
    out[(3 * c + 0) * S + rem] = d;
    out[(3 * c + 1) * S + rem] = cc;
    out[(3 * c + 2) * S + rem] = t;
}

template <typename TT>
struct LineRegArgs {
    Fine g;
    const TT *tx, *ty;             // face coefficients, natural layout
    const TT *pd, *pc, *pt;        // this colour's packed 1/p, cz, Tz/p
    TT *eself;                     // this colour's packed corrections
    const TT *eother;              // the other colour's packed corrections
    const double *r;
    double *x;
    int hx, ncol;                  // slots per row of one colour, hx * ny
    int cw, nch, L;                // columns per workgroup, chunks per column, cells per chunk (<= kLineLMax)
};

// Sum over the x/y neighbours (other colour) of T * correction.  Branch-free:
// every load is issued at an in-bounds index (the cell's own where the
// neighbour does not exist) and the product is dropped afterwards, so the
// loads of all cells of a chunk can be in flight together; a dropped product
// never reaches the sum, whatever the value read.  par = x & 1 relation:
// x = 2 j + par, the x neighbours are slots j + par - 1 and j + par of the
// other colour's row, the y neighbours slot j of the rows above and below.
template <typename TT>
__device__ inline TT xy_sum_r(const LineRegArgs<TT> &a, int i, int x, int y, int j, int par, size_t kq) {
    const bool hxm = x > 0, hxp = x + 1 < a.g.nx, hym = y > 0, hyp = y + 1 < a.g.ny;
    const int row = y * a.hx;
    const int own = row + j;
    const int qxm = hxm ? row + j + par - 1 : own, qxp = hxp ? row + j + par : own;
    const int qym = hym ? own - a.hx : own, qyp = hyp ? own + a.hx : own;
    const TT pxm = a.tx[hxm ? i - 1 : i] * a.eother[kq + qxm], pxp = a.tx[i] * a.eother[kq + qxp];
    const TT pym = a.ty[hym ? i - a.g.nx : i] * a.eother[kq + qym], pyp = a.ty[i] * a.eother[kq + qyp];
    TT s = hxm ? pxm : (TT)0;
    s += hxp ? pxp : (TT)0;
    s += hym ? pym : (TT)0;
    s += hyp ? pyp : (TT)0;
    return s;
}

// Apply the chunk maps (sA, sB) of chunks c0, c0 + dir, ... (cnt of them,
// dir = +1 or -1) in that order to v.  Eight maps are read from LDS before
// the first is applied, so the walk waits on one LDS round trip per eight
// chunks instead of one per chunk; the arithmetic and its order are those of
// applying the maps one by one.
template <typename TT>
__device__ inline TT chunk_combine(const TT *sA, const TT *sB, int cw, int cl, int c0, int dir, int cnt, TT v) {
    for (int base = 0; base < cnt; base += 8) {
        TT ga[8], gb[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int c = c0 + dir * min(base + t, cnt - 1);
            ga[t] = sA[c * cw + cl];
            gb[t] = sB[c * cw + cl];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (base + t < cnt) v = ga[t] + gb[t] * v;
    }
    return v;
}

// PHASE 0: red forward (writes w = y / p); 1: black forward and backward
// (writes z); 2: red backward (reads w, writes x of both colours).  Thread layout:
// column slot cl = threadIdx % cw, chunk ch = threadIdx / cw.  A cell is
// active where its 1/p is nonzero (inactive cells and non-positive pivots;
// their correction is exactly zero).
template <typename TT, int PHASE, bool ASSIGN>
__device__ __forceinline__ void lilu_reg_body(int bid, int nblk, LineRegArgs<TT> a, const int *done) {
    __shared__ TT sA[kLineThreads], sB[kLineThreads];
    // The skip flag: the FP32 red backward pass reads it once its operands
    // are in flight (every thread of the workgroup sees the same value, before
    // any barrier); the other passes measured as fast or faster reading it
    // first.
    constexpr bool kLateSkip = sizeof(TT) == 4 && PHASE == 2;
    if (!kLateSkip && done && *done) return;
    const int b = xcd_block(bid, nblk);
    if (b * a.cw >= a.ncol) return;
    const int cl = threadIdx.x % a.cw, ch = threadIdx.x / a.cw;
    int p = b * a.cw + cl;
    const int colour = PHASE == 1 ? 1 : 0;
    int y = p / a.hx, j = p % a.hx;
    const int par = (colour + y) & 1;
    int x = 2 * j + par;
    const bool mine = p < a.ncol && x < a.g.nx && ch < a.nch;
    const int z0 = ch * a.L;
    const int n = mine ? min(a.L, a.g.nz - z0) : 0;
    if (!mine) x = y = j = p = 0;  // loads below stay in bounds; nothing is written
    const int col = x + a.g.nx * y, nxy = a.g.nxy, nz = a.g.nz;
    auto layer = [&](int t) { return min(z0 + min(t, max(n - 1, 0)), nz - 1); };
    TT al[kLineLMax], be[kLineLMax], dv[kLineLMax];
    TT bt[PHASE == 1 ? kLineLMax : 1];  // black: Tz/p, loaded with the forward operands
    TT v;
    if (PHASE <= 1) {
        // forward: y_k = al_k + be_k y_{k-1}
#pragma unroll
        for (int t = 0; t < kLineLMax; ++t) {
            const int k = layer(t);
            const size_t kq = (size_t)k * a.ncol;
            const int i = col + nxy * k;
            TT s = (TT)a.r[i];
            if (PHASE == 1) s += xy_sum_r(a, i, x, y, j, par, kq);
            al[t] = s;
            be[t] = a.pc[kq + p];
            dv[t] = a.pd[kq + p];
            if (PHASE == 1) bt[t] = a.pt[kq + p];
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
        v = chunk_combine(sA, sB, a.cw, cl, 0, 1, ch, (TT)0);
#pragma unroll
        for (int t = 0; t < kLineLMax; ++t)
            if (t < n) {
                v = al[t] + be[t] * v;
                if (PHASE == 0) a.eself[(size_t)(z0 + t) * a.ncol + p] = v * dv[t];
                else al[t] = v;  // y, kept for the backward sweep
            }
        if (PHASE == 0) return;
        __syncthreads();  // LDS reuse
    }
    // x is updated in whole pairs {x, x ^ 1} of a row: the red pass writes
    // its cell and the black partner (black slot p as well: x ^ 1 = 2j + 1 -
    // par), so x is read and written once; the black pass writes x only
    // where the partner lies outside the row (odd nx).  No other thread
    // writes either cell of the pair, so the red pass loads the partner's z
    // and, when adding, both cells' x together with its other operands.
    const bool partner = (x ^ 1) < a.g.nx;
    const int ib = partner ? (x ^ 1) + a.g.nx * y : col;
    TT zp[PHASE == 2 ? kLineLMax : 1];
    double xo[PHASE == 2 && !ASSIGN ? kLineLMax : 1], xq[PHASE == 2 && !ASSIGN ? kLineLMax : 1];
    // backward: z_k = al_k + be_k z_{k+1}, be_k = Tz_k / p_k
#pragma unroll
    for (int t = 0; t < kLineLMax; ++t) {
        const int k = layer(t);
        const size_t kq = (size_t)k * a.ncol;
        if (PHASE == 2) {
            const int i = col + nxy * k;
            dv[t] = a.pd[kq + p];
            al[t] = a.eself[kq + p] + dv[t] * xy_sum_r(a, i, x, y, j, par, kq);
            be[t] = a.pt[kq + p];
            zp[t] = a.eother[kq + p];
            if (!ASSIGN) {
                xo[t] = a.x[i];
                xq[t] = a.x[ib + nxy * k];
            }
        } else {
            al[t] = al[t] * dv[t];
            be[t] = bt[PHASE == 1 ? t : 0];
        }
    }
    if (kLateSkip && done && *done) return;
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
    v = chunk_combine(sA, sB, a.cw, cl, a.nch - 1, -1, a.nch - 1 - ch, (TT)0);
    // A correction is exactly zero where 1/p is.
#pragma unroll
    for (int t = kLineLMax - 1; t >= 0; --t)
        if (t < n) {
            v = al[t] + be[t] * v;
            const size_t q = (size_t)(z0 + t) * a.ncol + p;
            const int i = col + nxy * (z0 + t);
            if (PHASE == 1) a.eself[q] = v;
            if (PHASE == 2) {
                if (dv[t] != (TT)0) a.x[i] = ASSIGN ? (double)v : xo[PHASE == 2 && !ASSIGN ? t : 0] + (double)v;
                else if (ASSIGN) a.x[i] = 0.0;
                if (partner) {
                    const double zb = (double)zp[t];
                    a.x[ib + nxy * (z0 + t)] = ASSIGN ? zb : xq[PHASE == 2 && !ASSIGN ? t : 0] + zb;
                }
            } else if (!partner) {
                if (dv[t] != (TT)0) a.x[i] = ASSIGN ? (double)v : a.x[i] + (double)v;
                else if (ASSIGN) a.x[i] = 0.0;
            }
        }
}

template <typename TT, int PHASE, bool ASSIGN>
__global__ __launch_bounds__(kLineThreads) void k_lilu_reg(LineRegArgs<TT> a, const int *done) {
    lilu_reg_body<TT, PHASE, ASSIGN>(blockIdx.x, gridDim.x, a, done);
}

// Register-path geometry of a box with nchp = lilu_reg_chunks(nz) > 0:
// column slots per row, columns, columns per workgroup, cells per chunk,
// chunks per column; returns the grid (workgroups).
static int lilu_reg_geometry(int nx, int ny, int nz, int nchp, int *hx, int *ncol, int *cw, int *L, int *nch) {
    *hx = (nx + 1) / 2;
    *ncol = *hx * ny;
    *cw = kLineThreads / nchp;
    *L = cdiv(nz, nchp);
    *nch = cdiv(nz, *L);
    return xcd_grid(cdiv(*ncol, *cw));
}

template <typename TT, bool ASSIGN>
static void lilu_dispatch(Ctx &c, const TT *tx, const TT *ty, const TT *tz, const TT *dinv, const TT *cz,
                          TT *packed, TT *pe, const double *r, double *x, const int *done) {
    const Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const int nchp = lilu_reg_chunks(c.nz);
    if (nchp) {
        const size_t S = lilu_slots(c.nx, c.ny, c.nz);
        LineRegArgs<TT> q;
        q.g = g;
        q.tx = tx; q.ty = ty;
        q.r = r; q.x = x;
        const dim3 grid(lilu_reg_geometry(c.nx, c.ny, c.nz, nchp, &q.hx, &q.ncol, &q.cw, &q.L, &q.nch)),
            blk(kLineThreads);
        TT *e_red = pe, *e_black = pe + S;
        // red forward
        q.pd = packed; q.pc = packed + S; q.pt = packed + 2 * S;
        q.eself = e_red; q.eother = e_black;
        hipLaunchKernelGGL((k_lilu_reg<TT, 0, ASSIGN>), grid, blk, 0, c.stream, q, done);
        // black forward and backward
        q.pd = packed + 3 * S; q.pc = packed + 4 * S; q.pt = packed + 5 * S;
        q.eself = e_black; q.eother = e_red;
        hipLaunchKernelGGL((k_lilu_reg<TT, 1, ASSIGN>), grid, blk, 0, c.stream, q, done);
        // red backward
        q.pd = packed; q.pc = packed + S; q.pt = packed + 2 * S;
        q.eself = e_red; q.eother = e_black;
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
        float *pk = (float *)c.lpack, *pe = (float *)c.lpe;
        if (assign) lilu_dispatch<float, true>(c, c.tx32, c.ty32, c.tz32, c.ldinv32, c.lcz32, pk, pe, r, x, done);
        else lilu_dispatch<float, false>(c, c.tx32, c.ty32, c.tz32, c.ldinv32, c.lcz32, pk, pe, r, x, done);
    } else {
        double *pk = (double *)c.lpack, *pe = (double *)c.lpe;
        if (assign) lilu_dispatch<double, true>(c, c.tx, c.ty, c.tz, c.ldinv, c.lcz, pk, pe, r, x, done);
        else lilu_dispatch<double, false>(c, c.tx, c.ty, c.tz, c.ldinv, c.lcz, pk, pe, r, x, done);
    }
}

// Batched: x = S r (assign) for every member of the batch, the three passes
// each one launch over all members.
template <typename TT, int PHASE>
__global__ __launch_bounds__(kLineThreads) void k_lilu_reg_b(const BMember *D, BGroup gp, const int *act, int rsel,
                                                             int xsel) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    const long S = d.l_S;
    const TT *pk = (const TT *)d.lpack;
    TT *pe = (TT *)d.lpe;
    LineRegArgs<TT> q;
    q.g = d.g;
    q.tx = (const TT *)d.wtx;
    q.ty = (const TT *)d.wty;
    q.r = bvec(d, rsel);
    q.x = bvec(d, xsel);
    q.hx = d.l_hx;
    q.ncol = d.l_ncol;
    q.cw = d.l_cw;
    q.nch = d.l_nch;
    q.L = d.l_L;
    const int c0 = PHASE == 1 ? 3 : 0;
    q.pd = pk + c0 * S;
    q.pc = pk + (c0 + 1) * S;
    q.pt = pk + (c0 + 2) * S;
    q.eself = PHASE == 1 ? pe + S : pe;
    q.eother = PHASE == 1 ? pe : pe + S;
    lilu_reg_body<TT, PHASE, true>(lb, nb, q, &d.status->done);
}

// A member's register-path geometry and working-precision operands; returns
// its grid, 0 if its columns are too tall for the register path.
int bat_member_lilu(const Ctx &c, BMember &d) {
    const int nchp = lilu_reg_chunks(c.nz);
    if (!nchp || !c.lpack) return 0;
    d.l_S = (long)lilu_slots(c.nx, c.ny, c.nz);
    d.lpack = c.lpack;
    d.lpe = c.lpe;
    return lilu_reg_geometry(c.nx, c.ny, c.nz, nchp, &d.l_hx, &d.l_ncol, &d.l_cw, &d.l_L, &d.l_nch);
}

template <typename TT>
static void bat_lilu_t(Batch &B, int rsel, int xsel) {
    for (const HGroup &h : B.lilu) {
        if (h.g.n == 0) continue;
        const dim3 grid(h.g.total), blk(kLineThreads);
        hipLaunchKernelGGL((k_lilu_reg_b<TT, 0>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act, rsel, xsel);
        hipLaunchKernelGGL((k_lilu_reg_b<TT, 1>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act, rsel, xsel);
        hipLaunchKernelGGL((k_lilu_reg_b<TT, 2>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act, rsel, xsel);
    }
}

void bat_lilu_assign(Batch &B, int rsel, int xsel) {
    if (B.mixed) bat_lilu_t<float>(B, rsel, xsel);
    else bat_lilu_t<double>(B, rsel, xsel);
}

}  // namespace msrsb
