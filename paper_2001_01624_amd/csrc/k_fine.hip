// Fine-grid kernels: two-point operator assembly, residual r = b - A x
// (eq. iterative_multiscale), smoothers S (damped Jacobi; ILU(0) in
// red-black order, which for the 7-point two-point stencil reduces to a
// diagonal-only modification), norms, fluxes and the GMRES vector kernels.
//
// Layout: every per-cell array is indexed in the full box, x fastest.  The
// face array tx[i] holds the face to the +x neighbour and is 0 on the last
// column, so tx[i-1] is automatically 0 on the first column (likewise ty
// across rows); only the z neighbour below the first layer needs a bounds
// test.  Inactive cells have diag = 0 and are skipped.
#include <algorithm>
#include <type_traits>

#include "batch.h"
#include "dev_util.h"
#include "msrsb_internal.h"
#include "stencil.h"

namespace msrsb {

static Fine fine_of(const Ctx &c) {
    Fine g;
    g.nx = c.nx; g.ny = c.ny; g.nz = c.nz; g.nxy = c.nx * c.ny; g.N = c.N;
    g.tx = c.tx; g.ty = c.ty; g.tz = c.tz; g.diag = c.diag;
    return g;
}

static int red_grid(int N) { return xcd_grid(std::min(kRedBlocks, cdiv(N, kBlock))); }


__global__ void k_assemble(Fine g, const double *__restrict__ bcdiag, const double *__restrict__ bcrhs,
                           const double *__restrict__ src, double *__restrict__ diag, double *__restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    double d = g.tx[i] + g.ty[i] + g.tz[i];
    if (i >= 1) d += g.tx[i - 1];
    if (i >= g.nx) d += g.ty[i - g.nx];
    if (i >= g.nxy) d += g.tz[i - g.nxy];
    d += bcdiag[i];
    diag[i] = d;
    b[i] = d > 0.0 ? src[i] + bcrhs[i] : 0.0;
}

void launch_assemble(Ctx &c) {
    Fine g = fine_of(c);
    hipLaunchKernelGGL(k_assemble, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, c.bcdiag, c.bcrhs, c.src,
                       c.diag, c.b);
}

__device__ __forceinline__ void rhs_body(int bid, int nblk, int N, const double *__restrict__ diag,
                                         const double *__restrict__ bcrhs, const double *__restrict__ src,
                                         double *__restrict__ b, double *__restrict__ keep) {
    const int i = bid * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double q = src[i];
    keep[i] = q;
    b[i] = diag[i] > 0.0 ? q + bcrhs[i] : 0.0;
}

__global__ void k_rhs(int N, const double *__restrict__ diag, const double *__restrict__ bcrhs,
                      const double *__restrict__ src, double *__restrict__ b, double *__restrict__ keep) {
    rhs_body(blockIdx.x, gridDim.x, N, diag, bcrhs, src, b, keep);
}

void launch_source_update(Ctx &c, const double *d_source) {
    hipLaunchKernelGGL(k_rhs, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, c.diag, c.bcrhs, d_source,
                       c.b, c.src);
}

// Red-black ILU(0) pivots: red cells (i+j+k even) come first in the
// elimination order and keep a_ii; every neighbour of a black cell is red and
// earlier, so its pivot is a_ii - sum_j T_ij^2 / a_jj.  (Two cells of the
// same colour are never coupled, so ILU(0) has no other non-zero change.)
__global__ void k_ilu_factor(Fine g, double *__restrict__ dtil, float *__restrict__ dtil32,
                             float *__restrict__ diag32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    const double d = g.diag[i];
    const int ix = i % g.nx, iy = (i / g.nx) % g.ny, iz = i / g.nxy;
    double p = d;
    if (d > 0.0 && ((ix + iy + iz) & 1)) {
        double s = 0.0;
        double t;
        if (i >= 1 && (t = g.tx[i - 1]) != 0.0) s += t * t / g.diag[i - 1];
        if ((t = g.tx[i]) != 0.0) s += t * t / g.diag[i + 1];
        if (i >= g.nx && (t = g.ty[i - g.nx]) != 0.0) s += t * t / g.diag[i - g.nx];
        if ((t = g.ty[i]) != 0.0) s += t * t / g.diag[i + g.nx];
        if (i >= g.nxy && (t = g.tz[i - g.nxy]) != 0.0) s += t * t / g.diag[i - g.nxy];
        if ((t = g.tz[i]) != 0.0) s += t * t / g.diag[i + g.nxy];
        p = d - s;
    }
    dtil[i] = p;
    dtil32[i] = (float)p;
    diag32[i] = (float)d;
}

void launch_ilu_factor(Ctx &c) {
    Fine g = fine_of(c);
    hipLaunchKernelGGL(k_ilu_factor, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, c.dtil, c.dtil32,
                       c.diag32);
    if (c.opt.smoother == MSRSB_SMOOTH_ILU0_LINE) launch_lilu_factor(c);
}

template <bool NORM>
__device__ __forceinline__ void residual_body(int bid, int nblk, Fine g, const double *__restrict__ b,
                                              const double *__restrict__ x, double *__restrict__ r,
                                              double *__restrict__ partial, const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    double acc = 0.0;
    const int lb = xcd_block(bid, nblk);
    for (int t = lb * blockDim.x + threadIdx.x; t < g.N; t += nblk * blockDim.x) {
        const int i = xzy_cell(t, g.nx, g.ny, g.nz);
        const double d = g.diag[i], bi = b[i];
        const double ax = ax_row(g, x, i, d);
        const double ri = d > 0.0 ? bi - ax : 0.0;
        r[i] = ri;
        acc += ri * ri;
    }
    if (NORM) {
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) partial[lb] = s;
    }
}

template <bool NORM>
__global__ __launch_bounds__(kBlock) void k_residual(Fine g, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ partial, const int *done) {
    residual_body<NORM>(blockIdx.x, gridDim.x, g, b, x, r, partial, done);
}

// r = b - A x with one wavefront per grid row (y, z) of at most 64 cells,
// lanes along x: no index division, the x neighbours (and tx of the cell
// before) from the adjacent lanes, every load issued before the skip flag is
// read.  Faces follow cell_faces (boundary faces carry T = 0 in the data), so
// a lane at a row end may take its own x with the zero coefficient: the
// operations and their order are those of residual_cell.
constexpr int kResRows = 4;  // rows (wavefronts) per workgroup

__global__ __launch_bounds__(64 * kResRows) void k_residual_rows(Fine g, const double *__restrict__ b,
                                                                 const double *__restrict__ x,
                                                                 double *__restrict__ r, const int *done) {
    const int row = xcd_block() * kResRows + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (row >= g.ny * g.nz) return;
    const int lane = threadIdx.x & 63;
    const int xx = min(lane, g.nx - 1);  // lanes past the row load its last cell and store nothing
    const int i = row * g.nx + xx;
    const bool dny = i >= g.nx, upy = i + g.nx < g.N, dnz = i >= g.nxy, upz = i + g.nxy < g.N;
    const double d = g.diag[i], bi = b[i], xi = x[i];
    const double txi = g.tx[i], tyi = g.ty[i], tzi = g.tz[i];
    const double tym = g.ty[dny ? i - g.nx : i], tzm = g.tz[dnz ? i - g.nxy : i];
    const double xym = x[dny ? i - g.nx : i], xyp = x[upy ? i + g.nx : i];
    const double xzm = x[dnz ? i - g.nxy : i], xzp = x[upz ? i + g.nxy : i];
    if (done && *done) return;
    const double txm = __shfl_up(txi, 1, 64), xxm = __shfl_up(xi, 1, 64), xxp = __shfl_down(xi, 1, 64);
    const double t[6] = {xx > 0 ? txm : 0.0, txi, dny ? tym : 0.0, upy ? tyi : 0.0, dnz ? tzm : 0.0,
                         upz ? tzi : 0.0};
    const double xl[6] = {xx > 0 ? xxm : xi, xx + 1 < g.nx ? xxp : xi, xym, xyp, xzm, xzp};
    double s = d * xi;
#pragma unroll
    for (int q = 0; q < 6; ++q) s -= t[q] * xl[q];
    if (lane < g.nx) r[i] = d > 0.0 ? bi - s : 0.0;
}

void launch_residual(Ctx &c, const double *b, const double *x, double *r, bool norm, const int *done) {
    ProfScope ps(c, MSRSB_K_RESIDUAL);
    Fine g = fine_of(c);
    const int grid = red_grid(c.N);
    if (!norm && c.nx <= 64) {
        hipLaunchKernelGGL(k_residual_rows, dim3(xcd_grid(cdiv(c.ny * c.nz, kResRows))), dim3(64 * kResRows), 0,
                           c.stream, g, b, x, r, done);
        return;
    }
    if (norm)
        hipLaunchKernelGGL(k_residual<true>, dim3(grid), dim3(kBlock), 0, c.stream, g, b, x, r, c.partial, done);
    else
        hipLaunchKernelGGL(k_residual<false>, dim3(grid), dim3(kBlock), 0, c.stream, g, b, x, r, c.partial, done);
}

template <bool NORM>
__global__ __launch_bounds__(kBlock) void k_matvec(Fine g, const double *__restrict__ x, double *__restrict__ y,
                                                   double *__restrict__ partial, const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    double acc = 0.0;
    const int lb = xcd_block();
    for (int t = lb * blockDim.x + threadIdx.x; t < g.N; t += gridDim.x * blockDim.x) {
        const int i = xzy_cell(t, g.nx, g.ny, g.nz);
        const double d = g.diag[i];
        const double ax = ax_row(g, x, i, d);
        const double v = d > 0.0 ? ax : 0.0;
        y[i] = v;
        acc += v * v;
    }
    if (NORM) {
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) partial[lb] = s;
    }
}

void launch_matvec(Ctx &c, const double *x, double *y, bool norm, const int *done) {
    ProfScope ps(c, MSRSB_K_MATVEC);
    Fine g = fine_of(c);
    const int grid = red_grid(c.N);
    if (norm)
        hipLaunchKernelGGL(k_matvec<true>, dim3(grid), dim3(kBlock), 0, c.stream, g, x, y, c.partial, done);
    else
        hipLaunchKernelGGL(k_matvec<false>, dim3(grid), dim3(kBlock), 0, c.stream, g, x, y, c.partial, done);
}

// Damped Jacobi: x += omega_s r / a_ii.
template <typename TT, bool ASSIGN>
__global__ void k_jacobi(int N, const TT *__restrict__ diag, TT omega, const double *__restrict__ r,
                         double *__restrict__ x, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const TT d = diag[i];
    if (ASSIGN) x[i] = d > (TT)0 ? (double)(omega * (TT)r[i] / d) : 0.0;
    else if (d > (TT)0) x[i] += (double)(omega * (TT)r[i] / d);
}

// Cell of colour `col` handled by thread t: rows (y,z) hold ceil(nx/2) slots.
// (rows visited z fastest, then y: see xzy_cell)
__device__ inline int colour_cell(const Fine &g, int col, int t) {
    const int hx = (g.nx + 1) >> 1;
    const int row = t / hx;
    if (row >= g.ny * g.nz) return -1;
    const int k = t - row * hx;
    const int iz = row % g.nz, iy = row / g.nz;
    const int ix = 2 * k + ((col + iy + iz) & 1);
    if (ix >= g.nx) return -1;
    return ix + g.nx * (iy + g.ny * iz);
}

// Red-black ILU(0) applied to r: with red cells first, L and U couple red to
// black only, so the forward pass leaves red rows unchanged and the backward
// pass is two colour sweeps.
//   black: e_b = (r_b + sum_{red l} T_bl r_l / a_ll) / dtil_b,
//   red:   e_r = (r_r + sum_{black l} T_rl e_l) / a_rr,
// x += e on each colour.  Faces with T = 0 (boundary, inactive neighbour)
// leave the sum untouched; cells with a non-positive pivot are skipped.
template <typename TT, bool ASSIGN>
__global__ __launch_bounds__(kBlock) void k_ilu_black(Fine g, const TT *__restrict__ tx, const TT *__restrict__ ty,
                                                      const TT *__restrict__ tz, const TT *__restrict__ diag,
                                                      const TT *__restrict__ dtil, const double *__restrict__ r,
                                                      double *__restrict__ e, double *__restrict__ x,
                                                      const int *done) {
    if (done && *done) return;
    const int i = colour_cell(g, 1, xcd_block() * blockDim.x + threadIdx.x);
    if (i < 0) return;
    int l[6];
    TT t[6], rl[6], dl[6];
    cell_faces(g, i, tx, ty, tz, l, t);
    const TT dt = dtil[i];
    TT s = (TT)r[i];
    const double xo = ASSIGN ? 0.0 : x[i];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        rl[q] = (TT)r[l[q]];
        dl[q] = diag[l[q]];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) s = t[q] != (TT)0 ? s + t[q] * (rl[q] / dl[q]) : s;
    const bool on = dt > (TT)0;
    const TT v = s / dt;
    e[i] = on ? (double)v : 0.0;
    x[i] = on ? (ASSIGN ? (double)v : xo + (double)v) : xo;
}

template <typename TT, bool ASSIGN>
__global__ __launch_bounds__(kBlock) void k_ilu_red(Fine g, const TT *__restrict__ tx, const TT *__restrict__ ty,
                                                    const TT *__restrict__ tz, const TT *__restrict__ diag,
                                                    const double *__restrict__ r, const double *__restrict__ e,
                                                    double *__restrict__ x, const int *done) {
    if (done && *done) return;
    const int i = colour_cell(g, 0, xcd_block() * blockDim.x + threadIdx.x);
    if (i < 0) return;
    int l[6];
    TT t[6], el[6];
    cell_faces(g, i, tx, ty, tz, l, t);
    const TT d = diag[i];
    TT s = (TT)r[i];
    const double xo = ASSIGN ? 0.0 : x[i];
#pragma unroll
    for (int q = 0; q < 6; ++q) el[q] = (TT)e[l[q]];
#pragma unroll
    for (int q = 0; q < 6; ++q) s = t[q] != (TT)0 ? s + t[q] * el[q] : s;
    x[i] = d > (TT)0 ? (ASSIGN ? (double)(s / d) : xo + (double)(s / d)) : xo;
}

// Both colours of the red-black ILU(0) application in one pass (rows of at
// most 62 cells).  A wavefront owns one row y with one halo lane on each side
// (lane l is x = l - 1); a workgroup holds kIluInner rows plus the row above
// and below, whose black corrections it computes for its own red cells.  The
// workgroup walks the layers of its z chunk, upward in even chunks and
// downward in odd ones, so that two neighbouring chunks read the layers
// around their common boundary at the same time (through the same L2).  Step
// L forms the black corrections of layer L (from r and the pivots of layers
// L-1..L+1) and the red corrections of the layer before it in the walk (from
// the black ones around it).  Each cell's ratio w = r / a_ii is formed once
// and shared: x neighbours from adjacent lanes, y neighbours through LDS (the
// outer neighbours of the two halo rows from memory), z neighbours in
// registers.  The loads of the next layer (and r, a_ii two layers ahead) are
// issued one step ahead of their use.  One barrier per step; x is read and
// written once.  The arithmetic per cell and the face order are those of
// k_ilu_black / k_ilu_red.
// 14 inner rows (1024 threads) measured fastest on the 60x220x85 model (6
// and 10 were slower): the halo rows cost 2/16 of the loads.
constexpr int kIluInner = 14, kIluRows = kIluInner + 2;

template <typename TT, bool ASSIGN>
__global__ __launch_bounds__(64 * kIluRows) void k_ilu_zm(Fine g, const TT *__restrict__ tx,
                                                           const TT *__restrict__ ty, const TT *__restrict__ tz,
                                                           const TT *__restrict__ diag, const TT *__restrict__ dtil,
                                                           const double *__restrict__ r, double *__restrict__ x,
                                                           int ngy, int nzc, int zc, int nblk, const int *done) {
    __shared__ TT eb[3][kIluRows][64];  // black corrections, by step mod 3
    __shared__ TT wb[2][kIluRows][64];  // w = r / a_ii, by step mod 2
    if (done && *done) return;
    const int b = xcd_block();
    if (b >= nblk) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = g.nxy;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int zk = b % nzc, yg = b / nzc;
    const int xr = lane - 1, y = yg * kIluInner - 1 + wv;
    const bool xin = xr >= 0 && xr < nx, yin = y >= 0 && y < ny;
    const bool inner = wv >= 1 && wv <= kIluInner && yin;
    const int xc = min(max(xr, 0), nx - 1), yc = min(max(y, 0), ny - 1);
    // faces of the (clamped) cell: rows and lanes outside the grid take the
    // neighbours of the cell they load, so every index stays inside the grid
    const bool fxm = xc > 0 && xr > 0, fym = yc > 0, fyp = yc + 1 < ny;
    const int z0 = zk * zc, z1 = min(nz, z0 + zc);
    const int col = xc + nx * yc;
    const int dym = fym ? nx : 0, dyp = fyp ? nx : 0;
    // the halo rows read their outer y neighbour from memory
    const bool top = wv == 0, bot = wv == kIluRows - 1;
    const int dout = top ? -dym : (bot ? dyp : 0);
    const int wup = wv > 0 ? wv - 1 : 0, wdn = wv + 1 < kIluRows ? wv + 1 : wv;
    auto at = [&](int L) { return col + nxy * min(max(L, 0), nz - 1); };
    // walk: black layers from Ls to Le (a halo layer at each end that exists),
    // red layers z0..z1-1; the last step only forms red
    const int dir = (zk & 1) ? -1 : 1;
    const int Ls = dir > 0 ? max(z0 - 1, 0) : min(z1, nz - 1);
    const int nsteps = dir > 0 ? z1 - Ls + 1 : Ls - z0 + 2;
    // tz of the face between layer L and L + dir (index of the lower layer)
    auto fz = [&](int L) { return at(dir > 0 ? L : L - 1); };
    // registers: own column at L - dir, L (w, r, a_ii), raw r, a_ii at L + dir;
    // faces of layer L and of the previous layer; z faces ahead (fa), behind
    // (fb) and behind the previous layer (fbb); the halo row's outer r, a_ii
    TT r0 = (TT)r[at(Ls)], d0 = diag[at(Ls)];
    TT w0 = r0 / d0;
    const int Lb = Ls - dir;
    const bool hasbeh = Lb >= 0 && Lb < nz;
    TT wm = hasbeh ? (TT)r[at(Lb)] / diag[at(Lb)] : (TT)0;
    TT rp = (TT)r[at(Ls + dir)], dp = diag[at(Ls + dir)];
    TT tx0 = tx[at(Ls)], ty0 = ty[at(Ls)], tym0 = ty[at(Ls) - dym], dt0 = dtil[at(Ls)];
    TT fa = tz[fz(Ls)], fb = hasbeh ? tz[fz(Lb)] : (TT)0, fbb = (TT)0;
    TT ro = (TT)0, dq = (TT)1;
    if (top || bot) {
        ro = (TT)r[at(Ls) + dout];
        dq = diag[at(Ls) + dout];
    }
    TT txp = (TT)0, typ = (TT)0, tymp = (TT)0, rprev = (TT)0, dprev = (TT)0;
    TT em = (TT)0, em2 = (TT)0;
    double xo = 0.0;
    wb[0][wv][lane] = w0;
    __syncthreads();
    for (int k = 0; k < nsteps; ++k) {
        const int L = Ls + k * dir;
        const bool hasb = L >= 0 && L < nz;  // the last step only forms red
        const int in1 = at(L + dir);
        // loads for the next step
        const TT rpn = (TT)r[at(L + 2 * dir)], dpn = diag[at(L + 2 * dir)];
        const TT txn = tx[in1], tyn = ty[in1], tymn = ty[in1 - dym], fan = tz[fz(L + dir)], dtn = dtil[in1];
        TT ron = (TT)0, don = (TT)1;
        if (top || bot) {  // wave-uniform: only the halo rows use the outer neighbour
            ron = (TT)r[in1 + dout];
            don = diag[in1 + dout];
        }
        const double xon = (ASSIGN || L < z0 || L >= z1) ? 0.0 : x[at(L)];
        // black corrections of layer L (faces -x, +x, -y, +y, -z, +z)
        const TT wp = rp / dp;
        TT e0 = (TT)0;
        {
            const TT wxm = __shfl_up(w0, 1, 64), wxp = __shfl_down(w0, 1, 64);
            const TT txm = __shfl_up(tx0, 1, 64);
            const TT wo = (top || bot) ? ro / dq : (TT)0;
            const TT wym = top ? wo : wb[k & 1][wup][lane], wyp = bot ? wo : wb[k & 1][wdn][lane];
            const TT tzl = dir > 0 ? fb : fa, tzu = dir > 0 ? fa : fb;  // faces to L - 1, L + 1
            const TT wzl = dir > 0 ? wm : wp, wzu = dir > 0 ? wp : wm;
            const TT t[6] = {fxm ? txm : (TT)0, tx0, fym ? tym0 : (TT)0, fyp ? ty0 : (TT)0,
                             L > 0 ? tzl : (TT)0, L + 1 < nz ? tzu : (TT)0};
            const TT wl[6] = {wxm, wxp, wym, wyp, wzl, wzu};
            TT sb = r0;
#pragma unroll
            for (int q = 0; q < 6; ++q) sb = t[q] != (TT)0 ? sb + t[q] * wl[q] : sb;
            const bool black = ((xr + y + L) & 1) == 1;
            const bool on = hasb && black && dt0 > (TT)0;
            const TT v = sb / dt0;
            e0 = on ? v : (TT)0;
        }
        eb[k % 3][wv][lane] = e0;
        wb[(k + 1) & 1][wv][lane] = wp;
        __syncthreads();
        // red corrections of the previous layer Lr = L - dir, and its stores
        const int Lr = L - dir;
        if (k > 0 && Lr >= z0 && Lr < z1) {
            const int kr = (k + 2) % 3;  // slot of step k - 1
            const TT exm = __shfl_up(em, 1, 64), exp_ = __shfl_down(em, 1, 64);
            const TT eym = eb[kr][wup][lane], eyp = eb[kr][wdn][lane];
            const TT txm = __shfl_up(txp, 1, 64);
            // faces of Lr: toward L is fb, away from L is fbb
            const TT tzl = dir > 0 ? fbb : fb, tzu = dir > 0 ? fb : fbb;
            const TT t[6] = {fxm ? txm : (TT)0, txp, fym ? tymp : (TT)0, fyp ? typ : (TT)0,
                             Lr > 0 ? tzl : (TT)0, Lr + 1 < nz ? tzu : (TT)0};
            const TT ezl = dir > 0 ? em2 : e0, ezu = dir > 0 ? e0 : em2;
            const TT el[6] = {exm, exp_, eym, eyp, ezl, ezu};
            TT sr = rprev;
            const bool red = ((xr + y + Lr) & 1) == 0;
            if (red) {
#pragma unroll
                for (int q = 0; q < 6; ++q) sr = t[q] != (TT)0 ? sr + t[q] * el[q] : sr;
            }
            double xn;
            if (red) xn = dprev > (TT)0 ? (ASSIGN ? (double)(sr / dprev) : xo + (double)(sr / dprev)) : xo;
            else xn = ASSIGN ? (double)em : xo + (double)em;  // em = 0 where the pivot is not positive
            if (inner && xin) x[at(Lr)] = xn;
        }
        // slide: layer L becomes the previous one, the prefetched layer the current
        em2 = em;
        em = e0;
        fbb = fb;
        fb = fa;
        fa = fan;
        txp = tx0;
        typ = ty0;
        tymp = tym0;
        rprev = r0;
        dprev = d0;
        wm = w0;
        w0 = wp;
        r0 = rp;
        d0 = dp;
        rp = rpn;
        dp = dpn;
        tx0 = txn;
        ty0 = tyn;
        tym0 = tymn;
        dt0 = dtn;
        ro = ron;
        dq = don;
        xo = xon;
    }
}

template <bool ASSIGN>
static void smooth_dispatch(Ctx &c, const double *r, double *x, const int *done) {
    Fine g = fine_of(c);
    const bool mixed = c.opt.precision == MSRSB_MIXED;
    if (c.opt.smoother == MSRSB_SMOOTH_ILU0_LINE) {
        launch_lilu_apply(c, r, x, done, ASSIGN);
        return;
    }
    if (c.opt.smoother == MSRSB_SMOOTH_JACOBI) {
        if (mixed)
            hipLaunchKernelGGL((k_jacobi<float, ASSIGN>), dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N,
                               c.diag32, (float)c.opt.omega_s, r, x, done);
        else
            hipLaunchKernelGGL((k_jacobi<double, ASSIGN>), dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N,
                               c.diag, c.opt.omega_s, r, x, done);
        return;
    }
    if (c.nx <= 62) {
        const int ngy = cdiv(c.ny, kIluInner);
        int nzc = std::min(c.nz, std::max(1, cdiv(4096, ngy * kIluRows)));
        const int zc = cdiv(c.nz, nzc);
        nzc = cdiv(c.nz, zc);
        const int nblk = nzc * ngy;
        const dim3 grid(xcd_grid(nblk)), blk(64 * kIluRows);
        if (mixed)
            hipLaunchKernelGGL((k_ilu_zm<float, ASSIGN>), grid, blk, 0, c.stream, g, c.tx32, c.ty32, c.tz32, c.diag32,
                               c.dtil32, r, x, ngy, nzc, zc, nblk, done);
        else
            hipLaunchKernelGGL((k_ilu_zm<double, ASSIGN>), grid, blk, 0, c.stream, g, c.tx, c.ty, c.tz, c.diag,
                               c.dtil, r, x, ngy, nzc, zc, nblk, done);
        return;
    }
    const int half = ((c.nx + 1) / 2) * c.ny * c.nz;
    const dim3 grid(xcd_grid(cdiv(half, kBlock)));
    if (mixed) {
        hipLaunchKernelGGL((k_ilu_black<float, ASSIGN>), grid, dim3(kBlock), 0, c.stream, g, c.tx32, c.ty32, c.tz32,
                           c.diag32, c.dtil32, r, c.e, x, done);
        hipLaunchKernelGGL((k_ilu_red<float, ASSIGN>), grid, dim3(kBlock), 0, c.stream, g, c.tx32, c.ty32, c.tz32,
                           c.diag32, r, c.e, x, done);
    } else {
        hipLaunchKernelGGL((k_ilu_black<double, ASSIGN>), grid, dim3(kBlock), 0, c.stream, g, c.tx, c.ty, c.tz,
                           c.diag, c.dtil, r, c.e, x, done);
        hipLaunchKernelGGL((k_ilu_red<double, ASSIGN>), grid, dim3(kBlock), 0, c.stream, g, c.tx, c.ty, c.tz, c.diag,
                           r, c.e, x, done);
    }
}

// x += S r, or x = S r (assign: x need not be initialised; inactive cells get 0).
void launch_smooth(Ctx &c, const double *r, double *x, const int *done, bool assign) {
    ProfScope ps(c, MSRSB_K_SMOOTH);
    if (assign) smooth_dispatch<true>(c, r, x, done);
    else smooth_dispatch<false>(c, r, x, done);
}

__device__ __forceinline__ void zero_inactive_body(int bid, int nblk, int N, const double *__restrict__ diag,
                                                   double *__restrict__ x) {
    const int i = bid * blockDim.x + threadIdx.x;
    if (i < N && !(diag[i] > 0.0)) x[i] = 0.0;
}

__global__ void k_zero_inactive(int N, const double *__restrict__ diag, double *__restrict__ x) {
    zero_inactive_body(blockIdx.x, gridDim.x, N, diag, x);
}

void launch_zero_inactive(Ctx &c, double *x) {
    hipLaunchKernelGGL(k_zero_inactive, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, c.diag, x);
}

// Start of a solve: status cleared, x zeroed on inactive cells, ||b||^2 into
// scal[1] and ||b|| (1 if b = 0) as the reference of the relative residual.
__device__ __forceinline__ void reset_body(Status *st, int *flag) {
    st->done = 0;
    st->iters = 0;
    st->flag = 0;
    st->jcur = 0;
    st->relres = 0.0;
    *flag = 0;
}

__global__ void k_reset(Status *st, int *flag) { reset_body(st, flag); }

__device__ __forceinline__ void set_bnorm_body(Status *st, const double *sq) {
    const double n = sqrt(*sq);
    st->bnorm = n > 0.0 ? n : 1.0;
}

__global__ void k_set_bnorm(Status *st, const double *sq) { set_bnorm_body(st, sq); }

// Fixed-order sum of the per-block partials of the last norm kernel.
__device__ __forceinline__ void norm_finish_body(const double *__restrict__ partial, int np, double *out,
                                                 const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    const double s = sum_partials(partial, np, lds);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kBlock) void k_norm_finish(const double *__restrict__ partial, int np, double *out,
                                                        const int *done) {
    norm_finish_body(partial, np, out, done);
}

void launch_norm_finish(Ctx &c, double *out_sq, const int *done) {
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(kBlock), 0, c.stream, c.partial, red_grid(c.N), out_sq, done);
}

// Richardson test after a full cycle: relres = ||r|| / ||b||.  scal[0] holds
// ||r||^2 of the current iterate.  `count` adds one iteration first.
__global__ void k_check(Status *st, const double *scal, double rtol, int max_iters, int count) {
    if (st->done) return;
    if (count) st->iters += 1;
    const double rel = sqrt(scal[0]) / st->bnorm;
    st->relres = rel;
    if (rel <= rtol || st->iters >= max_iters || !(rel == rel)) st->done = 1;
}

void launch_check(Ctx &c, double rtol, int max_iters, int count) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(1), 0, c.stream, c.status, c.scal, rtol, max_iters, count);
}

__global__ void k_fluxes(Fine g, const double *__restrict__ p, double *__restrict__ face) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    const double pi = p[i];
    double t;
    face[i] = (t = g.tx[i]) != 0.0 ? t * (pi - p[i + 1]) : 0.0;
    face[g.N + i] = (t = g.ty[i]) != 0.0 ? t * (pi - p[i + g.nx]) : 0.0;
    face[2 * (long)g.N + i] = (t = g.tz[i]) != 0.0 ? t * (pi - p[i + g.nxy]) : 0.0;
}

__global__ void k_bc_fluxes(int n, const int32_t *__restrict__ cell, const double *__restrict__ tr,
                            const double *__restrict__ val, const double *__restrict__ p, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = tr[k] * (p[cell[k]] - val[k]);
}

void launch_fluxes(Ctx &c, const double *p, double *face, double *bcf) {
    Fine g = fine_of(c);
    if (face) hipLaunchKernelGGL(k_fluxes, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, p, face);
    if (bcf && c.n_bc > 0)
        hipLaunchKernelGGL(k_bc_fluxes, dim3(cdiv(c.n_bc, kBlock)), dim3(kBlock), 0, c.stream, c.n_bc, c.bc_cell,
                           c.bc_trans, c.bc_value, p, bcf);
}

// ---------------------------------------------------------------- GMRES ----
// Classical Gram-Schmidt in two passes (CGS2): h = V^T w, w -= V h, twice.
// Dots use a fixed grid and a fixed-order final sum.

// partial[j][block] = sum over the block's cells of V_j w, eight vectors per
// pass over w (register accumulators, one combined reduction per pass).
__device__ __forceinline__ void multidot_body(int bid, int nblk, int N, const double *__restrict__ V, int k,
                                              const double *__restrict__ w, double *__restrict__ partial,
                                              const int *done) {
    __shared__ double red[8][kBlock / 64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < k; j0 += 8) {
        const int nb = min(8, k - j0);
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int i = bid * blockDim.x + threadIdx.x; i < N; i += nblk * blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nb) acc[q] += V[(long)(j0 + q) * N + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red[q][wv] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            double t = 0.0;
            for (int m = 0; m < (int)(blockDim.x >> 6); ++m) t += red[threadIdx.x][m];
            partial[(long)(j0 + threadIdx.x) * nblk + bid] = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_multidot(int N, const double *__restrict__ V, int k,
                                                     const double *__restrict__ w, double *__restrict__ partial,
                                                     const int *done) {
    multidot_body(blockIdx.x, gridDim.x, N, V, k, w, partial, done);
}

__device__ __forceinline__ void multidot_finish_body(int bid, int nblk, const double *__restrict__ partial, int np,
                                                     double *__restrict__ h, const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    const int j = bid;
    const double s = sum_partials(partial + (long)j * np, np, lds);
    if (threadIdx.x == 0) h[j] = s;
}

__global__ __launch_bounds__(kBlock) void k_multidot_finish(const double *__restrict__ partial, int np,
                                                            double *__restrict__ h, const int *done) {
    multidot_finish_body(blockIdx.x, gridDim.x, partial, np, h, done);
}

// Scalar layout in c.scal (device doubles):
//   [0]               norm^2 scratch
//   [8 .. 8+64)       h1 (first CGS pass)      [80 .. 144) h2 (second pass)
//   [160 .. 160+65*64) Hessenberg H (column-major, ld 65)
//   [4400 .. 4465)    g (rotated rhs)   [4480..4544) cs  [4544..4608) sn
//   [4608 .. 4672)    y (least-squares solution)   [4700] 1/h_{j+1,j}
constexpr int S_H1 = 8, S_H2 = 80, S_H = 160, S_G = 4400, S_CS = 4480, S_SN = 4544, S_Y = 4608, S_INV = 4700;

void launch_multidot(Ctx &c, const double *V, int k, const double *w, double *h_out, const int *done) {
    const int grid = red_grid(c.N);
    hipLaunchKernelGGL(k_multidot, dim3(grid), dim3(kBlock), 0, c.stream, c.N, V, k, w, c.partial, done);
    hipLaunchKernelGGL(k_multidot_finish, dim3(k), dim3(kBlock), 0, c.stream, c.partial, grid, h_out, done);
}

template <bool NORM, typename VT>
__device__ __forceinline__ void multiaxpy_body(int bid, int nblk, int N, const VT *__restrict__ V, int k,
                                               const double *__restrict__ h, double sign, double *__restrict__ w,
                                               double *__restrict__ partial, const int *done) {
    __shared__ double hs[kMaxRestart + 1];
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    double acc = 0.0;
    for (int i = bid * blockDim.x + threadIdx.x; i < N; i += nblk * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += hs[j] * (double)V[(long)j * N + i];
        const double v = w[i] + sign * s;
        w[i] = v;
        acc += v * v;
    }
    if (NORM) {
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) partial[bid] = s;
    }
}

template <bool NORM, typename VT>
__global__ __launch_bounds__(kBlock) void k_multiaxpy(int N, const VT *__restrict__ V, int k,
                                                      const double *__restrict__ h, double sign,
                                                      double *__restrict__ w, double *__restrict__ partial,
                                                      const int *done) {
    multiaxpy_body<NORM, VT>(blockIdx.x, gridDim.x, N, V, k, h, sign, w, partial, done);
}

template <typename VT>
static void multiaxpy_t(Ctx &c, const VT *V, int k, const double *h, double *w, double sign, bool norm,
                        const int *done) {
    const int grid = red_grid(c.N);
    if (norm)
        hipLaunchKernelGGL((k_multiaxpy<true, VT>), dim3(grid), dim3(kBlock), 0, c.stream, c.N, V, k, h, sign, w,
                           c.partial, done);
    else
        hipLaunchKernelGGL((k_multiaxpy<false, VT>), dim3(grid), dim3(kBlock), 0, c.stream, c.N, V, k, h, sign, w,
                           c.partial, done);
}

void launch_multiaxpy(Ctx &c, const double *V, int k, const double *h, double *w, double sign, bool norm,
                      const int *done) {
    multiaxpy_t<double>(c, V, k, h, w, sign, norm, done);
}

void launch_multiaxpy(Ctx &c, const float *V, int k, const double *h, double *w, double sign, bool norm,
                      const int *done) {
    multiaxpy_t<float>(c, V, k, h, w, sign, norm, done);
}

// Start of a restart cycle: beta = ||r|| (scal[0] holds ||r||^2), v0 = r/beta,
// g = beta e1.  Sets done when the current iterate already meets rtol or the
// iteration budget is spent; clears it otherwise.
__device__ __forceinline__ void gmres_begin_body(Status *st, double *scal, double rtol, int max_iters) {
    const double beta = sqrt(scal[0]);
    const double rel = beta / st->bnorm;
    st->relres = rel;
    st->jcur = 0;
    for (int j = 0; j <= kMaxRestart; ++j) scal[S_G + j] = 0.0;
    scal[S_G] = beta;
    scal[S_INV] = beta > 0.0 ? 1.0 / beta : 0.0;
    st->done = (rel <= rtol || st->iters >= max_iters || !(rel == rel)) ? 1 : 0;
}

__global__ void k_gmres_begin(Status *st, double *scal, double rtol, int max_iters) {
    gmres_begin_body(st, scal, rtol, max_iters);
}

__global__ void k_scale(int N, const double *__restrict__ w, double *__restrict__ v, const double *s, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) v[i] = w[i] * (*s);
}

void launch_gmres_start(Ctx &c, const double *r, double *v0, int /*restart*/) {
    hipLaunchKernelGGL(k_scale, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, r, v0, c.scal + S_INV,
                       (const int *)&c.status->done);
}

// Arnoldi step j: H(:,j) = h1 + h2, H(j+1,j) = ||w||; apply the previous
// Givens rotations, form rotation j, update g and the residual estimate.
__global__ void k_gmres_step(Status *st, double *scal, int j, double rtol, int max_iters, int restart) {
    if (st->done) return;
    double *H = scal + S_H;
    double *g = scal + S_G;
    double *cs = scal + S_CS;
    double *sn = scal + S_SN;
    const int ld = kMaxRestart + 1;
    for (int i = 0; i <= j; ++i) H[i + ld * j] = scal[S_H1 + i] + scal[S_H2 + i];
    const double hn = sqrt(scal[0]);
    H[j + 1 + ld * j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = H[i + ld * j], b = H[i + 1 + ld * j];
        H[i + ld * j] = cs[i] * a + sn[i] * b;
        H[i + 1 + ld * j] = -sn[i] * a + cs[i] * b;
    }
    const double a = H[j + ld * j], b = H[j + 1 + ld * j];
    const double rr = hypot(a, b);
    const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? b / rr : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    H[j + ld * j] = rr;
    H[j + 1 + ld * j] = 0.0;
    g[j + 1] = -sj * g[j];
    g[j] = cj * g[j];
    st->iters += 1;
    st->jcur = j + 1;
    const double rel = fabs(g[j + 1]) / st->bnorm;
    st->relres = rel;
    scal[S_INV] = hn > 0.0 ? 1.0 / hn : 0.0;
    if (rel <= rtol || st->iters >= max_iters || j + 1 >= restart || hn == 0.0 || !(rel == rel)) st->done = 1;
}

void launch_gmres_step(Ctx &c, int j, double rtol, int max_iters, int restart) {
    hipLaunchKernelGGL(k_gmres_step, dim3(1), dim3(1), 0, c.stream, c.status, c.scal, j, rtol, max_iters, restart);
}

void launch_gmres_scale(Ctx &c, const double *w, double *v, int /*j*/) {
    hipLaunchKernelGGL(k_scale, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, w, v, c.scal + S_INV,
                       (const int *)&c.status->done);
}

// Back substitution R y = g over the jcur completed steps.
// y = H^-1 g by back substitution (k = jcur columns); with zform also
// w = T^-1 y, so that M^-1 Q y = Z w for the stored candidates Z.  One
// wavefront stages the triangles and g in LDS; lane 0 then substitutes in the
// same order as a plain loop would (the global loads were its latency).
__device__ __forceinline__ void gmres_solve_small_body(Status *st, double *scal, int zform) {
    constexpr int KM = kMaxRestart;
    __shared__ double Hs[KM * KM];
    __shared__ double gs[KM], ys[KM];
    const double *H = scal + S_H;
    const double *g = scal + S_G;
    const int ld = kMaxRestart + 1;
    const int k = min(st->jcur, KM);
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e / k, m = e % k;
        Hs[e] = m >= i ? H[i + ld * m] : 0.0;
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double *y = scal + S_Y;
        for (int i = k - 1; i >= 0; --i) {
            double s = gs[i];
            for (int m = i + 1; m < k; ++m) s -= Hs[i * k + m] * ys[m];
            ys[i] = s / Hs[i * k + i];
            y[i] = ys[i];
        }
    }
    if (!zform) return;
    __syncthreads();
    const double *T = scal + kScalT;
    constexpr int lt = kDcgsMax + 1;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e / k, m = e % k;
        Hs[e] = m >= i ? T[i + lt * m] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *w = scal + kScalW;
        for (int i = k - 1; i >= 0; --i) {
            double s = ys[i];
            for (int m = i + 1; m < k; ++m) s -= Hs[i * k + m] * gs[m];
            gs[i] = s / Hs[i * k + i];  // gs now holds w
            w[i] = gs[i];
        }
    }
}

__global__ __launch_bounds__(64) void k_gmres_solve_small(Status *st, double *scal, int zform) {
    gmres_solve_small_body(st, scal, zform);
}

void launch_gmres_solve_small(Ctx &c, int /*restart*/, bool zform) {
    hipLaunchKernelGGL(k_gmres_solve_small, dim3(1), dim3(64), 0, c.stream, c.status, c.scal, zform ? 1 : 0);
}

__global__ void k_axpy(int N, double *__restrict__ x, const double *__restrict__ z, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] += z[i];
}

void launch_axpy(Ctx &c, double *x, const double *z, const int *done) {
    hipLaunchKernelGGL(k_axpy, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, x, z, done);
}

// Second Gram-Schmidt pass only when the first removed most of w
// (||w_after|| < 0.7 ||w_before||, the Daniel-Gragg-Kaufman-Stewart test);
// scal[2] = ||w_before||^2, scal[0] = ||w_after||^2.  Clears h2 either way.
__global__ void k_reorth_check(Status *st, double *scal, int k) {
    for (int i = 0; i < k; ++i) scal[S_H2 + i] = 0.0;
    st->skip2 = (st->done || !(scal[0] < 0.49 * scal[2])) ? 1 : 0;
}

void launch_reorth_check(Ctx &c, int k) {
    hipLaunchKernelGGL(k_reorth_check, dim3(1), dim3(1), 0, c.stream, c.status, c.scal, k);
}

// ---- fused Arnoldi step (w = A z, two Gram-Schmidt passes, norm) ----------
// Partials are laid out partial[q*grid + block] for dot q and
// partial[nd*grid + block] for the squared norm; the finish kernels add them
// in block order, one wavefront per quantity.

// w = A z; partial dots V_q^T w (q < k) and ||w||^2.
__global__ __launch_bounds__(kBlock) void k_mvdot(Fine g, const double *__restrict__ z, double *__restrict__ w,
                                                  const double *__restrict__ V, int k, double *__restrict__ partial,
                                                  const int *done) {
    __shared__ double red[9][kBlock / 64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, G = gridDim.x;
    double nrm = 0.0;
    for (int j0 = 0; j0 < k; j0 += 8) {
        const int nb = min(8, k - j0);
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += G * blockDim.x) {
            double wi;
            if (j0 == 0) {
                const double d = g.diag[i];
                const double ax = ax_row(g, z, i, d);
                wi = d > 0.0 ? ax : 0.0;
                w[i] = wi;
                nrm += wi * wi;
            } else {
                wi = w[i];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nb) acc[q] += V[(long)(j0 + q) * g.N + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red[q][wv] = v;
        }
        const double vn = wave_sum(nrm);
        if (lane == 0) red[8][wv] = vn;
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            double t = 0.0;
            for (int m = 0; m < (int)(blockDim.x >> 6); ++m) t += red[threadIdx.x][m];
            partial[(long)(j0 + threadIdx.x) * G + blockIdx.x] = t;
        }
        if (j0 == 0 && threadIdx.x == 8) {
            double t = 0.0;
            for (int m = 0; m < (int)(blockDim.x >> 6); ++m) t += red[8][m];
            partial[(long)kMaxRestart * 2 * G + blockIdx.x] = t;  // norm slot
        }
        __syncthreads();
    }
}

// Register-resident forms for k < KM basis vectors: every element of V is
// read once per kernel.  A thread keeps the KM - 1 dot accumulators (and
// the squared norm in the last slot); loads past k are clamped to vector
// k - 1 and weighted by zero, so no load sits behind a branch.  Totals per
// workgroup by group_sum_lds (fixed order).
template <int KM>
__global__ __launch_bounds__(kBlock) void k_mvdot_r(Fine g, const double *__restrict__ z, double *__restrict__ w,
                                                    const double *__restrict__ V, int k,
                                                    double *__restrict__ partial, const int *done) {
    __shared__ double red[(kBlock / 64 + 1) * KM];
    if (done && *done) return;
    const int G = gridDim.x;
    double acc[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += G * blockDim.x) {
        double vq[KM - 1];
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) vq[q] = V[(long)min(q, k - 1) * g.N + i];
        // faces as in cell_faces, with the zeroing applied after the loads
        const int step[3] = {1, g.nx, g.nxy};
        bool in[6];
        int l[6];
        double traw[6], xl[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double *Ta = a == 0 ? g.tx : (a == 1 ? g.ty : g.tz);
            in[2 * a] = i >= step[a];
            in[2 * a + 1] = i + step[a] < g.N;
            l[2 * a] = in[2 * a] ? i - step[a] : i;
            l[2 * a + 1] = in[2 * a + 1] ? i + step[a] : i;
            traw[2 * a] = Ta[l[2 * a]];
            traw[2 * a + 1] = Ta[i];
        }
        const double d = g.diag[i], xi = z[i];
#pragma unroll
        for (int q = 0; q < 6; ++q) xl[q] = z[l[q]];
        __builtin_amdgcn_sched_barrier(0);  // all loads of the element first
        double ax = d * xi;                 // (A z)_i, as ax_row
#pragma unroll
        for (int q = 0; q < 6; ++q) ax -= (in[q] ? traw[q] : 0.0) * xl[q];
        const double wi = d > 0.0 ? ax : 0.0;
        w[i] = wi;
        acc[KM - 1] += wi * wi;
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) acc[q] += vq[q] * (q < k ? wi : 0.0);
    }
    group_sum_lds<KM>(acc, red);
    const int nw = blockDim.x >> 6;
    if ((int)threadIdx.x < k) partial[(long)threadIdx.x * G + blockIdx.x] = red[nw * KM + threadIdx.x];
    if (threadIdx.x == KM - 1) partial[(long)kMaxRestart * 2 * G + blockIdx.x] = red[nw * KM + KM - 1];
}

// w -= V h (first pass), ||w||^2, and when the second pass is due the dots
// V^T w of the updated w, from the same loads of V.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_axpy_dot_r(int N, const double *__restrict__ V, int k,
                                                       const double *__restrict__ h, double *__restrict__ w,
                                                       double *__restrict__ partial, const Status *st,
                                                       const double *scal);

// Whether a second Gram-Schmidt pass is due, from ||w - V h||^2 =
// ||w||^2 - ||h||^2 (V orthonormal): iff that is < 0.49 ||w||^2 (the DGKS
// test ||w'|| < 0.7 ||w||).  Every kernel that needs the decision evaluates
// this same expression on the same scalars.
__device__ inline bool second_pass(const double *scal, int k) {
    double hh = 0.0;
    for (int q = 0; q < k; ++q) hh += scal[S_H1 + q] * scal[S_H1 + q];
    return scal[2] - hh < 0.49 * scal[2];
}

// One wavefront per quantity: out[q] = sum of dot partials q (q < nd), *nout
// = sum of the norm partials (q == nd); fixed order.  mode 2 (after the first
// update): when no second pass is due the dots are not summed and out
// (h2) is cleared instead.
__global__ __launch_bounds__(kBlock) void k_finish_dots(const double *__restrict__ partial, int G, int nd,
                                                       double *__restrict__ out, double *nout, const Status *st,
                                                       const double *scal, int mode) {
    __shared__ double lds[kBlock / 64];
    if (st->done) return;
    const int q = blockIdx.x;
    if (mode == 2 && q < nd && !second_pass(scal, nd)) {
        if (threadIdx.x == 0) out[q] = 0.0;
        return;
    }
    const long base = q < nd ? (long)q * G : (long)kMaxRestart * 2 * G;
    const double t = sum_partials(partial + base, G, lds);
    if (threadIdx.x == 0) {
        if (q < nd) out[q] = t;
        else *nout = t;
    }
}

// w -= V h1; if a second pass follows, partial dots V_q^T w; always ||w||^2.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_axpy_dot_r(int N, const double *__restrict__ V, int k,
                                                       const double *__restrict__ h, double *__restrict__ w,
                                                       double *__restrict__ partial, const Status *st,
                                                       const double *scal) {
    __shared__ double red[(kBlock / 64 + 1) * KM];
    if (st->done) return;
    const bool dots = second_pass(scal, k);
    const int G = gridDim.x;
    double hq[KM - 1];
#pragma unroll
    for (int q = 0; q < KM - 1; ++q) {
        const double hv = h[min(q, k - 1)];
        hq[q] = q < k ? hv : 0.0;
    }
    double acc[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += G * blockDim.x) {
        double vq[KM - 1];
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) vq[q] = V[(long)min(q, k - 1) * N + i];
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < KM - 1; ++q)
            if (q < k) sacc += hq[q] * vq[q];
        const double v = w[i] - sacc;
        w[i] = v;
        acc[KM - 1] += v * v;
        if (dots) {
#pragma unroll
            for (int q = 0; q < KM - 1; ++q) acc[q] += vq[q] * (q < k ? v : 0.0);
        }
    }
    group_sum_lds<KM>(acc, red);
    const int nw = blockDim.x >> 6;
    if (dots && (int)threadIdx.x < k) partial[(long)threadIdx.x * G + blockIdx.x] = red[nw * KM + threadIdx.x];
    if (threadIdx.x == KM - 1) partial[(long)kMaxRestart * 2 * G + blockIdx.x] = red[nw * KM + KM - 1];
}

__global__ __launch_bounds__(kBlock) void k_axpy_dot(int N, const double *__restrict__ V, int k,
                                                     const double *__restrict__ h, double *__restrict__ w,
                                                     double *__restrict__ partial, const Status *st,
                                                     const double *scal) {
    __shared__ double hs[kMaxRestart + 1];
    __shared__ double red[9][kBlock / 64];
    if (st->done) return;
    const bool dots = second_pass(scal, k);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, G = gridDim.x;
    for (int q = threadIdx.x; q < k; q += blockDim.x) hs[q] = h[q];
    __syncthreads();
    double nrm = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += G * blockDim.x) {
        double sacc = 0.0;
        for (int q = 0; q < k; ++q) sacc += hs[q] * V[(long)q * N + i];
        const double v = w[i] - sacc;
        w[i] = v;
        nrm += v * v;
    }
    {
        const double vn = wave_sum(nrm);
        if (lane == 0) red[8][wv] = vn;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int m = 0; m < (int)(blockDim.x >> 6); ++m) t += red[8][m];
            partial[(long)kMaxRestart * 2 * G + blockIdx.x] = t;
        }
        __syncthreads();
    }
    if (!dots) return;
    for (int j0 = 0; j0 < k; j0 += 8) {
        const int nb = min(8, k - j0);
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += G * blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nb) acc[q] += V[(long)(j0 + q) * N + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red[q][wv] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            double t = 0.0;
            for (int m = 0; m < (int)(blockDim.x >> 6); ++m) t += red[threadIdx.x][m];
            partial[(long)(j0 + threadIdx.x) * G + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// Second pass: w -= V h2 and ||w||^2 partials (only when a second pass is due).
__global__ __launch_bounds__(kBlock) void k_axpy_norm(int N, const double *__restrict__ V, int k,
                                                      const double *__restrict__ h, double *__restrict__ w,
                                                      double *__restrict__ partial, const Status *st,
                                                      const double *scal) {
    __shared__ double hs[kMaxRestart + 1];
    __shared__ double lds[kBlock / 64];
    if (st->done || !second_pass(scal, k)) return;
    const int G = gridDim.x;
    for (int q = threadIdx.x; q < k; q += blockDim.x) hs[q] = h[q];
    __syncthreads();
    double nrm = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += G * blockDim.x) {
        double sacc = 0.0;
        for (int q = 0; q < k; ++q) sacc += hs[q] * V[(long)q * N + i];
        const double v = w[i] - sacc;
        w[i] = v;
        nrm += v * v;
    }
    const double t = block_sum(nrm, lds);
    if (threadIdx.x == 0) partial[(long)kMaxRestart * 2 * G + blockIdx.x] = t;
}

// Norm of the orthogonalised w (second pass if any) then Arnoldi step j:
// H(:,j) = h1 + h2, H(j+1,j) = ||w||, Givens rotations, residual estimate.
__global__ __launch_bounds__(kBlock) void k_gmres_step2(Status *st, double *scal, const double *__restrict__ partial,
                                                       int G, int j, double rtol, int max_iters, int restart) {
    __shared__ double lds[kBlock / 64];
    if (st->done) return;
    double hn2;
    if (second_pass(scal, j + 1)) hn2 = sum_partials(partial + (long)kMaxRestart * 2 * G, G, lds);
    else hn2 = scal[3];
    // the new Hessenberg column and the previous rotations, staged in LDS
    __shared__ double col[kMaxRestart + 1], rc[kMaxRestart], rs[kMaxRestart];
    double *H = scal + S_H;
    double *gv = scal + S_G;
    double *cs = scal + S_CS;
    double *sn = scal + S_SN;
    const int ld = kMaxRestart + 1;
    const double hn = sqrt(hn2);
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) col[i] = i <= j ? scal[S_H1 + i] + scal[S_H2 + i] : hn;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        rc[i] = cs[i];
        rs[i] = sn[i];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double a_i = col[0];
    for (int i = 0; i < j; ++i) {
        const double b = col[i + 1];
        H[i + ld * j] = rc[i] * a_i + rs[i] * b;
        a_i = -rs[i] * a_i + rc[i] * b;
    }
    const double a = a_i, b = hn;
    const double rr = hypot(a, b);
    const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? b / rr : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    H[j + ld * j] = rr;
    H[j + 1 + ld * j] = 0.0;
    gv[j + 1] = -sj * gv[j];
    gv[j] = cj * gv[j];
    st->iters += 1;
    st->jcur = j + 1;
    const double rel = fabs(gv[j + 1]) / st->bnorm;
    st->relres = rel;
    scal[S_INV] = hn > 0.0 ? 1.0 / hn : 0.0;
    if (rel <= rtol || st->iters >= max_iters || j + 1 >= restart || hn == 0.0 || !(rel == rel)) st->done = 1;
}

// ---- GMRES with delayed reorthogonalisation (DCGS2) -------------------------
// Column j is formed from u_j, the once-orthogonalised candidate for q_j
// (u_0 = r).  Pass A: w = A M^{-1} u_j (z given) and the dots s = Q^T u_j,
// alpha = u_j.u_j, t = Q^T w, beta = u_j.w.  The step kernel finalises
// column j-1 (H(:,j-1) += s, H(j,j-1) = rho = sqrt(alpha - s.s), Givens,
// residual estimate) and forms column j in the small space:
//   g = H(0..j, 0..j-1) s,  h = ([t; (beta - s.t)/rho] - g) / rho,
// since A M^{-1} q_j = (w - Q_{j+1} g)/rho.  Pass B writes
//   q_j = (u_j - Q s)/rho  and  u_{j+1} = w/rho - Q_{j+1} (g/rho + h).
// Q = V(0..j-1) is read once per pass.  Scalars: totals of pass A at S_DA,
// unrotated Hessenberg at S_HU, update coefficients at S_DC, 1/rho at S_RHO.
constexpr int S_HU = 8192, S_DA = 12500, S_DC = 12700, S_RHO = 12800;

template <int KM, bool MV, typename VT>
__device__ __forceinline__ void dpass_a_body(int bid, int nblk, Fine g, const double *__restrict__ z,
                                             double *__restrict__ w, const VT *__restrict__ Q,
                                             const double *__restrict__ u, int j, double *__restrict__ partial,
                                             const int *done) {
    __shared__ double red[(kBlock / 64 + 1) * KM];
    if (done && *done) return;
    const int G = nblk;
    double as[KM], at[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) {
        as[q] = 0.0;
        at[q] = 0.0;
    }
    const int jc = j > 0 ? j - 1 : 0;
    const int lb = xcd_block(bid, nblk);
    const int ch = ((g.N + G - 1) / G + 63) & ~63;
    const int i0 = lb * ch, i1 = min(g.N, i0 + ch);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double vq[KM - 1];
#pragma unroll
        // slots q >= j are unused.  An FP64 basis skips their loads (a uniform
        // branch per slot: 31.0 against 32.8 us for the 16-vector pass on the
        // 60x220x85 model); an FP32 basis loads slot j - 1 in their place,
        // which measured far faster there than the branches (21.3 against 36.9 us)
        for (int q = 0; q < KM - 1; ++q) {
            if constexpr (std::is_same<VT, double>::value) vq[q] = q < j ? Q[(long)q * g.N + i] : 0.0;
            else vq[q] = (double)Q[(long)min(q, jc) * g.N + i];
        }
        const double ui = u[i];
        const int step[3] = {1, g.nx, g.nxy};
        bool in[6];
        double traw[6], xl[6], d = 0.0, xi = 0.0;
        if (MV) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double *Ta = a == 0 ? g.tx : (a == 1 ? g.ty : g.tz);
                in[2 * a] = i >= step[a];
                in[2 * a + 1] = i + step[a] < g.N;
                const int ld = in[2 * a] ? i - step[a] : i, lu = in[2 * a + 1] ? i + step[a] : i;
                traw[2 * a] = Ta[ld];
                traw[2 * a + 1] = Ta[i];
                xl[2 * a] = z[ld];
                xl[2 * a + 1] = z[lu];
            }
            d = g.diag[i];
            xi = z[i];
        }
        __builtin_amdgcn_sched_barrier(0);  // all loads of the element first
        as[KM - 1] += ui * ui;
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) as[q] += vq[q] * (q < j ? ui : 0.0);
        if (MV) {
            double ax = d * xi;  // (A z)_i, as ax_row
#pragma unroll
            for (int q = 0; q < 6; ++q) ax -= (in[q] ? traw[q] : 0.0) * xl[q];
            const double wi = d > 0.0 ? ax : 0.0;
            w[i] = wi;
            at[KM - 1] += ui * wi;
#pragma unroll
            for (int q = 0; q < KM - 1; ++q) at[q] += vq[q] * (q < j ? wi : 0.0);
        }
    }
    const int nw = blockDim.x >> 6;
    group_sum_lds<KM>(as, red);
    if ((int)threadIdx.x < j) partial[(long)threadIdx.x * G + lb] = red[nw * KM + threadIdx.x];
    if (threadIdx.x == KM - 1) partial[(long)j * G + lb] = red[nw * KM + KM - 1];
    if (MV) {
        group_sum_lds<KM>(at, red);
        if ((int)threadIdx.x < j) partial[(long)(j + 1 + threadIdx.x) * G + lb] = red[nw * KM + threadIdx.x];
        if (threadIdx.x == KM - 1) partial[(long)(2 * j + 1) * G + lb] = red[nw * KM + KM - 1];
    }
}

template <int KM, bool MV, typename VT>
__global__ __launch_bounds__(kBlock) void k_dpass_a(Fine g, const double *__restrict__ z, double *__restrict__ w,
                                                    const VT *__restrict__ Q, const double *__restrict__ u,
                                                    int j, double *__restrict__ partial, const int *done) {
    dpass_a_body<KM, MV, VT>(blockIdx.x, gridDim.x, g, z, w, Q, u, j, partial, done);
}

// out[q] = sum over blocks of partial[q*G + b], one workgroup per quantity.
__device__ __forceinline__ void finish_n_body(int bid, int nblk, const double *__restrict__ partial, int G,
                                              double *__restrict__ out, const Status *st) {
    __shared__ double lds[kBlock / 64];
    if (st->done) return;
    const double t = sum_partials(partial + (long)bid * G, G, lds);
    if (threadIdx.x == 0) out[bid] = t;
}

__global__ __launch_bounds__(kBlock) void k_finish_n(const double *__restrict__ partial, int G,
                                                     double *__restrict__ out, const Status *st) {
    finish_n_body(blockIdx.x, gridDim.x, partial, G, out, st);
}

// Finalise column j-1 and (unless final) prepare column j.  The pass-A
// totals and the needed part of the unrotated Hessenberg matrix are staged
// in LDS; sums run in index order.
// With G > 0 the step first forms the pass-A totals itself from the G
// per-block partials (one wavefront per total, lanes over the blocks, then
// the fixed wavefront tree) and stores them where pass B reads them; used
// when the grid of pass A is small enough that a separate finishing launch
// would cost more than the sums.
constexpr int kDstepFuseBlocks = 256;

// Grid of pass A: at most three workgroups per CU (256 CUs), so that with the
// FP64 matrix-vector form (about 133 VGPRs, three wavefronts per SIMD) every
// workgroup is resident at once and each XCD gets the same number.  On the
// 60x220x85 model this ran the 16-vector pass in 32.9 instead of 36.0 us
// (FP32 basis: 21.2 instead of 26.0 us) against the 2048 blocks of the other
// reductions; 512 was close, and 640 or 384 (uneven per CU) slower.
constexpr int kPassABlocks = 768;

__device__ __forceinline__ void dstep_body(Status *st, double *scal, int j, double rtol, int max_iters, int final_,
                                           const double *__restrict__ partial, int G) {
    constexpr int HL = kDcgsMax + 2;  // rows of the staged Hessenberg block
    __shared__ double Hs[HL][HL];     // Hs[l][i] = Hu(l, i)
    __shared__ double rcs[kDcgsMax + 1], rsn[kDcgsMax + 1], gv[kDcgsMax + 2];
    __shared__ double A[2 * kDcgsMax + 4];  // s[0..j), alpha, t[0..j), beta
    __shared__ double sh[3];
    __shared__ int stop;
    if (st->done) return;
    const int tid = threadIdx.x;
    const int ld = kMaxRestart + 1;
    double *Hu = scal + S_HU;
    double *H = scal + S_H;
    double *gg = scal + S_G;
    double *cs = scal + S_CS;
    double *sn = scal + S_SN;
    const int na = final_ ? j + 1 : 2 * j + 2;
    if (G > 0) {
        const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
        for (int q = wv; q < na; q += nwv) {
            double v = lane_strided_sum(partial + (long)q * G, lane, G);
            v = wave_sum(v);
            if (lane == 0) {
                A[q] = v;
                scal[S_DA + q] = v;
            }
        }
    } else {
        for (int i = tid; i < na; i += blockDim.x) A[i] = scal[S_DA + i];
    }
    // columns 0..j-1, rows 0..j (upper Hessenberg: rows up to i + 1)
    for (int e = tid; e < j * (j + 1); e += blockDim.x) {
        const int i = e / (j + 1), l = e % (j + 1);
        Hs[l][i] = l <= i + 1 ? Hu[l + ld * i] : 0.0;
    }
    for (int i = tid; i + 1 < j; i += blockDim.x) {
        rcs[i] = cs[i];
        rsn[i] = sn[i];
    }
    __syncthreads();
    if (tid < 64) {
        // s.s and s.t: lane sums in index order, then the fixed wave tree
        double ss = 0.0, sdt = 0.0;
        for (int i = tid; i < j; i += 64) {
            ss += A[i] * A[i];
            if (!final_) sdt += A[i] * A[j + 1 + i];
        }
        ss = wave_sum(ss);
        sdt = wave_sum(sdt);
        if (tid == 0) {
            const double r2 = A[j] - ss;
            sh[0] = r2 > 0.0 ? sqrt(r2) : 0.0;
            sh[1] = sdt;
            stop = 0;
        }
    }
    __syncthreads();
    const double rho = sh[0];
    // column j of T: q_j = (u_j - Q s) / rho, so M^-1 u_j = M^-1 Q s + rho M^-1 q_j
    if (!final_)
        for (int i = tid; i <= j; i += blockDim.x) scal[kScalT + i + (kDcgsMax + 1) * j] = i < j ? A[i] : rho;
    if (j > 0) {
        // finalise column j-1 of the Arnoldi matrix and of its rotated copy
        const int c = j - 1;
        for (int i = tid; i <= j; i += blockDim.x) {
            const double v = i < j ? Hs[i][c] + A[i] : rho;
            Hs[i][c] = v;
            Hu[i + ld * c] = v;
        }
        __syncthreads();
        if (tid == 0) {
            double a_i = Hs[0][c];
            for (int i = 0; i < c; ++i) {
                const double b = Hs[i + 1][c];
                H[i + ld * c] = rcs[i] * a_i + rsn[i] * b;
                a_i = -rsn[i] * a_i + rcs[i] * b;
            }
            const double a = a_i, b = Hs[c + 1][c];
            const double rr = hypot(a, b);
            const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? b / rr : 0.0;
            cs[c] = cj;
            sn[c] = sj;
            H[c + ld * c] = rr;
            H[c + 1 + ld * c] = 0.0;
            gg[c + 1] = -sj * gg[c];
            gg[c] = cj * gg[c];
            st->iters += 1;
            st->jcur = j;
            const double rel = fabs(gg[c + 1]) / st->bnorm;
            st->relres = rel;
            if (rel <= rtol || st->iters >= max_iters || !(rho > 0.0) || !(rel == rel) || final_) {
                st->done = 1;
                stop = 1;
            }
        }
        __syncthreads();
        if (stop) return;
    } else {
        if (tid == 0) {
            gg[0] = rho;  // ||r|| as used by q_0 = r / rho
            if (!(rho > 0.0)) {
                st->done = 1;
                stop = 1;
            }
        }
        __syncthreads();
        if (stop) return;
    }
    // column j: g = H(0..j, 0..j-1) s (upper Hessenberg)
    for (int l = tid; l <= j; l += blockDim.x) {
        double v = 0.0;
        for (int i = (l > 0 ? l - 1 : 0); i < j; ++i) v += Hs[l][i] * A[i];
        gv[l] = v;
    }
    __syncthreads();
    const double irho = 1.0 / rho;
    const double beta = A[2 * j + 1], sdt = sh[1];
    for (int l = tid; l <= j; l += blockDim.x) {
        const double proj = l < j ? A[j + 1 + l] : (beta - sdt) * irho;
        const double h = (proj - gv[l]) * irho;
        Hu[l + ld * j] = h;
        scal[S_DC + l] = gv[l] * irho + h;
    }
    if (tid == 0) scal[S_RHO] = irho;
}

__global__ __launch_bounds__(kBlock) void k_dstep(Status *st, double *scal, int j, double rtol, int max_iters,
                                                  int final_, const double *__restrict__ partial, int G) {
    dstep_body(st, scal, j, rtol, max_iters, final_, partial, G);
}

// q_j = (u_j - Q s) / rho into qout, u_{j+1} = w / rho - Q c(0..j-1) - c_j q_j
// into unext (qout may alias u).  q_j enters u_{j+1} as stored (rounded to
// VT), so u_{j+1} is formed against the basis that is kept.
template <int KM, typename VT>
__device__ __forceinline__ void dpass_b_body(int bid, int nblk, int N, const VT *__restrict__ Q, const double *u,
                                             const double *__restrict__ w, int j, VT *qout, double *__restrict__ unext,
                                             const double *__restrict__ scal, const Status *st) {
    if (st->done) return;
    const int jc = j > 0 ? j - 1 : 0;
    double sq[KM - 1], cq[KM - 1];
#pragma unroll
    for (int q = 0; q < KM - 1; ++q) {
        const double sv = scal[S_DA + min(q, jc)], cv = scal[S_DC + min(q, jc)];
        sq[q] = q < j ? sv : 0.0;
        cq[q] = q < j ? cv : 0.0;
    }
    const double cj = scal[S_DC + j], irho = scal[S_RHO];
    const int ch = ((N + nblk - 1) / nblk + 63) & ~63;
    const int i0 = xcd_block(bid, nblk) * ch, i1 = min(N, i0 + ch);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double vq[KM - 1];
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) {
            const double v = (double)Q[(long)min(q, jc) * N + i];
            vq[q] = q < j ? v : 0.0;  // unused slots may hold anything (V(0) before its first write)
        }
        const double ui = u[i], wi = w[i];
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < KM - 1; ++q) {
            a += sq[q] * vq[q];
            b += cq[q] * vq[q];
        }
        const VT qs = (VT)((ui - a) * irho);
        qout[i] = qs;
        unext[i] = wi * irho - (b + cj * (double)qs);
    }
}

template <int KM, typename VT>
__global__ __launch_bounds__(kBlock) void k_dpass_b(int N, const VT *__restrict__ Q, const double *u,
                                                    const double *__restrict__ w, int j, VT *qout,
                                                    double *__restrict__ unext, const double *__restrict__ scal,
                                                    const Status *st) {
    dpass_b_body<KM, VT>(blockIdx.x, gridDim.x, N, Q, u, w, j, qout, unext, scal, st);
}

template <int KM, typename VT>
static void dgmres_step_k(Ctx &c, const VT *Q, VT *qout, double *unext, const double *z, double *w, const double *u,
                          int j, double rtol, int max_iters, bool final_) {
    Fine g = fine_of(c);
    const int G = red_grid(c.N), GA = std::min(G, kPassABlocks);
    const int *done = &c.status->done;
    const Status *st = c.status;
    {
        ProfScope ps(c, final_ ? MSRSB_K_ORTHO : MSRSB_K_MATVEC);
        if (final_)
            hipLaunchKernelGGL((k_dpass_a<KM, false, VT>), dim3(GA), dim3(kBlock), 0, c.stream, g, z, w, Q, u, j,
                               c.partial, done);
        else
            hipLaunchKernelGGL((k_dpass_a<KM, true, VT>), dim3(GA), dim3(kBlock), 0, c.stream, g, z, w, Q, u, j,
                               c.partial, done);
    }
    const bool fuse = GA <= kDstepFuseBlocks;
    if (!fuse)
        hipLaunchKernelGGL(k_finish_n, dim3(final_ ? j + 1 : 2 * j + 2), dim3(kBlock), 0, c.stream, c.partial, GA,
                           c.scal + S_DA, st);
    hipLaunchKernelGGL(k_dstep, dim3(1), dim3(kBlock), 0, c.stream, c.status, c.scal, j, rtol, max_iters,
                       final_ ? 1 : 0, c.partial, fuse ? GA : 0);
    if (final_) return;
    ProfScope ps(c, MSRSB_K_ORTHO);
    hipLaunchKernelGGL((k_dpass_b<KM, VT>), dim3(G), dim3(kBlock), 0, c.stream, c.N, Q, u, w, j, qout, unext, c.scal,
                       st);
}

template <typename VT>
static void dgmres_step_t(Ctx &c, const VT *Q, VT *qout, double *unext, const double *z, double *w, const double *u,
                          int j, double rtol, int max_iters, bool final_) {
    if (j <= 7) dgmres_step_k<8, VT>(c, Q, qout, unext, z, w, u, j, rtol, max_iters, final_);
    else if (j <= 15) dgmres_step_k<16, VT>(c, Q, qout, unext, z, w, u, j, rtol, max_iters, final_);
    else dgmres_step_k<32, VT>(c, Q, qout, unext, z, w, u, j, rtol, max_iters, final_);
}

// One DCGS2 Arnoldi step for column j (final: only finalise column j - 1).
// FP64 basis: q_j overwrites u_j in V(j) and u_{j+1} goes to V(j + 1).  FP32
// basis (Vf set): q_j goes to Vf(j) and the candidates alternate between V(0)
// and V(1).
void launch_dgmres_step(Ctx &c, const double *z, double *w, const double *u, int j, double rtol, int max_iters,
                        bool final_) {
    const long N = c.N;
    if (c.Vf)
        dgmres_step_t<float>(c, c.Vf, c.Vf + (long)j * N, c.V + (long)((j + 1) & 1) * N, z, w, u, j, rtol, max_iters, final_);
    else
        dgmres_step_t<double>(c, c.V, c.V + (long)j * N, c.V + (long)(j + 1) * N, z, w, u, j, rtol, max_iters, final_);
}

void launch_arnoldi(Ctx &c, const double *z, double *w, int j, double rtol, int max_iters, int restart) {
    Fine g = fine_of(c);
    const int G = red_grid(c.N);
    const int *done = &c.status->done;
    const int k = j + 1;
    {
        ProfScope ps(c, MSRSB_K_MATVEC);
        if (k <= 7)
            hipLaunchKernelGGL(k_mvdot_r<8>, dim3(G), dim3(kBlock), 0, c.stream, g, z, w, c.V, k, c.partial, done);
        else if (k <= 15)
            hipLaunchKernelGGL(k_mvdot_r<16>, dim3(G), dim3(kBlock), 0, c.stream, g, z, w, c.V, k, c.partial, done);
        else if (k <= 31)
            hipLaunchKernelGGL(k_mvdot_r<32>, dim3(G), dim3(kBlock), 0, c.stream, g, z, w, c.V, k, c.partial, done);
        else
            hipLaunchKernelGGL(k_mvdot, dim3(G), dim3(kBlock), 0, c.stream, g, z, w, c.V, k, c.partial, done);
    }
    hipLaunchKernelGGL(k_finish_dots, dim3(j + 2), dim3(kBlock), 0, c.stream, c.partial, G, j + 1, c.scal + S_H1,
                       c.scal + 2, (const Status *)c.status, (const double *)c.scal, 1);
    {
        ProfScope ps(c, MSRSB_K_ORTHO);
        const double *h1 = c.scal + S_H1;
        const Status *st = c.status;
        const double *sc = c.scal;
        if (k <= 7)
            hipLaunchKernelGGL(k_axpy_dot_r<8>, dim3(G), dim3(kBlock), 0, c.stream, c.N, c.V, k, h1, w, c.partial, st, sc);
        else if (k <= 15)
            hipLaunchKernelGGL(k_axpy_dot_r<16>, dim3(G), dim3(kBlock), 0, c.stream, c.N, c.V, k, h1, w, c.partial, st, sc);
        else if (k <= 31)
            hipLaunchKernelGGL(k_axpy_dot_r<32>, dim3(G), dim3(kBlock), 0, c.stream, c.N, c.V, k, h1, w, c.partial, st, sc);
        else
            hipLaunchKernelGGL(k_axpy_dot, dim3(G), dim3(kBlock), 0, c.stream, c.N, c.V, k, h1, w, c.partial, st, sc);
    }
    hipLaunchKernelGGL(k_finish_dots, dim3(j + 2), dim3(kBlock), 0, c.stream, c.partial, G, j + 1, c.scal + S_H2,
                       c.scal + 3, (const Status *)c.status, (const double *)c.scal, 2);
    {
        ProfScope ps(c, MSRSB_K_ORTHO);
        hipLaunchKernelGGL(k_axpy_norm, dim3(G), dim3(kBlock), 0, c.stream, c.N, c.V, j + 1, c.scal + S_H2, w,
                           c.partial, (const Status *)c.status, (const double *)c.scal);
    }
    hipLaunchKernelGGL(k_gmres_step2, dim3(1), dim3(kBlock), 0, c.stream, c.status, c.scal, c.partial, G, j, rtol,
                       max_iters, restart);
    hipLaunchKernelGGL(k_scale, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, w,
                       c.V + (long)(j + 1) * c.N, c.scal + S_INV, done);
}

// exported for the solver driver
void launch_begin_solve(Ctx &c, const double *b, double *x) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, c.stream, c.status, c.flag);
    launch_zero_inactive(c, x);
    launch_multidot(c, b, 1, b, c.scal + 1, nullptr);  // ||b||^2 (b is 0 on inactive cells)
    hipLaunchKernelGGL(k_set_bnorm, dim3(1), dim3(1), 0, c.stream, c.status, c.scal + 1);
}

void launch_gmres_begin(Ctx &c, double rtol, int max_iters) {
    hipLaunchKernelGGL(k_gmres_begin, dim3(1), dim3(1), 0, c.stream, c.status, c.scal, rtol, max_iters);
}

// ------------------------------------------------------- batched launches ----
// One launch per kernel over the members of a group; each workgroup runs the
// body above for its member with the member's own grid size and arguments,
// so the member's arithmetic and reduction order are those of its own launch.

#define BAT_LOCATE()                              \
    int m, lb, nb;                                \
    if (!bat_locate(gp, act, m, lb, nb)) return;  \
    const BMember &d = D[m]

template <typename F>
static void each_group(const Groups &gs, F f) {
    for (const HGroup &h : gs)
        if (h.g.n > 0) f(h);
}

// reduction grids of a member: G for norms and dots, GA for pass A of the
// Arnoldi step; returns whether the step sums pass A's partials itself
bool bat_member_fine(const Ctx &c, BMember &d) {
    d.G = red_grid(c.N);
    d.GA = std::min(d.G, kPassABlocks);
    return d.GA <= kDstepFuseBlocks;
}

__global__ __launch_bounds__(kBlock) void k_rhs_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    if (!d.q) return;  // this member keeps its source
    rhs_body(lb, nb, d.g.N, d.g.diag, d.bcrhs, d.q, d.b, d.src);
}

void bat_source_update(Batch &B) {
    each_group(B.cells, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_rhs_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
}

__global__ void k_reset_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    reset_body(d.status, d.flag);
}

__global__ void k_zero_inactive_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    zero_inactive_body(lb, nb, d.g.N, d.g.diag, d.x);
}

__global__ __launch_bounds__(kBlock) void k_bnorm_dot_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    multidot_body(lb, nb, d.g.N, d.b, 1, d.b, d.partial, nullptr);
}

__global__ __launch_bounds__(kBlock) void k_bnorm_finish_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    multidot_finish_body(0, 1, d.partial, d.G, d.scal + 1, nullptr);
    __syncthreads();
    if (threadIdx.x == 0) set_bnorm_body(d.status, d.scal + 1);
}

void bat_begin_solve(Batch &B) {
    for (const HGroup &h : B.one)
        hipLaunchKernelGGL(k_reset_b, dim3(h.g.total), dim3(1), 0, B.stream, B.d_mem, h.g, B.d_act);
    each_group(B.cells, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_zero_inactive_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
    each_group(B.red, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_bnorm_dot_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
    each_group(B.one, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_bnorm_finish_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
}

// restart: r = b - A x into V(0) with its norm, then the restart test
__global__ __launch_bounds__(kBlock) void k_restart_res_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    residual_body<true>(lb, nb, d.g, d.b, d.x, d.V, d.partial, nullptr);
}

__global__ __launch_bounds__(kBlock) void k_restart_begin_b(const BMember *D, BGroup gp, const int *act, double rtol,
                                                            int max_iters) {
    BAT_LOCATE();
    norm_finish_body(d.partial, d.G, d.scal, nullptr);
    __syncthreads();
    if (threadIdx.x == 0) gmres_begin_body(d.status, d.scal, rtol, max_iters);
}

void bat_restart_residual(Batch &B, double rtol, int max_iters) {
    each_group(B.red, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_restart_res_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
    each_group(B.one, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_restart_begin_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act,
                           rtol, max_iters);
    });
}

// One DCGS2 Arnoldi step for column j of every member (final: only finalise
// column j - 1), with the member's candidate u_j and preconditioned Z(j).
template <int KM, bool MV, typename VT>
__global__ __launch_bounds__(kBlock) void k_dpass_a_b(const BMember *D, BGroup gp, const int *act, int j) {
    BAT_LOCATE();
    const VT *Q = std::is_same<VT, float>::value ? (const VT *)d.Vf : (const VT *)d.V;
    dpass_a_body<KM, MV, VT>(lb, nb, d.g, MV ? bvec(d, bvsel(BV_Z, j)) : nullptr, d.tmp, Q,
                             bvec(d, bvsel(BV_U, j)), j, d.partial, &d.status->done);
}

// na workgroups per member of a one-per-member group: workgroup q of member
// k sums quantity q, as in the member's own launch of na workgroups
__global__ __launch_bounds__(kBlock) void k_finish_n_b(const BMember *D, BGroup gp, const int *act, int na) {
    const int k = blockIdx.x / na, q = blockIdx.x - k * na;
    const int m = gp.mem[k];
    if (!act[m]) return;
    const BMember &d = D[m];
    finish_n_body(q, na, d.partial, d.GA, d.scal + S_DA, d.status);
}

__global__ __launch_bounds__(kBlock) void k_dstep_b(const BMember *D, BGroup gp, const int *act, int j, double rtol,
                                                    int max_iters, int final_) {
    BAT_LOCATE();
    const bool fuse = d.GA <= kDstepFuseBlocks;
    dstep_body(d.status, d.scal, j, rtol, max_iters, final_, d.partial, fuse ? d.GA : 0);
}

template <int KM, typename VT>
__global__ __launch_bounds__(kBlock) void k_dpass_b_b(const BMember *D, BGroup gp, const int *act, int j) {
    BAT_LOCATE();
    const long N = d.g.N;
    const bool f = std::is_same<VT, float>::value;
    VT *Q = f ? (VT *)d.Vf : (VT *)d.V;
    VT *qout = Q + (long)j * N;
    double *unext = d.V + (f ? (long)((j + 1) & 1) : (long)(j + 1)) * N;
    dpass_b_body<KM, VT>(lb, nb, d.g.N, Q, bvec(d, bvsel(BV_U, j)), d.tmp, j, qout, unext, d.scal, d.status);
}

template <int KM, typename VT>
static void bat_dgmres_k(Batch &B, int j, double rtol, int max_iters, bool final_) {
    const int na = final_ ? j + 1 : 2 * j + 2;
    each_group(B.passa, [&](const HGroup &h) {
        if (final_)
            hipLaunchKernelGGL((k_dpass_a_b<KM, false, VT>), dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem,
                               h.g, B.d_act, j);
        else
            hipLaunchKernelGGL((k_dpass_a_b<KM, true, VT>), dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem,
                               h.g, B.d_act, j);
    });
    // members whose pass-A grid is too large for the step to sum its partials
    each_group(B.nofuse, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_finish_n_b, dim3(h.g.n * na), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act, na);
    });
    each_group(B.one, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_dstep_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act, j, rtol,
                           max_iters, final_ ? 1 : 0);
    });
    if (final_) return;
    each_group(B.red, [&](const HGroup &h) {
        hipLaunchKernelGGL((k_dpass_b_b<KM, VT>), dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act,
                           j);
    });
}

template <typename VT>
static void bat_dgmres_t(Batch &B, int j, double rtol, int max_iters, bool final_) {
    if (j <= 7) bat_dgmres_k<8, VT>(B, j, rtol, max_iters, final_);
    else if (j <= 15) bat_dgmres_k<16, VT>(B, j, rtol, max_iters, final_);
    else bat_dgmres_k<32, VT>(B, j, rtol, max_iters, final_);
}

void bat_dgmres_step(Batch &B, int j, double rtol, int max_iters, bool final_) {
    if (B.mixed) bat_dgmres_t<float>(B, j, rtol, max_iters, final_);
    else bat_dgmres_t<double>(B, j, rtol, max_iters, final_);
}

// x += Z (T^-1 y) over the k = jcur columns of the restart (none if k = 0)
__global__ __launch_bounds__(64) void k_solve_small_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    if (d.status->jcur <= 0) return;
    gmres_solve_small_body(d.status, d.scal, 1);
}

__global__ __launch_bounds__(kBlock) void k_update_x_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    const int k = d.status->jcur;
    if (k <= 0) return;
    multiaxpy_body<false, double>(lb, nb, d.g.N, d.Z, k, d.scal + kScalW, 1.0, d.x, d.partial, nullptr);
}

void bat_solution_update(Batch &B) {
    each_group(B.one, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_solve_small_b, dim3(h.g.total), dim3(64), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
    each_group(B.red, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_update_x_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
    });
}

// every member's status and error flag into the batch's arrays (members that
// have left keep their last copy)
__global__ void k_gather_status_b(const BMember *D, BGroup gp, const int *act, Status *out, int *flags) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    out[m] = *d.status;
    flags[m] = d.flag[0];
}

void bat_gather_status(Batch &B) {
    each_group(B.one, [&](const HGroup &h) {
        hipLaunchKernelGGL(k_gather_status_b, dim3(h.g.total), dim3(1), 0, B.stream, B.d_mem, h.g, B.d_act, B.d_st,
                           B.d_flag);
    });
}

#undef BAT_LOCATE

}  // namespace msrsb
