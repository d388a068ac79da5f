// Rectilinear-stage transfer operators: restriction d = P^T r, prolongation
// x += P p_c and the Galerkin product A_c = P^T A P (the reduced pressure
// system with R = P^T).  Basis layout as in the sweeps: slot-major P[s*N + i]
// with implicit slots (at most two consecutive blocks per axis).
#include <algorithm>

#include <hip/hip_ext.h>

#include "batch.h"
#include "cart_util.h"
#include "dev_util.h"
#include "msrsb_internal.h"
#include "stencil.h"

namespace msrsb {


// ------------------------------------------------- restriction / prolongation

// d = P^T r in two deterministic passes.
// Cells whose first support block along every axis is the same (lo = L: the
// "dual box" between block centres L and L+1) share their eight slot->block
// maps, so P_is r_i can be summed per slot over a dual box and attributed
// afterwards.
// Pass 1 (k_restrict_rows): one wavefront per (dual interval Ly along y,
// layer z) walks the rows y of that interval; lane x keeps per-slot sums for
// its own column (its dual interval along x is fixed), so rows are read
// coalesced and every P entry once.  Lanes of one dual x-interval are then
// added in lane order:  part[((z*my + Ly)*mx + Lx)*NS + s].
// Pass 2 (k_restrict_gather): d_J = sum over s, and over the layers z of the
// dual interval J_z - s_z, of part[z, J_y - s_y, J_x - s_x, s] (fixed order).
// RES: r is not read but formed per cell as b - A x, with the operations of
// the residual kernel in the same order (the compiler's fused multiply-adds
// may still round differently from a stored residual's).
// W wavefronts per workgroup, U rows per wavefront in flight.  One workgroup
// per (dual y-interval Ly, layer z), numbered with Ly fastest and spread over
// the XCDs in contiguous ranges: the workgroups in flight on an XCD read
// whole consecutive layers (one contiguous address range), and the layers
// above and below go through the same L2.  (Numbering z fastest, so that one
// XCD walked the layers of an interval, was 10 % slower on the 60x220x85
// model.)  Rows of at most 64 cells (NCH = 1) take the x neighbours from the
// adjacent lanes.
template <int NS, typename PS, int NCH, bool RES, int W, int U>
__device__ __forceinline__ void restrict_rows_body(int bid, int nblk, CartDev cd, Fine g, const PS *__restrict__ P,
                                                   const double *__restrict__ rb, const double *__restrict__ x,
                                                   double *__restrict__ part, const int *done) {
    extern __shared__ double red[];  // [W][nx][NS]
    if (done && *done) return;
    const int mx = cd.m[0], my = cd.m[1];
    const int t = xcd_block(bid, nblk);
    if (t >= my * g.nz) return;
    const int z = t / my, Ly = t - z * my;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int y0 = 0, y1 = g.ny;
    if (cd.bit[1] >= 0) {
        y0 = Ly == 0 ? 0 : cd.split[1][Ly];
        y1 = Ly + 1 < my ? cd.split[1][Ly + 1] : g.ny;
    }
    constexpr bool SHX = RES && NCH == 1;  // x neighbours by lane exchange
    double acc[NCH][NS];
#pragma unroll
    for (int k = 0; k < NCH; ++k)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[k][s] = 0.0;
    // U rows per pass, all loads of a pass issued before the first use; rows
    // past the interval load row y0 and add nothing.  Each wavefront adds its
    // rows in increasing y, so the sums do not depend on U (they do on W).
    for (int yb = y0 + wv; yb < y1; yb += W * U) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int xx = lane + 64 * k;
            if (xx < g.nx) {
                double ri[U], pv[U][NS];
                double xi[U], xl[U][6], traw[U][6], dg[U], bi[U];
                bool in[U], fin[U][6];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int y = yb + u * W;
                    in[u] = y < y1;
                    const int i = g.nx * ((in[u] ? y : y0) + g.ny * z) + xx;
#pragma unroll
                    for (int s = 0; s < NS; ++s) pv[u][s] = ld_basis(P, (long)s * g.N + i);
                    if (RES) {
                        // faces as in cell_faces, the zeroing applied after the loads
                        const int step[3] = {1, g.nx, g.nxy};
#pragma unroll
                        for (int a = SHX ? 1 : 0; a < 3; ++a) {
                            const double *Ta = a == 0 ? g.tx : (a == 1 ? g.ty : g.tz);
                            fin[u][2 * a] = i >= step[a];
                            fin[u][2 * a + 1] = i + step[a] < g.N;
                            const int ld = fin[u][2 * a] ? i - step[a] : i, lu = fin[u][2 * a + 1] ? i + step[a] : i;
                            traw[u][2 * a] = Ta[ld];
                            xl[u][2 * a] = x[ld];
                            xl[u][2 * a + 1] = x[lu];
                        }
                        traw[u][1] = g.tx[i];
                        traw[u][3] = g.ty[i];
                        traw[u][5] = g.tz[i];
                        xi[u] = x[i];
                        dg[u] = g.diag[i];
                        bi[u] = rb[i];
                    } else {
                        ri[u] = rb[i];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                if (SHX) {
                    // tx of the cell before is the previous lane's own tx (0 on
                    // the first column, where the face does not exist); the end
                    // lanes use their own x, multiplied by a zero coefficient
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double tl = __shfl_up(traw[u][1], 1, 64), xm = __shfl_up(xi[u], 1, 64);
                        const double xp = __shfl_down(xi[u], 1, 64);
                        fin[u][0] = fin[u][1] = true;
                        traw[u][0] = xx > 0 ? tl : 0.0;
                        xl[u][0] = xx > 0 ? xm : xi[u];
                        xl[u][1] = xx + 1 < g.nx ? xp : xi[u];
                    }
                }
                if (RES) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        double ax = dg[u] * xi[u];  // (A x)_i as ax_row
#pragma unroll
                        for (int q = 0; q < 6; ++q) ax -= (fin[u][q] ? traw[u][q] : 0.0) * xl[u][q];
                        ri[u] = dg[u] > 0.0 ? bi[u] - ax : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int s = 0; s < NS; ++s) acc[k][s] = in[u] ? acc[k][s] + pv[u][s] * ri[u] : acc[k][s];
            }
        }
    }
    double *mine = red + (long)wv * g.nx * NS;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        const int xx = lane + 64 * k;
        if (xx < g.nx)
#pragma unroll
            for (int s = 0; s < NS; ++s) mine[xx * NS + s] = acc[k][s];
    }
    __syncthreads();
    // thread (Lx, s) adds waves, then columns of dual x-interval Lx, in order
    for (int e = threadIdx.x; e < mx * NS; e += blockDim.x) {
        const int Lx = e / NS, s = e % NS;
        int x0 = 0, x1 = g.nx;
        if (cd.bit[0] >= 0) {
            x0 = Lx == 0 ? 0 : cd.split[0][Lx];
            x1 = Lx + 1 < mx ? cd.split[0][Lx + 1] : g.nx;
        }
        double tot = 0.0;
        for (int xx = x0; xx < x1; ++xx)
            for (int w = 0; w < W; ++w) tot += red[((long)w * g.nx + xx) * NS + s];
        part[(((long)z * my + Ly) * mx + Lx) * NS + s] = tot;
    }
}

template <int NS, typename PS, int NCH, bool RES, int W, int U>
__global__ __launch_bounds__(64 * W) void k_restrict_rows(CartDev cd, Fine g, const PS *__restrict__ P,
                                                          const double *__restrict__ rb,
                                                          const double *__restrict__ x, double *__restrict__ part,
                                                          const int *done) {
    restrict_rows_body<NS, PS, NCH, RES, W, U>(blockIdx.x, gridDim.x, cd, g, P, rb, x, part, done);
}

// NARROW: every dual z-interval has at most 64 layers, so each lane adds at
// most one layer per slot.  The z split table is staged in LDS, so the only
// global round trips are the block id and one partial per slot; the partials
// are loaded unconditionally (clamped index) and masked by a factor 0 or 1.
constexpr int kGatherSplitLds = 1024;  // dual z-intervals held in LDS

template <int NS, bool NARROW>
__device__ __forceinline__ void restrict_gather_body(int bid, int nblk, CartDev cd, Fine g, int M,
                                                     const double *__restrict__ part, double *__restrict__ d,
                                                     const int *done) {
    __shared__ int spz[kGatherSplitLds];
    if (done && *done) return;
    const int mx = cd.m[0], my = cd.m[1], mz = cd.m[2];
    for (int t = threadIdx.x; t < mz; t += blockDim.x) spz[t] = cd.split[2][t];
    const int j = bid * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int cid = cd.present[min(j, M - 1)];
    __syncthreads();
    if (j >= M) return;
    const int J[3] = {cid % mx, (cid / mx) % my, cid / (mx * my)};
    // work items: (slot s, layer z of the dual interval J_z - s_z)
    int L[NS][3], z0[NS], z1[NS];
    bool ok[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        ok[s] = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[s][a] = J[a] - (cd.bit[a] >= 0 ? (s >> cd.bit[a]) & 1 : 0);
            ok[s] = ok[s] && L[s][a] >= 0;
        }
        const int l2 = max(L[s][2], 0);
        const bool zs = cd.bit[2] >= 0 && ok[s];
        z0[s] = zs && l2 > 0 ? spz[l2] : 0;
        z1[s] = zs && l2 + 1 < mz ? spz[l2 + 1] : g.nz;
    }
    double v = 0.0;
    if (NARROW) {
        double pv[NS], f[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int z = z0[s] + lane;
            const bool in = ok[s] && z < z1[s];
            const long at = in ? (((long)z * my + L[s][1]) * mx + L[s][0]) * NS + s : 0;
            pv[s] = part[at];
            f[s] = in ? 1.0 : 0.0;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) v += pv[s] * f[s];
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (!ok[s]) continue;
            for (int z = z0[s] + lane; z < z1[s]; z += 64) v += part[(((long)z * my + L[s][1]) * mx + L[s][0]) * NS + s];
        }
    }
    v = wave_sum(v);
    if (lane == 0) d[j] = v;
}

template <int NS, bool NARROW>
__global__ __launch_bounds__(256) void k_restrict_gather(CartDev cd, Fine g, int M, const double *__restrict__ part,
                                                         double *__restrict__ d, const int *done) {
    restrict_gather_body<NS, NARROW>(blockIdx.x, gridDim.x, cd, g, M, part, d, done);
}

// x_i += sum_s P_is p_c[block(i, s)], one wavefront per grid row (y, z) with
// lanes along x.  The y and z parts of the slot -> block map are uniform over
// the row, and p_c is held per Cartesian block (zero on dropped blocks), so
// the block of a slot is index arithmetic on the packed per-axis tables.
// Inactive cells and slots outside the support hold zero basis values (the
// sweeps store zeros there) and add nothing.  The skip flag is read after the
// data loads are issued, so it costs no separate round trip.
constexpr int kProWaves = 4;

template <int NS, typename PS, int NCH>
__device__ __forceinline__ void prolong_rows_body(int bid, int nblk, CartDev cd, Fine g, const PS *__restrict__ P,
                                                  const double *__restrict__ pcc, double *__restrict__ x,
                                                  const int *done) {
    const int row = xcd_block(bid, nblk) * kProWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (row >= g.ny * g.nz) return;
    const int lane = threadIdx.x & 63;
    const int z = row / g.ny, y = row - z * g.ny;
    const int wy = cd.bit[1] >= 0 ? cd.pack[1][y] : 0;
    const int wz = cd.bit[2] >= 0 ? cd.pack[2][z] : 0;
    const int mx = cd.m[0], mxy = cd.m[0] * cd.m[1];
    const int byz = mx * (wy & 0xFFFFF) + mxy * (wz & 0xFFFFF);
    const int ny2 = (wy >> 20) & 1, nz2 = (wz >> 20) & 1;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        const int xx = lane + 64 * k;
        if (xx >= g.nx) continue;
        const long i = (long)row * g.nx + xx;
        // the table load first: the gathers wait for it, not for the basis
        const int wx = cd.bit[0] >= 0 ? cd.pack[0][xx] : 0;
        double pv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) pv[s] = ld_basis(P, (long)s * g.N + i);
        const double xo = x[i];
        if (done && *done) return;
        const int b0 = byz + (wx & 0xFFFFF), nx2 = (wx >> 20) & 1;
        // every gather issued (clamped index) before the first use, and the
        // slot mask applied to the basis value: no branch per slot
        double pcv[NS];
        bool ok[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int sx = cd.bit[0] >= 0 ? (s >> cd.bit[0]) & 1 : 0;
            const int sy = cd.bit[1] >= 0 ? (s >> cd.bit[1]) & 1 : 0;
            const int sz = cd.bit[2] >= 0 ? (s >> cd.bit[2]) & 1 : 0;
            ok[s] = sx <= nx2 && sy <= ny2 && sz <= nz2;
            pcv[s] = pcc[ok[s] ? b0 + sx + mx * sy + mxy * sz : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) acc += (ok[s] ? pv[s] : 0.0) * pcv[s];
        x[i] = xo + acc;
    }
}

template <int NS, typename PS, int NCH>
__global__ __launch_bounds__(64 * kProWaves) void k_prolong_rows(CartDev cd, Fine g, const PS *__restrict__ P,
                                                                 const double *__restrict__ pcc,
                                                                 double *__restrict__ x, const int *done) {
    prolong_rows_body<NS, PS, NCH>(blockIdx.x, gridDim.x, cd, g, P, pcc, x, done);
}

// four wavefronts with one row each in flight measured fastest on the
// 60x220x85 model (25.6 and 28.0 us on its two stages, against 26.5 and
// 28.8 us with two rows each: fewer registers, more wavefronts resident);
// 8x1 won on one stage and lost on the other, and 2x1, 2x2, 4x3, 4x4, 8x2,
// 8x3, 16x1 and 16x2 were slower
constexpr int kRestrictWaves = 4, kRestrictUnroll = 1;

template <typename PS, bool RES>
static void restrict_dispatch(Ctx &c, Stage &s, const PS *P, const double *rb, const double *x, const int *done) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const int nch = cdiv(c.nx, 64);
    constexpr int W = kRestrictWaves;
    const dim3 grid(xcd_grid(s.cart.m[1] * c.nz)), blk(64 * W), fgrid(cdiv(s.M, 4)), fblk(256);
    const size_t lds = sizeof(double) * W * (size_t)c.nx * s.ns;
    hipEvent_t e0, e1;  // the pass over the fine grid alone, timed by its dispatch when profiled
    prof_pair(c, MSRSB_K_RESTRICT_ROWS, &e0, &e1);
#define MSRSB_RR(NS, NCH, W_, U_) \
    hipExtLaunchKernelGGL((k_restrict_rows<NS, PS, NCH, RES, W_, U_>), grid, blk, lds, c.stream, e0, e1, 0, s.cart, g, P, rb, x, s.rpart, done)
#define MSRSB_RNS(NS)                                                                                        \
    {                                                                                                        \
        if (nch == 1) MSRSB_RR(NS, 1, W, kRestrictUnroll);                                                   \
        else if (nch == 2) MSRSB_RR(NS, 2, W, kRestrictUnroll);                                              \
        else MSRSB_RR(NS, 4, W, kRestrictUnroll);                                                            \
        if (s.zwide <= 64)                                                                                   \
            hipLaunchKernelGGL((k_restrict_gather<NS, true>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done); \
        else                                                                                                 \
            hipLaunchKernelGGL((k_restrict_gather<NS, false>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done); \
    }
    switch (s.ns) {
    case 1: MSRSB_RNS(1) break;
    case 2: MSRSB_RNS(2) break;
    case 4: MSRSB_RNS(4) break;
    default: MSRSB_RNS(8) break;
    }
#undef MSRSB_RNS
#undef MSRSB_RR
}

template <typename PS>
static void prolong_dispatch(Ctx &c, Stage &s, const PS *P, double *x, const int *done) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const dim3 grid(xcd_grid(cdiv(c.ny * c.nz, kProWaves))), blk(64 * kProWaves);
    const int nch = cdiv(c.nx, 64);
#define MSRSB_PROWS(NS, NCH) \
    hipLaunchKernelGGL((k_prolong_rows<NS, PS, NCH>), grid, blk, 0, c.stream, s.cart, g, P, s.pc, x, done)
#define MSRSB_PNS(NS)                         \
    {                                         \
        if (nch == 1) MSRSB_PROWS(NS, 1);     \
        else if (nch == 2) MSRSB_PROWS(NS, 2); \
        else MSRSB_PROWS(NS, 4);              \
    }
    switch (s.ns) {
    case 1: MSRSB_PNS(1) break;
    case 2: MSRSB_PNS(2) break;
    case 4: MSRSB_PNS(4) break;
    default: MSRSB_PNS(8) break;
    }
#undef MSRSB_PNS
#undef MSRSB_PROWS
}

void launch_restrict(Ctx &c, Stage &s, const double *r, const int *done) {
    ProfScope ps(c, MSRSB_K_RESTRICT);
    if (s.kind == 2) {
        launch_xrestrict(c, s, r, done);
        return;
    }
    if (c.opt.precision == MSRSB_MIXED) restrict_dispatch<uint16_t, false>(c, s, s.Pbf, r, nullptr, done);
    else restrict_dispatch<double, false>(c, s, s.P64[s.cur], r, nullptr, done);
}

// d = P^T (b - A x) without storing the residual (rectilinear stages).
void launch_residual_restrict(Ctx &c, Stage &s, const double *b, const double *x, const int *done) {
    ProfScope ps(c, MSRSB_K_RESTRICT);
    if (c.opt.precision == MSRSB_MIXED) restrict_dispatch<uint16_t, true>(c, s, s.Pbf, b, x, done);
    else restrict_dispatch<double, true>(c, s, s.P64[s.cur], b, x, done);
}

void launch_prolong(Ctx &c, Stage &s, double *x, const int *done) {
    ProfScope ps(c, MSRSB_K_PROLONG);
    if (s.kind == 2) {
        launch_xprolong(c, s, x, done);
        return;
    }
    if (c.opt.precision == MSRSB_MIXED) prolong_dispatch<uint16_t>(c, s, s.Pbf, x, done);
    else prolong_dispatch<double>(c, s, s.P64[s.cur], x, done);
}

// ------------------------------------------------------------ Galerkin ----
// A_c = P^T A P with A = D - T (D the diagonal including boundary terms, T
// the face transmissibilities), summed per dual box: the cells L whose first
// support block is L along every axis share the slot -> block map
// block(s) = L + bits(s).  With P_i the slot vector of cell i,
//   A_c = sum_L [ S_L  on blocks (L+s, L+t) ]
//       + sum_L sum_a [ X_La on (L+s, L+e_a+t) and its transpose ],
//   S_L   = sum_{i in L} P_i Q_i^T,  Q_i = D_i P_i - sum_{l ~ i, l in L} T_il P_l,
//   X_La  = - sum_{i in L, l = i + e_a in L + e_a} T_il P_i P_l^T.
// S_L is symmetric; only its upper triangle is formed.  Pass 1
// (k_rap_box) reads the basis once, one workgroup per dual box, and reduces
// each quantity over the workgroup in a fixed order; pass 2 (k_rap_gather)
// adds the contributions of every coarse entry in a fixed order, one thread
// per entry (j, k) with k >= j, which writes both (j, k) and (k, j).
constexpr int kRapThreads = 256;

template <int NS>
struct RapLayout {
    static constexpr int nsym = NS * (NS + 1) / 2;
    static constexpr int spad = nsym <= 1 ? 1 : (nsym <= 4 ? 4 : (nsym <= 16 ? 16 : 64));
    static constexpr int stride = spad + 3 * NS * NS;  // [S][X_x][X_y][X_z]
    __host__ __device__ static constexpr int sym(int s, int t) { return s * NS - s * (s - 1) / 2 + (t - s); }
};

__device__ inline void box_range(const CartDev &cd, int a, int L, int &lo, int &hi) {
    if (cd.bit[a] < 0) {
        lo = 0;
        hi = cd.n[a];
        return;
    }
    lo = L == 0 ? 0 : cd.split[a][L];
    hi = L + 1 < cd.m[a] ? cd.split[a][L + 1] : cd.n[a];
}

template <int AM, typename PS>
__device__ __forceinline__ void rap_box_body(int bid, int nblk, CartDev cd, Fine g, const PS *__restrict__ P,
                                             double *__restrict__ part, int nbox) {
    constexpr int NS = 1 << __builtin_popcount(AM);
    using Lay = RapLayout<NS>;
    __shared__ double red[(kRapThreads / 64) * 64];
    const int box = xcd_block(bid, nblk);
    if (box >= nbox) return;
    const int Lc[3] = {box % cd.m[0], (box / cd.m[0]) % cd.m[1], box / (cd.m[0] * cd.m[1])};
    int lo[3], hi[3], ext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        box_range(cd, a, Lc[a], lo[a], hi[a]);
        ext[a] = hi[a] - lo[a];
    }
    const int N = g.N;
    const int step[3] = {1, g.nx, g.nxy};
    double *out = part + (long)box * Lay::stride;

    // S_L: upper triangle of sum_i P_i Q_i^T
    {
        double acc[Lay::spad];
#pragma unroll
        for (int q = 0; q < Lay::spad; ++q) acc[q] = 0.0;
        const int vol = ext[0] * ext[1] * ext[2];
        for (int t = threadIdx.x; t < vol; t += blockDim.x) {
            const int c[3] = {lo[0] + t % ext[0], lo[1] + (t / ext[0]) % ext[1], lo[2] + t / (ext[0] * ext[1])};
            const int i = c[0] + g.nx * (c[1] + g.ny * c[2]);
            const double d = g.diag[i];
            double p[NS], nb[6][NS], T[6];
            bool in[6];
            int l[6];
#pragma unroll
            for (int s = 0; s < NS; ++s) p[s] = ld_basis(P, (long)s * N + i);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double *Ta = a == 0 ? g.tx : (a == 1 ? g.ty : g.tz);
                in[2 * a] = c[a] - 1 >= lo[a];
                in[2 * a + 1] = c[a] + 1 < hi[a];
                l[2 * a] = in[2 * a] ? i - step[a] : i;
                l[2 * a + 1] = in[2 * a + 1] ? i + step[a] : i;
                const double td = Ta[l[2 * a]], tu = Ta[i];
                T[2 * a] = in[2 * a] ? td : 0.0;
                T[2 * a + 1] = in[2 * a + 1] ? tu : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int s = 0; s < NS; ++s) nb[q][s] = ld_basis(P, (long)s * N + l[q]);
            double Q[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                double v = d * p[s];
#pragma unroll
                for (int q = 0; q < 6; ++q) v -= T[q] * nb[q][s];
                Q[s] = v;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int u = s; u < NS; ++u) acc[Lay::sym(s, u)] += p[s] * Q[u];
        }
        group_sum_store<Lay::spad>(acc, Lay::spad, red, out);
    }
    // X_La over the faces leaving the box along +a
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!((AM >> a) & 1)) continue;
        double acc[NS * NS];
#pragma unroll
        for (int q = 0; q < NS * NS; ++q) acc[q] = 0.0;
        const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        const bool has_next = hi[a] < cd.n[a];
        const int cnt = has_next ? ext[b1] * ext[b2] : 0;
        const double *Ta = a == 0 ? g.tx : (a == 1 ? g.ty : g.tz);
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            int c[3];
            c[a] = hi[a] - 1;
            c[b1] = lo[b1] + t % ext[b1];
            c[b2] = lo[b2] + t / ext[b1];
            const int i = c[0] + g.nx * (c[1] + g.ny * c[2]);
            const int l = i + step[a];
            const double T = Ta[i];
            double p[NS], q[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                p[s] = ld_basis(P, (long)s * N + i);
                q[s] = ld_basis(P, (long)s * N + l);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const double tp = -T * p[s];
#pragma unroll
                for (int u = 0; u < NS; ++u) acc[s * NS + u] += tp * q[u];
            }
        }
        group_sum_store<NS * NS>(acc, NS * NS, red, out + Lay::spad + a * NS * NS);
    }
}

template <int AM, typename PS>
__global__ __launch_bounds__(kRapThreads) void k_rap_box(CartDev cd, Fine g, const PS *__restrict__ P,
                                                         double *__restrict__ part, int nbox) {
    rap_box_body<AM, PS>(blockIdx.x, gridDim.x, cd, g, P, part, nbox);
}

template <int AM>
__device__ __forceinline__ void rap_gather_body(int bid, int nblk, CartDev cd, const double *__restrict__ part,
                                                double *__restrict__ Ac, int M, int Mp) {
    constexpr int NS = 1 << __builtin_popcount(AM);
    constexpr int NB = __builtin_popcount(AM);
    constexpr int NOFF = NB == 0 ? 1 : (NB == 1 ? 5 : (NB == 2 ? 25 : 125));
    using Lay = RapLayout<NS>;
    const int j = bid, o = threadIdx.x;
    if (j >= M || o >= NOFF) return;
    const int m[3] = {cd.m[0], cd.m[1], cd.m[2]};
    const int cid = cd.present[j];
    const int J[3] = {cid % m[0], (cid / m[0]) % m[1], cid / (m[0] * m[1])};
    int K[3];
    {
        int rem = o;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if ((AM >> a) & 1) {
                K[a] = J[a] + rem % 5 - 2;
                rem /= 5;
            } else {
                K[a] = 0;
            }
            if (K[a] < 0 || K[a] >= m[a]) return;
        }
    }
    const int kc = cd.cmap[K[0] + m[0] * (K[1] + m[1] * K[2])];
    if (kc < j) return;  // dropped block, or the entry of the row kc
    auto bitoff = [](int s, int a) { return ((AM >> a) & 1) ? (s >> __builtin_popcount(AM & ((1 << a) - 1))) & 1 : 0; };
    auto slot_of = [](const int u[3]) {
        int s = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if ((AM >> a) & 1) s |= u[a] << __builtin_popcount(AM & ((1 << a) - 1));
        return s;
    };
    double sum = 0.0;
    // S terms: L = J - off(s), K - L in {0,1}^3
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int L[3], u[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[a] = J[a] - bitoff(s, a);
            u[a] = K[a] - L[a];
            if (L[a] < 0 || u[a] < 0 || u[a] > 1) ok = false;
        }
        if (!ok) continue;
        const int t = slot_of(u);
        const long bx = L[0] + (long)m[0] * (L[1] + (long)m[1] * L[2]);
        sum += part[bx * Lay::stride + (s <= t ? Lay::sym(s, t) : Lay::sym(t, s))];
    }
    // X terms: (L + off(s), L + e_a + off(t)) and the transposed position
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!((AM >> a) & 1)) continue;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int *R = side == 0 ? J : K;  // holds L + off(s)
                const int *C = side == 0 ? K : J;  // holds L + e_a + off(t)
                int L[3], u[3];
                bool ok = true;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    L[b] = R[b] - bitoff(s, b);
                    u[b] = C[b] - L[b] - (b == a ? 1 : 0);
                    if (L[b] < 0 || u[b] < 0 || u[b] > 1) ok = false;
                }
                if (!ok || L[a] + 1 >= m[a]) continue;
                const int t = slot_of(u);
                const long bx = L[0] + (long)m[0] * (L[1] + (long)m[1] * L[2]);
                sum += part[bx * Lay::stride + Lay::spad + a * NS * NS + s * NS + t];
            }
        }
    }
    Ac[(long)j * Mp + kc] = sum;
    Ac[(long)kc * Mp + j] = sum;
}

template <int AM>
__global__ __launch_bounds__(128) void k_rap_gather(CartDev cd, const double *__restrict__ part,
                                                    double *__restrict__ Ac, int M, int Mp) {
    rap_gather_body<AM>(blockIdx.x, gridDim.x, cd, part, Ac, M, Mp);
}

__device__ __forceinline__ void pad_identity_body(int bid, int nblk, double *A, int M, int Mp) {
    const int k = M + bid * blockDim.x + threadIdx.x;
    if (k < Mp) A[(long)k * Mp + k] = 1.0;
}

__global__ void k_pad_identity(double *A, int M, int Mp) {
    pad_identity_body(blockIdx.x, gridDim.x, A, M, Mp);
}

// A := (A + A^T)/2 on the leading M x M part (rows are built independently).
__global__ void k_symmetrize(double *A, int M, int Mp) {
    const int i = blockIdx.y * 16 + threadIdx.y;
    const int j = blockIdx.x * 16 + threadIdx.x;
    if (i >= M || j >= M || j <= i) return;
    const double v = 0.5 * (A[(long)i * Mp + j] + A[(long)j * Mp + i]);
    A[(long)i * Mp + j] = v;
    A[(long)j * Mp + i] = v;
}

void launch_pad_identity(Ctx &c, double *A, int M, int Mp) {
    if (Mp > M) hipLaunchKernelGGL(k_pad_identity, dim3(cdiv(Mp - M, 64)), dim3(64), 0, c.stream, A, M, Mp);
}

void launch_symmetrize(Ctx &c, double *A, int M, int Mp) {
    hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(M, 16), cdiv(M, 16)), dim3(16, 16), 0, c.stream, A, M, Mp);
    if (Mp > M) hipLaunchKernelGGL(k_pad_identity, dim3(cdiv(Mp - M, 64)), dim3(64), 0, c.stream, A, M, Mp);
}

template <typename PS>
static void rap_dispatch(Ctx &c, Stage &s, const PS *P) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const CartDev &cd = s.cart;
    const int nbox = cd.m[0] * cd.m[1] * cd.m[2];
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (cd.bit[a] >= 0) am |= 1 << a;
    const dim3 grid(xcd_grid(nbox)), blk(kRapThreads), ggrid(s.M), gblk(128);
#define MSRSB_RAP(AM)                                                                                           \
    case AM:                                                                                                    \
        hipLaunchKernelGGL((k_rap_box<AM, PS>), grid, blk, 0, c.stream, cd, g, P, s.rap_part, nbox);           \
        hipLaunchKernelGGL((k_rap_gather<AM>), ggrid, gblk, 0, c.stream, cd, s.rap_part, s.Ac, s.M, s.Mp);    \
        break;
    switch (am) {
        MSRSB_RAP(0) MSRSB_RAP(1) MSRSB_RAP(2) MSRSB_RAP(3)
        MSRSB_RAP(4) MSRSB_RAP(5) MSRSB_RAP(6) MSRSB_RAP(7)
    }
#undef MSRSB_RAP
    if (s.Mp > s.M)
        hipLaunchKernelGGL(k_pad_identity, dim3(cdiv(s.Mp - s.M, 64)), dim3(64), 0, c.stream, s.Ac, s.M, s.Mp);
}

size_t rap_part_doubles(int ns, int nbox) {
    switch (ns) {
    case 1: return (size_t)RapLayout<1>::stride * nbox;
    case 2: return (size_t)RapLayout<2>::stride * nbox;
    case 4: return (size_t)RapLayout<4>::stride * nbox;
    default: return (size_t)RapLayout<8>::stride * nbox;
    }
}

void launch_rap(Ctx &c, Stage &s) {
    ProfScope ps(c, MSRSB_K_RAP);
    if (s.kind == 2) {
        launch_xrap(c, s);
        return;
    }
    hipMemsetAsync(s.Ac, 0, sizeof(double) * (size_t)s.Mp * s.Mp, c.stream);
    if (c.opt.precision == MSRSB_MIXED) rap_dispatch<uint16_t>(c, s, s.Pbf);
    else rap_dispatch<double>(c, s, s.P64[s.cur]);
}

__global__ void k_export_vals(long n, const uint16_t *__restrict__ in, double *__restrict__ out) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = (double)bf16_to_float(in[k]);
}

// Current basis values of a rectilinear stage as FP64 (device buffer).
// Widen n BF16 basis values to FP64 (d_in and d_out on the context's device).
void launch_export_bf16(Ctx &c, const uint16_t *d_in, long n, double *d_out) {
    hipLaunchKernelGGL(k_export_vals, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, d_in, d_out);
}

void launch_export_cart(Ctx &c, Stage &s, double *d_vals) {
    const long n = (long)s.ns * c.N;
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_export_vals, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, s.Pbf, d_vals);
    else
        hipMemcpyAsync(d_vals, s.P64[s.cur], sizeof(double) * n, hipMemcpyDeviceToDevice, c.stream);
}

// ------------------------------------------------------- batched launches ----
// Residual restriction and prolongation of every member's rectilinear stage,
// one launch per template key (slots per cell, 64-cell chunks per row).

// grids and template keys of a member's transfers: [0] residual restriction
// rows (key NS * 8 + NCH), [1] gather (key NS * 2 + narrow), [2] prolongation
// (key NS * 8 + NCH); lds = the restriction's dynamic LDS
void bat_member_transfer(const Ctx &c, const Stage &s, int grid[3], int key[3], size_t *lds) {
    const int nch = cdiv(c.nx, 64), nchk = nch == 1 ? 1 : (nch == 2 ? 2 : 4);
    const int ns = s.ns <= 1 ? 1 : (s.ns <= 2 ? 2 : (s.ns <= 4 ? 4 : 8));
    grid[0] = xcd_grid(s.cart.m[1] * c.nz);
    key[0] = ns * 8 + nchk;
    grid[1] = cdiv(s.M, 4);
    key[1] = ns * 2 + (s.zwide <= 64 ? 1 : 0);
    grid[2] = xcd_grid(cdiv(c.ny * c.nz, kProWaves));
    key[2] = ns * 8 + nchk;
    *lds = sizeof(double) * kRestrictWaves * (size_t)c.nx * s.ns;
}

#define BAT_LOCATE()                              \
    int m, lb, nb;                                \
    if (!bat_locate(gp, act, m, lb, nb)) return;  \
    const BMember &d = D[m]

template <int NS, typename PS, int NCH>
__global__ __launch_bounds__(64 * kRestrictWaves) void k_restrict_rows_b(const BMember *D, BGroup gp, const int *act,
                                                                         int bsel, int xsel) {
    BAT_LOCATE();
    restrict_rows_body<NS, PS, NCH, true, kRestrictWaves, kRestrictUnroll>(
        lb, nb, d.cd, d.g, (const PS *)d.Pt, bvec(d, bsel), bvec(d, xsel), d.rpart, &d.status->done);
}

template <int NS, bool NARROW>
__global__ __launch_bounds__(256) void k_restrict_gather_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    restrict_gather_body<NS, NARROW>(lb, nb, d.cd, d.g, d.M, d.rpart, d.dvec, &d.status->done);
}

template <int NS, typename PS, int NCH>
__global__ __launch_bounds__(64 * kProWaves) void k_prolong_rows_b(const BMember *D, BGroup gp, const int *act,
                                                                   int xsel) {
    BAT_LOCATE();
    prolong_rows_body<NS, PS, NCH>(lb, nb, d.cd, d.g, (const PS *)d.Pt, d.pc, bvec(d, xsel), &d.status->done);
}

#undef BAT_LOCATE

template <typename PS>
static void bat_rrows_t(Batch &B, const HGroup &h, int bsel, int xsel) {
    const dim3 grid(h.g.total), blk(64 * kRestrictWaves);
#define MSRSB_BRR(NS, NCH)                                                                                        \
    case NS * 8 + NCH:                                                                                            \
        hipLaunchKernelGGL((k_restrict_rows_b<NS, PS, NCH>), grid, blk, h.lds, B.stream, B.d_mem, h.g, B.d_act,   \
                           bsel, xsel);                                                                           \
        break
    switch (h.key) {
        MSRSB_BRR(1, 1); MSRSB_BRR(1, 2); MSRSB_BRR(1, 4);
        MSRSB_BRR(2, 1); MSRSB_BRR(2, 2); MSRSB_BRR(2, 4);
        MSRSB_BRR(4, 1); MSRSB_BRR(4, 2); MSRSB_BRR(4, 4);
        MSRSB_BRR(8, 1); MSRSB_BRR(8, 2); MSRSB_BRR(8, 4);
    default: break;
    }
#undef MSRSB_BRR
}

template <typename PS>
static void bat_prolong_t(Batch &B, const HGroup &h, int xsel) {
    const dim3 grid(h.g.total), blk(64 * kProWaves);
#define MSRSB_BPR(NS, NCH)                                                                                        \
    case NS * 8 + NCH:                                                                                            \
        hipLaunchKernelGGL((k_prolong_rows_b<NS, PS, NCH>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act, xsel); \
        break
    switch (h.key) {
        MSRSB_BPR(1, 1); MSRSB_BPR(1, 2); MSRSB_BPR(1, 4);
        MSRSB_BPR(2, 1); MSRSB_BPR(2, 2); MSRSB_BPR(2, 4);
        MSRSB_BPR(4, 1); MSRSB_BPR(4, 2); MSRSB_BPR(4, 4);
        MSRSB_BPR(8, 1); MSRSB_BPR(8, 2); MSRSB_BPR(8, 4);
    default: break;
    }
#undef MSRSB_BPR
}

// d = P^T (b - A x) for every member (b, x: the selected vectors)
void bat_residual_restrict(Batch &B, int bsel, int xsel) {
    for (const HGroup &h : B.rrows) {
        if (h.g.n == 0) continue;
        if (B.mixed) bat_rrows_t<uint16_t>(B, h, bsel, xsel);
        else bat_rrows_t<double>(B, h, bsel, xsel);
    }
    for (const HGroup &h : B.gather) {
        if (h.g.n == 0) continue;
        const dim3 grid(h.g.total), blk(256);
#define MSRSB_BG(NS, NW)                                                                                          \
    case NS * 2 + NW:                                                                                             \
        hipLaunchKernelGGL((k_restrict_gather_b<NS, NW != 0>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act);   \
        break
        switch (h.key) {
            MSRSB_BG(1, 0); MSRSB_BG(1, 1); MSRSB_BG(2, 0); MSRSB_BG(2, 1);
            MSRSB_BG(4, 0); MSRSB_BG(4, 1); MSRSB_BG(8, 0); MSRSB_BG(8, 1);
        default: break;
        }
#undef MSRSB_BG
    }
}

// x += P p_c for every member (x: the selected vector)
void bat_prolong(Batch &B, int xsel) {
    for (const HGroup &h : B.prolong) {
        if (h.g.n == 0) continue;
        if (B.mixed) bat_prolong_t<uint16_t>(B, h, xsel);
        else bat_prolong_t<double>(B, h, xsel);
    }
}

// Galerkin operators of every member: the box pass and the gather per
// split-axis mask, then the identity on the padding rows.
void bat_member_rap(const Stage &s, int grid[3], int *key) {
    const CartDev &cd = s.cart;
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (cd.bit[a] >= 0) am |= 1 << a;
    grid[0] = xcd_grid(cd.m[0] * cd.m[1] * cd.m[2]);
    grid[1] = s.M;
    grid[2] = s.Mp > s.M ? cdiv(s.Mp - s.M, 64) : 0;
    *key = am;
}

template <int AM, typename PS>
__global__ __launch_bounds__(kRapThreads) void k_rap_box_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    rap_box_body<AM, PS>(lb, nb, d.cd, d.g, (const PS *)d.Pt, d.rap_part, d.cd.m[0] * d.cd.m[1] * d.cd.m[2]);
}

template <int AM>
__global__ __launch_bounds__(128) void k_rap_gather_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    rap_gather_body<AM>(lb, nb, d.cd, d.rap_part, d.Ac, d.M, d.Mp);
}

__global__ void k_pad_identity_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    pad_identity_body(lb, nb, d.Ac, d.M, d.Mp);
}

// A_c = 0 before the gather adds its entries (grid: the coarse copy's,
// 2048 entries per workgroup)
__global__ __launch_bounds__(256) void k_zero_ac_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    const long n = (long)d.Mp * d.Mp, e0 = (long)lb * 2048 + threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const long e = e0 + (long)q * 256;
        if (e < n) d.Ac[e] = 0.0;
    }
}

template <typename PS>
static void bat_rap_t(Batch &B) {
    for (const HGroup &h : B.gjcopy)
        hipLaunchKernelGGL(k_zero_ac_b, dim3(h.g.total), dim3(256), 0, B.stream, B.d_mem, h.g, B.d_act);
    for (const HGroup &h : B.rapbox) {
#define MSRSB_BRB(AM)                                                                                           \
    case AM:                                                                                                    \
        hipLaunchKernelGGL((k_rap_box_b<AM, PS>), dim3(h.g.total), dim3(kRapThreads), 0, B.stream, B.d_mem, h.g, \
                           B.d_act);                                                                            \
        break
        switch (h.key) {
            MSRSB_BRB(0); MSRSB_BRB(1); MSRSB_BRB(2); MSRSB_BRB(3);
            MSRSB_BRB(4); MSRSB_BRB(5); MSRSB_BRB(6); MSRSB_BRB(7);
        default: break;
        }
#undef MSRSB_BRB
    }
    for (const HGroup &h : B.rapgather) {
#define MSRSB_BRG(AM)                                                                                           \
    case AM:                                                                                                    \
        hipLaunchKernelGGL((k_rap_gather_b<AM>), dim3(h.g.total), dim3(128), 0, B.stream, B.d_mem, h.g, B.d_act); \
        break
        switch (h.key) {
            MSRSB_BRG(0); MSRSB_BRG(1); MSRSB_BRG(2); MSRSB_BRG(3);
            MSRSB_BRG(4); MSRSB_BRG(5); MSRSB_BRG(6); MSRSB_BRG(7);
        default: break;
        }
#undef MSRSB_BRG
    }
    for (const HGroup &h : B.pad)
        hipLaunchKernelGGL(k_pad_identity_b, dim3(h.g.total), dim3(64), 0, B.stream, B.d_mem, h.g, B.d_act);
}

void bat_rap(Batch &B) {
    if (B.mixed) bat_rap_t<uint16_t>(B);
    else bat_rap_t<double>(B);
}

}  // namespace msrsb
