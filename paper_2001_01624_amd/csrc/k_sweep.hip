// Rectilinear-stage basis kernels: restricted-smoothing sweeps (MsRSB) with
// the device-side stop rule.
//
// Basis layout: slot-major, P[s*N + i].  A cell lies in the supports of at
// most two consecutive blocks per axis (lo[i] and lo[i]+1), so its slots are
// implicit: slot s picks, for every axis d with more than one block, block
// lo_d + bit_d(s).  No block indices are stored; a slot that is not in the
// support (beyond nv, an inactive cell, a dropped block) holds exactly 0.
#include <algorithm>

#include <hip/hip_ext.h>

#include "batch.h"
#include "cart_util.h"
#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

// ---------------------------------------------------------------- sweeps ----

template <int NS, typename PT>
__device__ __forceinline__ void basis_init_body(int bid, int nblk, CartDev cd, Fine g, PT *__restrict__ P) {
    const int i = bid * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    int s0 = -1;
    if (g.diag[i] > 0.0) {
        int c[3];
        cell_coords(g, i, c);
        s0 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (cd.bit[a] >= 0) {
                const int J = (int)(((long)c[a] * cd.m[a]) / cd.n[a]);
                s0 |= (J - cd.lo[a][c[a]]) << cd.bit[a];
            }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) P[(long)s * g.N + i] = (s == s0) ? (PT)1 : (PT)0;
}

template <int NS, typename PT>
__global__ void k_basis_init(CartDev cd, Fine g, PT *__restrict__ P) {
    basis_init_body<NS, PT>(blockIdx.x, gridDim.x, cd, g, P);
}

// One restricted-smoothing sweep for every cell:
//   P' = P - omega D_b^{-1} A_b P  on the support slots (others stay 0),
//   P  = P' / rowsum(P'),
// with A_b the zero-row-sum part of A (face transmissibilities only, so
// (A_b P)_is = sum_l T_il (P_is - P_l,s)) and D_b its diagonal.  The largest
// entry change of the workgroup goes to part[workgroup].
//
// AM is the mask of split axes (m_d > 1); axis d owns slot bit
// popcount(AM & ((1 << d) - 1)).  Neighbour l of cell i along a split axis
// holds block lo_i + b (slot bit b) in its slot bit b + (lo_i - lo_l), where
// lo_i - lo_l is 0 or +-1; a shifted bit outside {0,1} means the block is not
// in l's support (value 0).  So the values cell i needs from l are l's own
// NS slots, permuted (bit flipped where lo differs) and masked.
//
// Work layout (z march): a wavefront owns a run of 64 cells along x at one
// row y and walks the layers z0..z1-1 of its chunk.  It keeps the slots of
// layers z-1, z, z+1 of its run in registers (the z neighbours), takes the
// x neighbours from the adjacent lanes, and the rows y-1 and y+1 from the
// neighbouring wavefronts of its workgroup through LDS (the first and last
// row of the workgroup load the row beyond from memory, with the uniform
// slot permutation in the scalar load offsets).  Loads go through buffer
// resources with the slot offset in a scalar register.  Faces outside the
// grid have T = 0 and their loads are clamped to the cell.
// Faces are added in the order -x, +x, -y, +y, -z, +z.
template <int AM>
__device__ constexpr int am_bit(int a) {
    return __builtin_popcount(AM & ((1 << a) - 1));
}


typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer access: the byte offset is voff + soff; the resource's range
// check applies to voff alone, so voff must be a valid non-negative offset.
template <typename PT>
__device__ inline PT bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(PT) == 8)
        return __builtin_bit_cast(PT, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(PT, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <typename PT>
__device__ inline void bstore(PT v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(PT) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *p, long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// Rows (wavefronts) per workgroup: the first and last row also load the row
// beyond, so more rows mean fewer repeated loads but more LDS and registers
// per workgroup.  Measured on the 60x220x85 model: FP32 is fastest with 8
// rows, FP64 (two wavefronts per SIMD either way) with 4.
template <typename PT>
constexpr int sweep_rows() {
    return sizeof(PT) == 8 ? 4 : 8;
}

template <int AM, typename PT, int kSweepRows>
__device__ __forceinline__ void sweep_body(int bid, int ngrid, CartDev cd, Fine g, const PT *__restrict__ tx,
                                           const PT *__restrict__ ty, const PT *__restrict__ tz,
                                           const PT *__restrict__ Pin, PT *__restrict__ Pout, PT omega,
                                           double *__restrict__ part, int *flag, int check_blocks, const int *done,
                                           int nxt, int ngy, int nzc, int zc, int nblk,
                                           const unsigned long long *__restrict__ xmask, const int *__restrict__ packy,
                                           const int *__restrict__ packz) {
    constexpr int NS = 1 << __builtin_popcount(AM);
    constexpr int SZ = sizeof(PT);
    __shared__ double lds[kSweepRows];
    const int b = xcd_block(bid, ngrid);
    if (b >= nblk) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = g.nxy, N = g.N;
    const int NSZ = N * SZ;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // block id: z chunk fastest, then row group, then x tile
    const int zk = b % nzc, r2 = b / nzc;
    const int yg = r2 % ngy, xt = r2 / ngy;
    const int y = yg * kSweepRows + wv;
    const bool row_ok = y < ny;
    const int yc = min(y, ny - 1);
    const int x = xt * 64 + lane;
    const bool own = row_ok && x < nx;
    const int xc = min(x, nx - 1);
    const int z0 = zk * zc, z1 = min(nz, z0 + zc);
    // neighbouring z chunks march in opposite directions (up in even chunks,
    // down in odd ones), so the layers around a common boundary are read by
    // both chunks at about the same time, through the same L2
    const int dir = (zk & 1) ? -1 : 1;
    const int zs = dir > 0 ? z0 : z1 - 1;

    const __amdgpu_buffer_rsrc_t rP = rsrc(Pin, (long)NS * N * SZ), rO = rsrc(Pout, (long)NS * N * SZ);
    const __amdgpu_buffer_rsrc_t rX = rsrc(tx, (long)N * SZ), rY = rsrc(ty, (long)N * SZ), rZ = rsrc(tz, (long)N * SZ);
    const __amdgpu_buffer_rsrc_t rD = rsrc(g.diag, (long)N * 8);
    // table words without the lo field (bits 20-22): x per lane, y per row
    int wx = 0;
    if (AM & 1) {
        const unsigned long long *mk = xmask + 3 * xt;
#pragma unroll
        for (int f = 0; f < 3; ++f) wx |= (int)((mk[f] >> lane) & 1) << (20 + f);
    }
    const int wy = (AM & 2) ? packy[yc] : 0;
    constexpr int mX = (AM & 1) ? 1 << am_bit<AM>(0) : 0;
    constexpr int mY = (AM & 2) ? 1 << am_bit<AM>(1) : 0;
    constexpr int mZ = (AM & 4) ? 1 << am_bit<AM>(2) : 0;
    const bool shx0 = (AM & 1) && ((wx >> 21) & 1), shx1 = (AM & 1) && ((wx >> 22) & 1);
    const bool shy0 = (AM & 2) && ((wy >> 21) & 1), shy1 = (AM & 2) && ((wy >> 22) & 1);
    const bool fxm = xc > 0, fxp = xc + 1 < nx, fym = yc > 0, fyp = yc + 1 < ny;
    // y neighbours: permuted slot offsets, uniform over the wavefront
    int sym_[NS], syp_[NS], soym[NS], soyp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sym_[s] = shy0 ? (s | mY) : s;
        syp_[s] = shy1 ? (s & ~mY) : s;
        soym[s] = sym_[s] * NSZ;
        soyp[s] = syp_[s] * NSZ;
    }
    const int base = xc + nx * yc;
    // Pm: the layer behind in the walk; tzm: the face between it and the
    // current layer (tz holds each cell's face to the layer above)
    int i = base + nxy * zs;
    const bool hasb = dir > 0 ? zs > 0 : zs + 1 < nz;
    const int ib = hasb ? i - dir * nxy : i;
    PT Pm[NS], Pc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Pc[s] = bload<PT>(rP, i * SZ, s * NSZ);
        Pm[s] = bload<PT>(rP, ib * SZ, s * NSZ);
    }
    const PT tzm0 = bload<PT>(rZ, (dir > 0 ? ib : i) * SZ, 0);
    if (*done) return;  // read once the first layers are in flight, before any barrier
    PT tzm = hasb ? tzm0 : (PT)0;
    double chg = 0.0;

    // rows y-1 and y+1 of the current layer: from the neighbouring
    // wavefronts through LDS (double buffered, one barrier per layer); the
    // first and last row of the workgroup load the row beyond from memory
    __shared__ PT rowbuf[2][kSweepRows][NS][64];
    const bool ym_mem = wv == 0, yp_mem = wv == kSweepRows - 1;
    for (int st = 0; st < z1 - z0; ++st, i += dir * nxy) {
        const int z = zs + st * dir;
        const bool fza = dir > 0 ? z + 1 < nz : z > 0;  // a layer ahead in the walk
        const int lym = fym ? i - nx : i, lyp = fyp ? i + nx : i;
        const int buf = st & 1;
#pragma unroll
        for (int s = 0; s < NS; ++s) rowbuf[buf][wv][s][lane] = Pc[s];
        PT Pn[NS], Ym[NS], Yp[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) Pn[s] = bload<PT>(rP, (fza ? i + dir * nxy : i) * SZ, s * NSZ);
        if (ym_mem) {
#pragma unroll
            for (int s = 0; s < NS; ++s) Ym[s] = bload<PT>(rP, lym * SZ, soym[s]);
        }
        if (yp_mem) {
#pragma unroll
            for (int s = 0; s < NS; ++s) Yp[s] = bload<PT>(rP, lyp * SZ, soyp[s]);
        }
        const PT txc = bload<PT>(rX, i * SZ, 0), tym = bload<PT>(rY, lym * SZ, 0);
        const PT tyc = bload<PT>(rY, i * SZ, 0);
        const PT tzc = bload<PT>(rZ, (dir > 0 || !fza ? i : i - nxy) * SZ, 0);  // face toward the layer ahead
        const double dg = bload<double>(rD, i * 8, 0);
        const int wz = (AM & 4) ? packz[z] : 0;
        const bool shz0 = (AM & 4) && ((wz >> 21) & 1), shz1 = (AM & 4) && ((wz >> 22) & 1);
        __syncthreads();
        if (!ym_mem) {
#pragma unroll
            for (int s = 0; s < NS; ++s) Ym[s] = rowbuf[buf][wv - 1][sym_[s]][lane];
        }
        if (!yp_mem) {
#pragma unroll
            for (int s = 0; s < NS; ++s) Yp[s] = rowbuf[buf][wv + 1][syp_[s]][lane];
        }

        // x neighbours from the adjacent lanes; lanes at a tile edge fetch
        // across it
        PT xm[NS], xp[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xm[s] = __shfl_up(Pc[s], 1, 64);
            xp[s] = __shfl_down(Pc[s], 1, 64);
        }
        PT txm = __shfl_up(txc, 1, 64);
        if (nxt > 1) {
            if (lane == 0 && fxm) {
#pragma unroll
                for (int s = 0; s < NS; ++s) xm[s] = bload<PT>(rP, (i - 1) * SZ, s * NSZ);
                txm = bload<PT>(rX, (i - 1) * SZ, 0);
            }
            if (lane == 63 && fxp) {
#pragma unroll
                for (int s = 0; s < NS; ++s) xp[s] = bload<PT>(rP, (i + 1) * SZ, s * NSZ);
            }
        }
        // Neighbour slot permutation along split axes (see above): a down
        // face with the shift reads slot s|m for the slots without bit m, an
        // up face reads slot s&~m for the slots with bit m; the other slots
        // are empty and weighted by zero.
        PT nb[6][NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            nb[0][s] = (mX && !(s & mX) && shx0) ? xm[s | mX] : xm[s];
            nb[1][s] = (mX && (s & mX) && shx1) ? xp[s & ~mX] : xp[s];
            nb[2][s] = Ym[s];
            nb[3][s] = Yp[s];
            // below (z - 1) and above (z + 1): behind and ahead in an upward
            // walk, ahead and behind in a downward one
            const PT lo = dir > 0 ? Pm[s] : Pn[s], lo2 = dir > 0 ? Pm[s | mZ] : Pn[s | mZ];
            const PT up = dir > 0 ? Pn[s] : Pm[s], up2 = dir > 0 ? Pn[s & ~mZ] : Pm[s & ~mZ];
            nb[4][s] = (mZ && !(s & mZ) && shz0) ? lo2 : lo;
            nb[5][s] = (mZ && (s & mZ) && shz1) ? up2 : up;
        }
        const bool sh[6] = {shx0, shx1, shy0, shy1, shz0, shz1};
        const PT tza = fza ? tzc : (PT)0;
        const PT T[6] = {fxm ? txm : (PT)0, txc, fym ? tym : (PT)0, fyp ? tyc : (PT)0, dir > 0 ? tzm : tza,
                         dir > 0 ? tza : tzm};

        PT acc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = (PT)0;
        PT db = (PT)0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int a = q >> 1;
            const bool up = q & 1;
            const PT Tq = T[q];
            const PT Tz = sh[q] ? (PT)0 : Tq;
            db += Tq;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const bool empty = ((AM >> a) & 1) && (up ? !(s & (1 << am_bit<AM>(a))) : (s & (1 << am_bit<AM>(a))));
                acc[s] += (empty ? Tz : Tq) * nb[q][s];
            }
        }
        // Inactive cells store zeros; a row whose new sum is not positive
        // keeps its old values and raises flag bit 2.
        const bool active = dg > 0.0;
        const int w[3] = {wx, wy, wz};
        bool ok[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bool v = true;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (((AM >> a) & 1) && (s & (1 << am_bit<AM>(a))) && !((w[a] >> 20) & 1)) v = false;
            ok[s] = v;
        }
        if (check_blocks && active) {
            const int lo[3] = {(AM & 1) ? cd.pack[0][xc] & 0xFFFFF : 0, wy & 0xFFFFF, wz & 0xFFFFF};
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (ok[s] && slot_block(cd, lo, s) < 0) ok[s] = false;
        }
        const PT idb = db > (PT)0 ? (PT)1 / db : (PT)0;
        PT pn[NS];
        PT rs = (PT)0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const PT v = db > (PT)0 ? Pc[s] - omega * (Pc[s] - acc[s] * idb) : Pc[s];
            pn[s] = ok[s] ? v : (PT)0;
            rs += pn[s];
        }
        const bool bad = own && active && !(rs > (PT)0);
        if (bad) atomicOr(flag, 2);
        const PT irs = (PT)1 / rs;
        double c = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const PT v = pn[s] * irs;
            const PT o = active ? (bad ? Pc[s] : v) : (PT)0;
            c = fmax(c, fabs((double)v - (double)Pc[s]));
            if (own) bstore<PT>(o, rO, i * SZ, s * NSZ);
        }
        chg = (own && active && !bad) ? fmax(chg, c) : chg;
        // slide the window
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Pm[s] = Pc[s];
            Pc[s] = Pn[s];
        }
        tzm = tzc;
    }
    const double mx = block_max(chg, lds);
    if (threadIdx.x == 0) part[b] = mx;
}

template <int AM, typename PT, int kSweepRows = sweep_rows<PT>()>
__global__ __launch_bounds__(64 * kSweepRows) void k_sweep(CartDev cd, Fine g, const PT *__restrict__ tx,
                                                           const PT *__restrict__ ty, const PT *__restrict__ tz,
                                                           const PT *__restrict__ Pin, PT *__restrict__ Pout,
                                                           PT omega, double *__restrict__ part, int *flag,
                                                           int check_blocks, const int *done, int nxt, int ngy,
                                                           int nzc, int zc, int nblk,
                                                           const unsigned long long *__restrict__ xmask,
                                                           const int *__restrict__ packy,
                                                           const int *__restrict__ packz) {
    sweep_body<AM, PT, kSweepRows>(blockIdx.x, gridDim.x, cd, g, tx, ty, tz, Pin, Pout, omega, part, flag,
                                   check_blocks, done, nxt, ngy, nzc, zc, nblk, xmask, packy, packz);
}

// Stop rule after sweep k: done once the change of sweep k is <= tol.  The
// change is the maximum of the npart per-workgroup maxima in part, or (npart
// = 0) the value already in maxbits[k]; it is recorded in maxbits[k].
__global__ __launch_bounds__(256) void k_sweep_check(Status *st, unsigned long long *maxbits, int k, double tol,
                                                     int max_sweeps, const double *__restrict__ part, int npart) {
    __shared__ double lds[4];
    if (st->done) return;
    double m = 0.0;
#pragma unroll 8
    for (int t = threadIdx.x; t < npart; t += blockDim.x) m = fmax(m, part[t]);
    m = block_max(m, lds);
    if (threadIdx.x == 0) {
        const double chg = npart > 0 ? m : __longlong_as_double((long long)maxbits[k]);
        maxbits[k] = (unsigned long long)__double_as_longlong(chg);
        st->iters = k + 1;
        st->relres = chg;
        if (chg <= tol || k + 1 >= max_sweeps) st->done = 1;
    }
}

// Stop rule after the sweeps k and k+1 of a pair (npair = 2), or after sweep
// k alone (npair = 1): the maxima of sweep k are in part[0..n0), those of
// sweep k+1 in part[stride..stride+n1), and sweep k+1 raised its row-sum flag
// in flag[1].  Sweep k is decided first, exactly as alone; if it stops, the
// extra sweep k+1 does not count (its result went to the other buffer and its
// flag is dropped), otherwise sweep k+1 is decided and its flag kept.
__device__ __forceinline__ void sweep_check_pair_body(Status *st, unsigned long long *maxbits, int k, int npair,
                                                      double tol, int max_sweeps, const double *__restrict__ part,
                                                      int n0, int n1, int stride, int *flag) {
    __shared__ double lds[4];
    if (st->done) return;
    double m0 = 0.0, m1 = 0.0;
    for (int t = threadIdx.x; t < n0; t += blockDim.x) m0 = fmax(m0, part[t]);
    m0 = block_max(m0, lds);
    if (npair > 1) {
        for (int t = threadIdx.x; t < n1; t += blockDim.x) m1 = fmax(m1, part[stride + t]);
        m1 = block_max(m1, lds);
    }
    if (threadIdx.x == 0) {
        maxbits[k] = (unsigned long long)__double_as_longlong(m0);
        st->iters = k + 1;
        st->relres = m0;
        if (m0 <= tol || k + 1 >= max_sweeps) {
            st->done = 1;
            flag[1] = 0;
        } else if (npair > 1) {
            maxbits[k + 1] = (unsigned long long)__double_as_longlong(m1);
            st->iters = k + 2;
            st->relres = m1;
            flag[0] |= flag[1];
            flag[1] = 0;
            if (m1 <= tol || k + 2 >= max_sweeps) st->done = 1;
        }
    }
}

__global__ __launch_bounds__(256) void k_sweep_check_pair(Status *st, unsigned long long *maxbits, int k,
                                                          int npair, double tol, int max_sweeps,
                                                          const double *__restrict__ part, int n0, int n1,
                                                          int stride, int *flag) {
    sweep_check_pair_body(st, maxbits, k, npair, tol, max_sweeps, part, n0, n1, stride, flag);
}

// Offset of the second sweep's maxima in c.partial (which holds at least
// twice as many doubles).
constexpr int kSweepPartStride = 65536;

// Workgroups of k_sweep<AM, PT> the device holds at once (occupancy x CUs),
// queried once per kernel instance.
template <int AM, typename PT>
static int sweep_resident(const Ctx &c) {
    static int cached = 0;
    if (cached == 0) {
        int per_cu = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep<AM, PT>, 64 * sweep_rows<PT>(), 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess || ncu < 1)
            ncu = 256;
        cached = per_cu * ncu;
    }
    return cached;
}

// Returns the number of per-workgroup maxima written to c.partial.  The z
// chunks are sized so that the whole grid is resident at once (one round of
// workgroups: a partial second round leaves a tail; measured on the
// 60x220x85 model, 41.7 -> 39.5 us in FP64).
template <int AM, typename PT>
static int sweep_launch(Ctx &c, Stage &s, const PT *tx, const PT *ty, const PT *tz, const PT *in, PT *out,
                        int check_blocks, double *part, int *flag) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    constexpr int kSweepRows = sweep_rows<PT>();
    const int nxt = cdiv(c.nx, 64), ngy = cdiv(c.ny, kSweepRows);
    int nzc = std::min(c.nz, std::max(1, sweep_resident<AM, PT>(c) / (ngy * nxt)));
    const int zc = cdiv(c.nz, nzc);
    nzc = cdiv(c.nz, zc);
    const int nblk = nzc * ngy * nxt;
    const dim3 grid(xcd_grid(nblk)), blk(64 * kSweepRows);
    const PT om = (PT)c.opt.omega;
    const int *done = &c.status->done;
    hipEvent_t e0, e1;  // timed by the dispatch when sweeps are profiled
    prof_pair(c, MSRSB_K_SWEEP, &e0, &e1);
    hipExtLaunchKernelGGL((k_sweep<AM, PT>), grid, blk, 0, c.stream, e0, e1, 0, s.cart, g, tx, ty, tz, in, out, om,
                          part, flag, check_blocks, done, nxt, ngy, nzc, zc, nblk,
                          (const unsigned long long *)s.cart.xmask, s.cart.pack[1], s.cart.pack[2]);
    return nblk;
}

template <typename PT>
static int sweep_dispatch(Ctx &c, Stage &s, const PT *tx, const PT *ty, const PT *tz, const PT *in, PT *out,
                          int check_blocks, double *part, int *flag) {
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (s.cart.bit[a] >= 0) am |= 1 << a;
    switch (am) {
    case 0: return sweep_launch<0, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 1: return sweep_launch<1, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 2: return sweep_launch<2, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 3: return sweep_launch<3, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 4: return sweep_launch<4, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 5: return sweep_launch<5, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    case 6: return sweep_launch<6, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    default: return sweep_launch<7, PT>(c, s, tx, ty, tz, in, out, check_blocks, part, flag);
    }
}

template <typename PT>
static void init_dispatch(Ctx &c, Stage &s, PT *P) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const dim3 grid(cdiv(c.N, kBlock)), blk(kBlock);
    switch (s.ns) {
    case 1: hipLaunchKernelGGL((k_basis_init<1, PT>), grid, blk, 0, c.stream, s.cart, g, P); break;
    case 2: hipLaunchKernelGGL((k_basis_init<2, PT>), grid, blk, 0, c.stream, s.cart, g, P); break;
    case 4: hipLaunchKernelGGL((k_basis_init<4, PT>), grid, blk, 0, c.stream, s.cart, g, P); break;
    default: hipLaunchKernelGGL((k_basis_init<8, PT>), grid, blk, 0, c.stream, s.cart, g, P); break;
    }
}

__device__ __forceinline__ void to_bf16_body(int bid, int nblk, long n, const float *__restrict__ in,
                                             uint16_t *__restrict__ out) {
    const long k = (long)bid * blockDim.x + threadIdx.x;
    if (k < n) out[k] = float_to_bf16(in[k]);
}

__global__ void k_to_bf16(long n, const float *__restrict__ in, uint16_t *__restrict__ out) {
    to_bf16_body(blockIdx.x, gridDim.x, n, in, out);
}

__device__ __forceinline__ void status_reset_body(Status *st, int *flag) {
    st->done = 0;
    st->iters = 0;
    st->relres = 0.0;
    flag[0] = 0;
    flag[1] = 0;
}

__global__ void k_status_reset(Status *st, int *flag) {
    status_reset_body(st, flag);
}

// Run up to max_sweeps sweeps (device-side stop rule); returns MSRSB status.
int launch_sweeps(Ctx &c, Stage &s, int max_sweeps, double tol, bool warm, int *sweeps, double *change) {
    const bool mixed = c.opt.precision == MSRSB_MIXED;
    const int check_blocks = (int)s.h_present.size() != s.cart.m[0] * s.cart.m[1] * s.cart.m[2];
    if (!warm) {
        if (s.kind == 2) launch_xinit(c, s);
        else if (mixed) init_dispatch<float>(c, s, s.P32[0]);
        else init_dispatch<double>(c, s, s.P64[0]);
        s.cur = 0;
    }
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, c.stream, c.status, c.flag);
    int done_sweeps = 0;
    double last = nan("");
    if (max_sweeps > 0) {
        if (hipMemsetAsync(c.maxbits, 0, sizeof(unsigned long long) * (size_t)max_sweeps, c.stream) != hipSuccess)
            return hip_fail(hipGetLastError(), "memset");
        int k = 0;
        int chunk = 8;
        // a sweep has at most max(resident workgroups, row groups x x tiles)
        // workgroups; pairs need that many maxima per half of c.partial
        const bool pairs = s.kind != 2 && (long)cdiv(c.ny, 4) * cdiv(c.nx, 64) <= kSweepPartStride;
        while (k < max_sweeps) {
            const int kend = std::min(max_sweeps, k + chunk);
            while (k < kend) {
                if (!pairs) {
                    const int in = (s.cur + k) & 1, out = in ^ 1;
                    int npart = 0;
                    if (s.kind == 2) {
                        ProfScope ps(c, MSRSB_K_SWEEP);
                        npart = launch_xsweep(c, s, in, out);
                    } else if (mixed) {
                        npart = sweep_dispatch<float>(c, s, c.tx32, c.ty32, c.tz32, s.P32[in], s.P32[out],
                                                      check_blocks, c.partial, c.flag);
                    } else {
                        npart = sweep_dispatch<double>(c, s, c.tx, c.ty, c.tz, s.P64[in], s.P64[out], check_blocks,
                                                       c.partial, c.flag);
                    }
                    hipLaunchKernelGGL(k_sweep_check, dim3(1), dim3(256), 0, c.stream, c.status, c.maxbits, k, tol,
                                       max_sweeps, c.partial, npart);
                    ++k;
                    continue;
                }
                // rectilinear stages: two sweeps per stop-rule check (one
                // launch fewer per pair), each with its own maxima and flag
                const int npair = k + 1 < kend ? 2 : 1;
                int np[2] = {0, 0};
                for (int q = 0; q < npair; ++q) {
                    const int in = (s.cur + k + q) & 1, out = in ^ 1;
                    double *part = c.partial + (size_t)q * kSweepPartStride;
                    if (mixed)
                        np[q] = sweep_dispatch<float>(c, s, c.tx32, c.ty32, c.tz32, s.P32[in], s.P32[out],
                                                      check_blocks, part, c.flag + q);
                    else
                        np[q] = sweep_dispatch<double>(c, s, c.tx, c.ty, c.tz, s.P64[in], s.P64[out], check_blocks,
                                                       part, c.flag + q);
                }
                hipLaunchKernelGGL(k_sweep_check_pair, dim3(1), dim3(256), 0, c.stream, c.status, c.maxbits, k,
                                   npair, tol, max_sweeps, c.partial, np[0], np[1], kSweepPartStride, c.flag);
                k += npair;
            }
            hipError_t e = hipMemcpyAsync(c.h_status, c.status, sizeof(Status), hipMemcpyDeviceToHost, c.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
            if (e != hipSuccess) return hip_fail(e, "sweep status");
            if (c.h_status->done) break;
            chunk = std::min(chunk * 2, 64);
        }
        done_sweeps = c.h_status->iters;
        last = c.h_status->relres;
        int hflag = 0;
        hipError_t e = hipMemcpyAsync(&hflag, c.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return hip_fail(e, "sweep flag");
        if (hflag & 2) {
            set_error("basis row sum not positive");
            return MSRSB_E_SINGULAR;
        }
    }
    s.cur = (s.cur + done_sweeps) & 1;
    if (mixed) {
        const long n = (long)s.ns * c.N;
        hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, s.P32[s.cur], s.Pbf);
    }
    if (s.kind == 2) launch_xlist(c, s);
    s.sweeps = done_sweeps;
    s.change = last;
    if (sweeps) *sweeps = done_sweeps;
    if (change) *change = last;
    return MSRSB_OK;
}
// ------------------------------------------------------- batched launches ----
// Cold basis construction of every member's rectilinear stage: one launch per
// sweep (per split-axis mask) over all members, the stop rule per member.  A
// batched sweep walks each column in a few chunks; a sweep's
// values do not depend on the chunks, and its change is a maximum.

// z chunks per column group of a batched sweep (FP64 rows come four to a
// workgroup, FP32 rows eight: the FP32 form has half as many workgroups)
template <typename PT>
constexpr int batch_sweep_zchunks() {
    return sizeof(PT) == 8 ? 1 : 2;
}

// sweep grid and key (split-axis mask) of a member; fills its sweep geometry
int bat_member_sweep(const Ctx &c, const Stage &s, BMember &d, int *key) {
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (s.cart.bit[a] >= 0) am |= 1 << a;
    const int rows = c.opt.precision == MSRSB_MIXED ? sweep_rows<float>() : sweep_rows<double>();
    d.s_nxt = cdiv(c.nx, 64);
    d.s_ngy = cdiv(c.ny, rows);
    const int nzc = std::min(c.nz, c.opt.precision == MSRSB_MIXED ? batch_sweep_zchunks<float>()
                                                                   : batch_sweep_zchunks<double>());
    d.s_zc = cdiv(c.nz, nzc);
    d.s_nzc = cdiv(c.nz, d.s_zc);
    d.s_nblk = d.s_nzc * d.s_nxt * d.s_ngy;
    d.check_blocks = (int)s.h_present.size() != s.cart.m[0] * s.cart.m[1] * s.cart.m[2];
    *key = am;
    return xcd_grid(d.s_nblk);
}

#define BAT_LOCATE()                              \
    int m, lb, nb;                                \
    if (!bat_locate(gp, act, m, lb, nb)) return;  \
    const BMember &d = D[m]

template <int NS, typename PT>
__global__ void k_basis_init_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    basis_init_body<NS, PT>(lb, nb, d.cd, d.g, (PT *)d.P[0]);
}

__global__ __launch_bounds__(256) void k_sweep_reset_b(const BMember *D, BGroup gp, const int *act, int max_sweeps) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    if (threadIdx.x == 0) status_reset_body(d.status, d.flag);
    for (int k = threadIdx.x; k < max_sweeps; k += blockDim.x) d.maxbits[k] = 0ull;
}

template <int AM, typename PT>
__global__ __launch_bounds__(64 * sweep_rows<PT>()) void k_sweep_b(const BMember *D, BGroup gp, const int *act,
                                                                  int in, int q, PT omega) {
    BAT_LOCATE();
    sweep_body<AM, PT, sweep_rows<PT>()>(lb, nb, d.cd, d.g, (const PT *)d.wtx, (const PT *)d.wty, (const PT *)d.wtz,
                                         (const PT *)d.P[in], (PT *)d.P[in ^ 1], omega,
                                         d.partial + (size_t)q * kSweepPartStride, d.flag + q, d.check_blocks,
                                         &d.status->done, d.s_nxt, d.s_ngy, d.s_nzc, d.s_zc, d.s_nblk,
                                         (const unsigned long long *)d.cd.xmask, d.cd.pack[1], d.cd.pack[2]);
}

__global__ __launch_bounds__(256) void k_sweep_check_pair_b(const BMember *D, BGroup gp, const int *act, int k,
                                                            int npair, double tol, int max_sweeps) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    sweep_check_pair_body(d.status, d.maxbits, k, npair, tol, max_sweeps, d.partial, d.s_nblk, d.s_nblk,
                          kSweepPartStride, d.flag);
}

__global__ void k_to_bf16_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    to_bf16_body(lb, nb, (long)d.ns * d.g.N, (const float *)d.P[d.cur], d.Pbf);
}

#undef BAT_LOCATE

template <typename PT>
static void bat_init_t(Batch &B, const HGroup &h) {
    const dim3 grid(h.g.total), blk(kBlock);
    switch (h.key) {
    case 1: hipLaunchKernelGGL((k_basis_init_b<1, PT>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act); break;
    case 2: hipLaunchKernelGGL((k_basis_init_b<2, PT>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act); break;
    case 4: hipLaunchKernelGGL((k_basis_init_b<4, PT>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act); break;
    default: hipLaunchKernelGGL((k_basis_init_b<8, PT>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act); break;
    }
}

// basis from the partition of unity of the blocks, status and sweep maxima cleared
void bat_sweep_begin(Batch &B, int max_sweeps) {
    for (const HGroup &h : B.init) {
        if (h.g.n == 0) continue;
        if (B.mixed) bat_init_t<float>(B, h);
        else bat_init_t<double>(B, h);
    }
    for (const HGroup &h : B.one)
        if (h.g.n > 0)
            hipLaunchKernelGGL(k_sweep_reset_b, dim3(h.g.total), dim3(256), 0, B.stream, B.d_mem, h.g, B.d_act,
                               max_sweeps);
}

template <typename PT>
static void bat_sweep_t(Batch &B, const HGroup &h, int in, int q, PT om) {
    const dim3 grid(h.g.total), blk(64 * sweep_rows<PT>());
#define MSRSB_BSW(AM)                                                                                       \
    case AM:                                                                                                \
        hipLaunchKernelGGL((k_sweep_b<AM, PT>), grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act, in, q, om);  \
        break
    switch (h.key) {
        MSRSB_BSW(0); MSRSB_BSW(1); MSRSB_BSW(2); MSRSB_BSW(3);
        MSRSB_BSW(4); MSRSB_BSW(5); MSRSB_BSW(6); MSRSB_BSW(7);
    default: break;
    }
#undef MSRSB_BSW
}

// sweeps k and k+1 (npair = 2) or k alone, then the stop rule of each member
void bat_sweep_pair(Batch &B, int k, int npair, double omega, double tol, int max_sweeps) {
    for (int q = 0; q < npair; ++q) {
        const int in = (k + q) & 1;
        for (const HGroup &h : B.sweep) {
            if (h.g.n == 0) continue;
            if (B.mixed) bat_sweep_t<float>(B, h, in, q, (float)omega);
            else bat_sweep_t<double>(B, h, in, q, omega);
        }
    }
    for (const HGroup &h : B.one)
        if (h.g.n > 0)
            hipLaunchKernelGGL(k_sweep_check_pair_b, dim3(h.g.total), dim3(256), 0, B.stream, B.d_mem, h.g, B.d_act,
                               k, npair, tol, max_sweeps);
}

// the BF16 copy of every member's final FP32 basis
void bat_to_bf16(Batch &B) {
    for (const HGroup &h : B.bf16)
        if (h.g.n > 0)
            hipLaunchKernelGGL(k_to_bf16_b, dim3(h.g.total), dim3(kBlock), 0, B.stream, B.d_mem, h.g, B.d_act);
}

}  // namespace msrsb
