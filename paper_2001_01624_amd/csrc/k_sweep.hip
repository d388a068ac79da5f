// Rectilinear-stage basis kernels: restricted-smoothing sweeps (MsRSB) with
// the device-side stop rule.
//
// Basis layout: slot-major, P[s*N + i].  A cell lies in the supports of at
// most two consecutive blocks per axis (lo[i] and lo[i]+1), so its slots are
// implicit: slot s picks, for every axis d with more than one block, block
// lo_d + bit_d(s).  No block indices are stored; a slot that is not in the
// support (beyond nv, an inactive cell, a dropped block) holds exactly 0.
#include <algorithm>

#include "cart_util.h"
#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

// ---------------------------------------------------------------- sweeps ----

template <int NS, typename PT>
__global__ void k_basis_init(CartDev cd, Fine g, PT *__restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
// Work layout: a wavefront owns a run of 64 cells along x of one row (y, z);
// rows are visited z fastest, so the z neighbours of a row are the rows of
// the adjacent wavefronts.  Within a wavefront y and z (and so the y and z
// neighbour shifts) are uniform.  Loads go through buffer resources with
// the slot offset in a scalar register, so a neighbour's NS slots cost one
// vector address.  All loads of a cell are issued before the first use;
// faces outside the grid have T = 0 and their loads are clamped to the cell.
// Faces are added in the order -x, +x, -y, +y, -z, +z.
template <int AM>
__device__ constexpr int am_bit(int a) {
    return __builtin_popcount(AM & ((1 << a) - 1));
}

constexpr int kSweepRows = 4;  // rows (wavefronts) per workgroup

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

template <int AM, typename PT>
__global__ __launch_bounds__(64 * kSweepRows) void k_sweep(CartDev cd, Fine g, const PT *__restrict__ tx,
                                                           const PT *__restrict__ ty, const PT *__restrict__ tz,
                                                           const PT *__restrict__ Pin, PT *__restrict__ Pout,
                                                           PT omega, double *__restrict__ part, int *flag,
                                                           int check_blocks, const int *done, int nxt, int nblk,
                                                           const unsigned long long *__restrict__ xmask,
                                                           const int *__restrict__ packy,
                                                           const int *__restrict__ packz) {
    constexpr int NS = 1 << __builtin_popcount(AM);
    constexpr int SZ = sizeof(PT);
    __shared__ double lds[kSweepRows];
    if (*done) return;
    const int b = xcd_block();
    if (b >= nblk) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = g.nxy, N = g.N;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xt = b % nxt;
    const int row = (b / nxt) * kSweepRows + wv;  // row = z + nz * y
    const bool row_ok = row < ny * nz;
    const int rc = row_ok ? row : ny * nz - 1;
    const int y = rc / nz, z = rc - y * nz;
    const int x = xt * 64 + lane;
    const bool own = row_ok && x < nx;
    const int xc = min(x, nx - 1);
    const int i = xc + nx * y + nxy * z;

    const __amdgpu_buffer_rsrc_t rP = rsrc(Pin, (long)NS * N * SZ), rO = rsrc(Pout, (long)NS * N * SZ);
    const __amdgpu_buffer_rsrc_t rX = rsrc(tx, (long)N * SZ), rY = rsrc(ty, (long)N * SZ), rZ = rsrc(tz, (long)N * SZ);
    // neighbour cells (clamped to i outside the grid) in face order
    const bool fin[6] = {xc > 0, xc + 1 < nx, y > 0, y + 1 < ny, z > 0, z + 1 < nz};
    const int l[6] = {fin[0] ? i - 1 : i, fin[1] ? i + 1 : i, fin[2] ? i - nx : i,
                      fin[3] ? i + nx : i, fin[4] ? i - nxy : i, fin[5] ? i + nxy : i};
    // table words without the lo field (bits 20-22); y and z are uniform
    int wx = 0;
    if (AM & 1) {
        const unsigned long long *mk = xmask + 3 * xt;
#pragma unroll
        for (int f = 0; f < 3; ++f) wx |= (int)((mk[f] >> lane) & 1) << (20 + f);
    }
    const int wy = (AM & 2) ? packy[y] : 0;
    const int wz = (AM & 4) ? packz[z] : 0;
    const int w[3] = {wx, wy, wz};
    // Face q along a split axis with its shift bit set (lo of the neighbour
    // differs): on a down face slot s reads the neighbour's slot s|m and the
    // slots with bit m are empty; on an up face slot s reads slot s&~m and
    // the slots without bit m are empty.  The permutation goes into the load
    // offsets (scalar for y and z, where the shift is uniform; per lane for
    // x) and the empty slots are weighted by Tz = 0 instead of T.
    bool sh[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) sh[q] = ((AM >> (q >> 1)) & 1) && ((w[q >> 1] >> ((q & 1) ? 22 : 21)) & 1);
    const int NSZ = N * SZ;
    PT p[NS], nb[6][NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) p[s] = bload<PT>(rP, i * SZ, s * NSZ);
    const PT t0 = bload<PT>(rX, l[0] * SZ, 0), t1 = bload<PT>(rX, i * SZ, 0);
    const PT t2 = bload<PT>(rY, l[2] * SZ, 0), t3 = bload<PT>(rY, i * SZ, 0);
    const PT t4 = bload<PT>(rZ, l[4] * SZ, 0), t5 = bload<PT>(rZ, i * SZ, 0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int a = q >> 1;
        const bool up = q & 1;
        if (!((AM >> a) & 1)) {
#pragma unroll
            for (int s = 0; s < NS; ++s) nb[q][s] = bload<PT>(rP, l[q] * SZ, s * NSZ);
            continue;
        }
        const int m = 1 << am_bit<AM>(a);
        if (a == 0) {
            // per-lane shift.  Down face: the moved slots s read s + m, the
            // vector offset gains m planes when shifted.  Up face: the moved
            // slots read s - m, put in the scalar offset, and the vector offset
            // gains the m planes back when not shifted (a vector offset stays
            // non-negative: the buffer range check applies to it alone).
            const int vo = l[q] * SZ, vs = vo + ((sh[q] != up) ? m * NSZ : 0);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const bool moved = up ? (s & m) : !(s & m);
                nb[q][s] = bload<PT>(rP, moved ? vs : vo, (moved && up ? s - m : s) * NSZ);
            }
        } else {
            const bool shu = __builtin_amdgcn_readfirstlane(sh[q]);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int s2 = shu ? (up ? (s & ~m) : (s | m)) : s;
                nb[q][s] = bload<PT>(rP, l[q] * SZ, s2 * NSZ);
            }
        }
    }
    const double dg = g.diag[i];
    // keep every load above this point: one memory round trip per wavefront
    __builtin_amdgcn_sched_barrier(0);
    const PT T[6] = {fin[0] ? t0 : (PT)0, fin[1] ? t1 : (PT)0, fin[2] ? t2 : (PT)0,
                     fin[3] ? t3 : (PT)0, fin[4] ? t4 : (PT)0, fin[5] ? t5 : (PT)0};

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
    // Inactive cells store zeros; a row whose new sum is not positive keeps
    // its old values and raises flag bit 2.
    const bool active = dg > 0.0;
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
        const PT v = db > (PT)0 ? p[s] - omega * (p[s] - acc[s] * idb) : p[s];
        pn[s] = ok[s] ? v : (PT)0;
        rs += pn[s];
    }
    const bool bad = own && active && !(rs > (PT)0);
    if (bad) atomicOr(flag, 2);
    const PT irs = (PT)1 / rs;
    double chg = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const PT v = pn[s] * irs;
        const PT o = active ? (bad ? p[s] : v) : (PT)0;
        chg = fmax(chg, fabs((double)v - (double)p[s]));
        if (own) bstore<PT>(o, rO, i * SZ, s * N * SZ);
    }
    chg = (own && active && !bad) ? chg : 0.0;
    const double mx = block_max(chg, lds);
    if (threadIdx.x == 0) part[b] = mx;
}

// Stop rule after sweep k: done once the change of sweep k is <= tol.  The
// change is the maximum of the npart per-workgroup maxima in part, or (npart
// = 0) the value already in maxbits[k]; it is recorded in maxbits[k].
__global__ __launch_bounds__(256) void k_sweep_check(Status *st, unsigned long long *maxbits, int k, double tol,
                                                     int max_sweeps, const double *__restrict__ part, int npart) {
    __shared__ double lds[4];
    if (st->done) return;
    double m = 0.0;
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

// Returns the number of per-workgroup maxima written to c.partial.
template <typename PT>
static int sweep_dispatch(Ctx &c, Stage &s, const PT *tx, const PT *ty, const PT *tz, const PT *in, PT *out,
                          int check_blocks) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const int nxt = cdiv(c.nx, 64);
    const int nblk = nxt * cdiv((long)c.ny * c.nz, kSweepRows);
    const dim3 grid(xcd_grid(nblk)), blk(64 * kSweepRows);
    const PT om = (PT)c.opt.omega;
    const int *done = &c.status->done;
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (s.cart.bit[a] >= 0) am |= 1 << a;
#define MSRSB_SWEEP(AM)                                                                                         \
    case AM:                                                                                                    \
        hipLaunchKernelGGL((k_sweep<AM, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om,       \
                           c.partial, c.flag, check_blocks, done, nxt, nblk, (const unsigned long long *)s.cart.xmask,\
                           s.cart.pack[1], s.cart.pack[2]);                                                     \
        break;
    switch (am) {
        MSRSB_SWEEP(0) MSRSB_SWEEP(1) MSRSB_SWEEP(2) MSRSB_SWEEP(3)
        MSRSB_SWEEP(4) MSRSB_SWEEP(5) MSRSB_SWEEP(6) MSRSB_SWEEP(7)
    }
#undef MSRSB_SWEEP
    return nblk;
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

__global__ void k_to_bf16(long n, const float *__restrict__ in, uint16_t *__restrict__ out) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = float_to_bf16(in[k]);
}

__global__ void k_status_reset(Status *st, int *flag) {
    st->done = 0;
    st->iters = 0;
    st->relres = 0.0;
    *flag = 0;
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
        while (k < max_sweeps) {
            const int kend = std::min(max_sweeps, k + chunk);
            for (; k < kend; ++k) {
                const int in = (s.cur + k) & 1, out = in ^ 1;
                int npart = 0;
                {
                    ProfScope ps(c, MSRSB_K_SWEEP);
                    if (s.kind == 2)
                        launch_xsweep(c, s, in, out, c.maxbits + k);
                    else if (mixed)
                        npart = sweep_dispatch<float>(c, s, c.tx32, c.ty32, c.tz32, s.P32[in], s.P32[out],
                                                      check_blocks);
                    else
                        npart = sweep_dispatch<double>(c, s, c.tx, c.ty, c.tz, s.P64[in], s.P64[out], check_blocks);
                }
                hipLaunchKernelGGL(k_sweep_check, dim3(1), dim3(256), 0, c.stream, c.status, c.maxbits, k, tol,
                                   max_sweeps, c.partial, npart);
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
    s.sweeps = done_sweeps;
    s.change = last;
    if (sweeps) *sweeps = done_sweeps;
    if (change) *change = last;
    return MSRSB_OK;
}
}  // namespace msrsb
