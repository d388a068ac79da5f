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
// entry change goes to maxbits (bit pattern of a non-negative double).
//
// AM is the mask of split axes (m_d > 1); axis d owns slot bit
// popcount(AM & ((1 << d) - 1)).  Neighbour l of cell i along a split axis
// holds block lo_i + b (slot bit b) in its slot bit b + (lo_i - lo_l), where
// lo_i - lo_l is 0 or +-1; a shifted bit outside {0,1} means the block is not
// in l's support (value 0).  So the values cell i needs from l are l's own
// NS slots, permuted (bit flipped where lo differs) and masked: every load
// address depends on i alone and all loads of a cell are issued before the
// first use.  Faces outside the grid and faces with zero transmissibility
// contribute exactly zero; their loads are clamped to cell i.
template <int AM>
__device__ constexpr int am_bit(int a) {
    return __builtin_popcount(AM & ((1 << a) - 1));
}

template <int AM, typename PT>
__global__ __launch_bounds__(kBlock) void k_sweep(CartDev cd, Fine g, const PT *__restrict__ tx,
                                                  const PT *__restrict__ ty, const PT *__restrict__ tz,
                                                  const PT *__restrict__ Pin, PT *__restrict__ Pout, PT omega,
                                                  unsigned long long *maxbits, int *flag, int check_blocks,
                                                  const int *done) {
    constexpr int NS = 1 << __builtin_popcount(AM);
    __shared__ double lds[kBlock / 64];
    if (*done) return;
    const int i = xzy_cell(xcd_block() * blockDim.x + threadIdx.x, g.nx, g.ny, g.nz);
    double chg = 0.0;
    if (i >= 0) {
        const int N = g.N;
        int c[3];
        cell_coords(g, i, c);
        int w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a] = (AM >> a) & 1 ? cd.pack[a][c[a]] : 0;
        const bool active = g.diag[i] > 0.0;
        PT p[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) p[s] = Pin[s * N + i];
        // faces in the order -x, +x, -y, +y, -z, +z
        int l[6];
        PT T[6];
        const int step[3] = {1, g.nx, g.nxy};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const PT *Ta = a == 0 ? tx : (a == 1 ? ty : tz);
            const bool dn = i >= step[a], up = i + step[a] < N;
            l[2 * a] = dn ? i - step[a] : i;
            l[2 * a + 1] = up ? i + step[a] : i;
            const PT td = Ta[l[2 * a]], tu = Ta[i];
            T[2 * a] = dn ? td : (PT)0;
            T[2 * a + 1] = up ? tu : (PT)0;
        }
        PT nb[6][NS];
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s) nb[q][s] = Pin[s * N + l[q]];

        PT acc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = (PT)0;
        PT db = (PT)0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int a = q >> 1;
            const PT Tq = T[q];
            db += Tq;
            if (!((AM >> a) & 1)) {
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[s] += Tq * nb[q][s];
            } else {
                const int m = 1 << am_bit<AM>(a);
                // down face: lo_i - lo_l = (w >> 21) & 1; up face: lo_l - lo_i = (w >> 22) & 1
                const bool shift = (q & 1) ? ((w[a] >> 22) & 1) : ((w[a] >> 21) & 1);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    PT v;
                    if (q & 1)
                        v = (s & m) ? nb[q][s & ~m] : (PT)0;  // l's bit 0 is i's bit 1
                    else
                        v = (s & m) ? (PT)0 : nb[q][s | m];   // l's bit 1 is i's bit 0
                    acc[s] += Tq * (shift ? v : nb[q][s]);
                }
            }
        }
        // Inactive cells store zeros; a row whose new sum is not positive keeps
        // its old values and raises flag bit 2.  Selects rather than branches,
        // so that no load is sunk behind the test on diag.
        int lo[3];
        bool ok[NS];
#pragma unroll
        for (int a = 0; a < 3; ++a) lo[a] = w[a] & 0xFFFFF;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bool v = true;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (((AM >> a) & 1) && (s & (1 << am_bit<AM>(a))) && !((w[a] >> 20) & 1)) v = false;
            ok[s] = v;
        }
        if (check_blocks && active) {
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
        const bool bad = active && !(rs > (PT)0);
        if (bad) atomicOr(flag, 2);
        const PT irs = (PT)1 / rs;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const PT v = pn[s] * irs;
            const PT o = active ? (bad ? p[s] : v) : (PT)0;
            chg = (active && !bad) ? fmax(chg, fabs((double)v - (double)p[s])) : chg;
            Pout[s * N + i] = o;
        }
    }
    const double m = block_max(chg, lds);
    if (threadIdx.x == 0 && m > 0.0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
}

// Stop rule after sweep k: done once the change of sweep k is <= tol.
__global__ void k_sweep_check(Status *st, const unsigned long long *maxbits, int k, double tol, int max_sweeps) {
    if (st->done) return;
    const double chg = __longlong_as_double((long long)maxbits[k]);
    st->iters = k + 1;
    st->relres = chg;
    if (chg <= tol || k + 1 >= max_sweeps) st->done = 1;
}

template <typename PT>
static void sweep_dispatch(Ctx &c, Stage &s, const PT *tx, const PT *ty, const PT *tz, const PT *in, PT *out,
                           unsigned long long *bits, int check_blocks) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const dim3 grid(xcd_grid(cdiv(c.N, kBlock))), blk(kBlock);
    const PT om = (PT)c.opt.omega;
    const int *done = &c.status->done;
    int am = 0;
    for (int a = 0; a < 3; ++a)
        if (s.cart.bit[a] >= 0) am |= 1 << a;
#define MSRSB_SWEEP(AM) \
    case AM: hipLaunchKernelGGL((k_sweep<AM, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om, bits, c.flag, check_blocks, done); break;
    switch (am) {
        MSRSB_SWEEP(0) MSRSB_SWEEP(1) MSRSB_SWEEP(2) MSRSB_SWEEP(3)
        MSRSB_SWEEP(4) MSRSB_SWEEP(5) MSRSB_SWEEP(6) MSRSB_SWEEP(7)
    }
#undef MSRSB_SWEEP
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
                ProfScope ps(c, MSRSB_K_SWEEP);
                if (s.kind == 2)
                    launch_xsweep(c, s, in, out, c.maxbits + k);
                else if (mixed)
                    sweep_dispatch<float>(c, s, c.tx32, c.ty32, c.tz32, s.P32[in], s.P32[out], c.maxbits + k,
                                          check_blocks);
                else
                    sweep_dispatch<double>(c, s, c.tx, c.ty, c.tz, s.P64[in], s.P64[out], c.maxbits + k,
                                           check_blocks);
                hipLaunchKernelGGL(k_sweep_check, dim3(1), dim3(1), 0, c.stream, c.status, c.maxbits, k, tol,
                                   max_sweeps);
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
