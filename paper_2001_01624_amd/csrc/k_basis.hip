// Rectilinear-stage basis kernels: restricted-smoothing sweeps (MsRSB),
// restriction d = P^T r, prolongation x += P p_c and the Galerkin product
// A_c = P^T A P (eq. pressure_system_reduced with R = P^T).
//
// Basis layout: slot-major, P[s*N + i].  A cell lies in the supports of at
// most two consecutive blocks per axis (lo[i] and lo[i]+1), so its slots are
// implicit: slot s picks, for every axis d with more than one block, block
// lo_d + bit_d(s).  No block indices are stored; a slot that is not in the
// support (beyond nv, an inactive cell, a dropped block) holds exactly 0.
#include <algorithm>

#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

__device__ inline int axis_stride(const Fine &g, int a) { return a == 0 ? 1 : (a == 1 ? g.nx : g.nxy); }

template <typename PT>
__device__ inline const PT *axis_T(int a, const PT *tx, const PT *ty, const PT *tz) {
    return a == 0 ? tx : (a == 1 ? ty : tz);
}

__device__ inline void cell_coords(const Fine &g, int i, int c[3]) {
    c[0] = i % g.nx;
    c[1] = (i / g.nx) % g.ny;
    c[2] = i / g.nxy;
}

// Is slot s of a cell with per-axis (lo, nv) inside the support?
__device__ inline bool slot_ok(const CartDev &cd, const int nv[3], int s) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (cd.bit[a] >= 0 && ((s >> cd.bit[a]) & 1) >= nv[a]) return false;
    return true;
}

__device__ inline int slot_block(const CartDev &cd, const int lo[3], int s) {
    int J[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) J[a] = lo[a] + (cd.bit[a] >= 0 ? ((s >> cd.bit[a]) & 1) : 0);
    return cd.cmap[J[0] + cd.m[0] * (J[1] + cd.m[1] * J[2])];
}

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
// Neighbour l of cell i along a split axis holds block lo_i + b (slot bit b)
// in its slot bit b + (lo_i - lo_l), where lo_i - lo_l is 0 or +-1; a shifted
// bit outside {0,1} means the block is not in l's support (value 0).  Slots
// with bit b >= nv_l hold exact zeros, so no other test is needed.  The
// per-axis table word packs lo, nv and the two neighbour shifts.
template <int NS, typename PT>
__global__ __launch_bounds__(kBlock) void k_sweep(CartDev cd, Fine g, const PT *__restrict__ tx,
                                                  const PT *__restrict__ ty, const PT *__restrict__ tz,
                                                  const PT *__restrict__ Pin, PT *__restrict__ Pout, PT omega,
                                                  unsigned long long *maxbits, int *flag, int check_blocks,
                                                  const int *done) {
    __shared__ double lds[kBlock / 64];
    if (*done) return;
    const int i = xzy_cell(xcd_block() * blockDim.x + threadIdx.x, g.nx, g.ny, g.nz);
    double chg = 0.0;
    if (i >= 0) {
        const long N = g.N;
        if (!(g.diag[i] > 0.0)) {
#pragma unroll
            for (int s = 0; s < NS; ++s) Pout[s * N + i] = (PT)0;
        } else {
            int c[3], lo[3], nv2[3], dmin[3], dpl[3];
            cell_coords(g, i, c);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int w = cd.pack[a][c[a]];
                lo[a] = w & 0xFFFFF;
                nv2[a] = (w >> 20) & 1;
                dmin[a] = (w >> 21) & 1;  // lo[c] - lo[c-1]
                dpl[a] = (w >> 22) & 1;   // lo[c+1] - lo[c]
            }
            PT p[NS], acc[NS];
            bool ok[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                bool v = true;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (cd.bit[a] >= 0 && ((s >> cd.bit[a]) & 1) > nv2[a]) v = false;
                if (check_blocks && v && slot_block(cd, lo, s) < 0) v = false;
                ok[s] = v;
                p[s] = Pin[s * N + i];
                acc[s] = (PT)0;
            }
            PT db = (PT)0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int a = q >> 1;
                const bool up = q & 1;
                const int step = axis_stride(g, a);
                const PT *Ta = axis_T(a, tx, ty, tz);
                int l;
                PT T;
                if (up) {
                    T = Ta[i];
                    l = i + step;
                } else {
                    if (i < step) continue;
                    l = i - step;
                    T = Ta[l];
                }
                if (T == (PT)0) continue;
                db += T;
                const int bit = cd.bit[a];
                if (bit < 0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) acc[s] += T * Pin[s * N + l];
                } else {
                    const int d = up ? -dpl[a] : dmin[a];  // lo_i - lo_l
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const int sd2 = ((s >> bit) & 1) + d;
                        const int s2 = (s & ~(1 << bit)) | ((sd2 & 1) << bit);
                        const PT v = Pin[s2 * N + l];
                        acc[s] += ((unsigned)sd2 <= 1u) ? T * v : (PT)0;
                    }
                }
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
            if (!(rs > (PT)0)) {
                atomicOr(flag, 2);
#pragma unroll
                for (int s = 0; s < NS; ++s) Pout[s * N + i] = p[s];
            } else {
                const PT irs = (PT)1 / rs;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const PT v = pn[s] * irs;
                    chg = fmax(chg, fabs((double)v - (double)p[s]));
                    Pout[s * N + i] = v;
                }
            }
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
    switch (s.ns) {
    case 1: hipLaunchKernelGGL((k_sweep<1, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om, bits, c.flag, check_blocks, done); break;
    case 2: hipLaunchKernelGGL((k_sweep<2, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om, bits, c.flag, check_blocks, done); break;
    case 4: hipLaunchKernelGGL((k_sweep<4, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om, bits, c.flag, check_blocks, done); break;
    default: hipLaunchKernelGGL((k_sweep<8, PT>), grid, blk, 0, c.stream, s.cart, g, tx, ty, tz, in, out, om, bits, c.flag, check_blocks, done); break;
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
constexpr int kRowChunks = 4;  // rows up to 64*kRowChunks cells

constexpr int kRowWaves = 4;

template <int NS, typename PS>
__global__ __launch_bounds__(64 * kRowWaves) void k_restrict_rows(CartDev cd, Fine g, const PS *__restrict__ P,
                                                                  const double *__restrict__ r,
                                                                  double *__restrict__ part, const int *done) {
    extern __shared__ double red[];  // [kRowWaves][nx][NS]
    if (done && *done) return;
    const int Ly = blockIdx.x, z = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int mx = cd.m[0], my = cd.m[1];
    int y0 = 0, y1 = g.ny;
    if (cd.bit[1] >= 0) {
        y0 = Ly == 0 ? 0 : cd.split[1][Ly];
        y1 = Ly + 1 < my ? cd.split[1][Ly + 1] : g.ny;
    }
    const int nch = (g.nx + 63) >> 6;
    double acc[kRowChunks][NS];
#pragma unroll
    for (int k = 0; k < kRowChunks; ++k)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[k][s] = 0.0;
    for (int y = y0 + wv; y < y1; y += kRowWaves) {
        const long row = (long)g.nx * (y + (long)g.ny * z);
#pragma unroll
        for (int k = 0; k < kRowChunks; ++k) {
            const int x = lane + 64 * k;
            if (k < nch && x < g.nx) {
                const long i = row + x;
                const double ri = r[i];
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[k][s] += ld_basis(P, (long)s * g.N + i) * ri;
            }
        }
    }
    double *mine = red + (long)wv * g.nx * NS;
#pragma unroll
    for (int k = 0; k < kRowChunks; ++k) {
        const int x = lane + 64 * k;
        if (k < nch && x < g.nx)
#pragma unroll
            for (int s = 0; s < NS; ++s) mine[x * NS + s] = acc[k][s];
    }
    __syncthreads();
    // thread (Lx, s) adds waves, then columns of dual x-interval Lx, in order
    for (int t = threadIdx.x; t < mx * NS; t += blockDim.x) {
        const int Lx = t / NS, s = t % NS;
        int x0 = 0, x1 = g.nx;
        if (cd.bit[0] >= 0) {
            x0 = Lx == 0 ? 0 : cd.split[0][Lx];
            x1 = Lx + 1 < mx ? cd.split[0][Lx + 1] : g.nx;
        }
        double tot = 0.0;
        for (int x = x0; x < x1; ++x)
            for (int w = 0; w < kRowWaves; ++w) tot += red[((long)w * g.nx + x) * NS + s];
        part[(((long)z * my + Ly) * mx + Lx) * NS + s] = tot;
    }
}

template <int NS>
__global__ __launch_bounds__(256) void k_restrict_gather(CartDev cd, Fine g, int M, const double *__restrict__ part,
                                                         double *__restrict__ d, const int *done) {
    if (done && *done) return;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= M) return;
    const int mx = cd.m[0], my = cd.m[1], mz = cd.m[2];
    const int cid = cd.present[j];
    const int J[3] = {cid % mx, (cid / mx) % my, cid / (mx * my)};
    // work items: (slot s, layer z of the dual interval J_z - s_z)
    double v = 0.0;
    for (int s = 0; s < NS; ++s) {
        int L[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[a] = J[a] - (cd.bit[a] >= 0 ? (s >> cd.bit[a]) & 1 : 0);
            if (L[a] < 0) ok = false;
        }
        if (!ok) continue;
        int z0 = 0, z1 = g.nz;
        if (cd.bit[2] >= 0) {
            z0 = L[2] == 0 ? 0 : cd.split[2][L[2]];
            z1 = L[2] + 1 < mz ? cd.split[2][L[2] + 1] : g.nz;
        }
        for (int z = z0 + lane; z < z1; z += 64) v += part[(((long)z * my + L[1]) * mx + L[0]) * NS + s];
    }
    v = wave_sum(v);
    if (lane == 0) d[j] = v;
}

// x_i += sum_s P_is p_c[block(i,s)]
template <int NS, typename PS>
__global__ __launch_bounds__(kBlock) void k_prolong(CartDev cd, Fine g, const PS *__restrict__ P,
                                                    const double *__restrict__ pc, double *__restrict__ x,
                                                    const int *done) {
    if (done && *done) return;
    const int i = xzy_cell(xcd_block() * blockDim.x + threadIdx.x, g.nx, g.ny, g.nz);
    if (i < 0 || !(g.diag[i] > 0.0)) return;
    int c[3], lo[3], nv[3];
    cell_coords(g, i, c);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = cd.lo[a][c[a]];
        nv[a] = cd.nv[a][c[a]];
    }
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (!slot_ok(cd, nv, s)) continue;
        const int blk = slot_block(cd, lo, s);
        if (blk >= 0) acc += ld_basis(P, (long)s * g.N + i) * pc[blk];
    }
    x[i] += acc;
}

template <typename PS>
static void rp_dispatch(Ctx &c, Stage &s, const PS *P, const double *r, double *x, bool restrict_, const int *done) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    if (restrict_) {
        const dim3 grid(s.cart.m[1], c.nz), blk(64 * kRowWaves), fgrid(cdiv(s.M, 4)), fblk(256);
        const size_t lds = sizeof(double) * kRowWaves * (size_t)c.nx * s.ns;
        switch (s.ns) {
        case 1:
            hipLaunchKernelGGL((k_restrict_rows<1, PS>), grid, blk, lds, c.stream, s.cart, g, P, r, s.rpart, done);
            hipLaunchKernelGGL((k_restrict_gather<1>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done);
            break;
        case 2:
            hipLaunchKernelGGL((k_restrict_rows<2, PS>), grid, blk, lds, c.stream, s.cart, g, P, r, s.rpart, done);
            hipLaunchKernelGGL((k_restrict_gather<2>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done);
            break;
        case 4:
            hipLaunchKernelGGL((k_restrict_rows<4, PS>), grid, blk, lds, c.stream, s.cart, g, P, r, s.rpart, done);
            hipLaunchKernelGGL((k_restrict_gather<4>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done);
            break;
        default:
            hipLaunchKernelGGL((k_restrict_rows<8, PS>), grid, blk, lds, c.stream, s.cart, g, P, r, s.rpart, done);
            hipLaunchKernelGGL((k_restrict_gather<8>), fgrid, fblk, 0, c.stream, s.cart, g, s.M, s.rpart, s.dvec, done);
            break;
        }
    } else {
        const dim3 grid(xcd_grid(cdiv(c.N, kBlock))), blk(kBlock);
        switch (s.ns) {
        case 1: hipLaunchKernelGGL((k_prolong<1, PS>), grid, blk, 0, c.stream, s.cart, g, P, s.pc, x, done); break;
        case 2: hipLaunchKernelGGL((k_prolong<2, PS>), grid, blk, 0, c.stream, s.cart, g, P, s.pc, x, done); break;
        case 4: hipLaunchKernelGGL((k_prolong<4, PS>), grid, blk, 0, c.stream, s.cart, g, P, s.pc, x, done); break;
        default: hipLaunchKernelGGL((k_prolong<8, PS>), grid, blk, 0, c.stream, s.cart, g, P, s.pc, x, done); break;
        }
    }
}

void launch_restrict(Ctx &c, Stage &s, const double *r, const int *done) {
    ProfScope ps(c, MSRSB_K_RESTRICT);
    if (s.kind == 2) {
        launch_xrestrict(c, s, r, done);
        return;
    }
    if (c.opt.precision == MSRSB_MIXED) rp_dispatch<uint16_t>(c, s, s.Pbf, r, nullptr, true, done);
    else rp_dispatch<double>(c, s, s.P64[s.cur], r, nullptr, true, done);
}

void launch_prolong(Ctx &c, Stage &s, double *x, const int *done) {
    ProfScope ps(c, MSRSB_K_PROLONG);
    if (s.kind == 2) {
        launch_xprolong(c, s, x, done);
        return;
    }
    if (c.opt.precision == MSRSB_MIXED) rp_dispatch<uint16_t>(c, s, s.Pbf, nullptr, x, false, done);
    else rp_dispatch<double>(c, s, s.P64[s.cur], nullptr, x, false, done);
}

// ------------------------------------------------------------ Galerkin ----
// Row j of A_c = P^T A P from the face form of A:
//   A = sum_f T_f (e_a - e_b)(e_a - e_b)^T + sum_bc T_bc e_i e_i^T, so
//   A_c[j,k] = sum_f T_f (P_aj - P_bj)(P_ak - P_bk) + sum_i bc_i P_ij P_ik.
// One 64-thread workgroup per row; each thread owns a private accumulator
// for every relative block offset (k - j in [-2,2] per split axis) and the
// private sums are added in thread order at the end, so the row does not
// depend on scheduling.
constexpr int kRapThreads = 64;

template <int NS, typename PS>
__global__ __launch_bounds__(kRapThreads) void k_rap_cart(CartDev cd, Fine g, const PS *__restrict__ P,
                                                          const double *__restrict__ bcdiag, double *__restrict__ Ac,
                                                          int Mp, int noff) {
    extern __shared__ double acc[];
    const int tid = threadIdx.x;
    for (int o = 0; o < noff; ++o) acc[o * kRapThreads + tid] = 0.0;
    const long N = g.N;
    const int j = blockIdx.x;
    const int cid = cd.present[j];
    const int J[3] = {cid % cd.m[0], (cid / cd.m[0]) % cd.m[1], cid / (cd.m[0] * cd.m[1])};
    int mul[3];
    {
        int m5 = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mul[a] = cd.bit[a] >= 0 ? m5 : 0;
            if (cd.bit[a] >= 0) m5 *= 5;
        }
    }
    int b0[3], sz[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b0[a] = max(cd.slo[a][J[a]] - 1, 0);
        sz[a] = cd.shi[a][J[a]] - b0[a] + 1;
    }
    const int vol = sz[0] * sz[1] * sz[2];
    for (int t = tid; t < vol; t += kRapThreads) {
        int ca[3];
        ca[0] = b0[0] + t % sz[0];
        const int rem = t / sz[0];
        ca[1] = b0[1] + rem % sz[1];
        ca[2] = b0[2] + rem / sz[1];
        const int ia = ca[0] + g.nx * (ca[1] + g.ny * ca[2]);
        if (!(g.diag[ia] > 0.0)) continue;
        int loA[3], nvA[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            loA[a] = cd.lo[a][ca[a]];
            nvA[a] = cd.nv[a][ca[a]];
        }
        // slot of block j in cell a (if a lies in S_j)
        bool inA = true;
        int sjA = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (cd.bit[a] < 0) continue;
            const int sd = J[a] - loA[a];
            if (sd < 0 || sd >= nvA[a]) inA = false;
            else sjA |= sd << cd.bit[a];
        }
        const double PjA = inA ? ld_basis(P, sjA * N + ia) : 0.0;
        const double bc = bcdiag[ia];
        if (bc > 0.0 && PjA != 0.0) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!slot_ok(cd, nvA, s)) continue;
                int off = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (cd.bit[a] >= 0) off += (loA[a] + ((s >> cd.bit[a]) & 1) - J[a] + 2) * mul[a];
                if ((unsigned)off < (unsigned)noff) acc[off * kRapThreads + tid] += bc * PjA * ld_basis(P, s * N + ia);
            }
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double T = (ax == 0 ? g.tx : (ax == 1 ? g.ty : g.tz))[ia];
            if (T == 0.0) continue;
            const int ib = ia + axis_stride(g, ax);
            const int loB = cd.lo[ax][ca[ax] + 1], nvB = cd.nv[ax][ca[ax] + 1];
            const int bit = cd.bit[ax];
            // value of block j at b
            double PjB = 0.0;
            {
                bool inB = true;
                int sjB = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (cd.bit[a] < 0) continue;
                    const int lb = a == ax ? loB : loA[a];
                    const int vb = a == ax ? nvB : nvA[a];
                    const int sd = J[a] - lb;
                    if (sd < 0 || sd >= vb) inB = false;
                    else sjB |= sd << cd.bit[a];
                }
                if (inB) PjB = ld_basis(P, sjB * N + ib);
            }
            const double gj = PjA - PjB;
            if (gj == 0.0) continue;
            const double Tg = T * gj;
            const int delta = loA[ax] - loB;  // 0 or -1
            // blocks held by a (with b's value of the same block)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!slot_ok(cd, nvA, s)) continue;
                double pbk = 0.0;
                if (bit >= 0) {
                    const int sd2 = ((s >> bit) & 1) + delta;
                    if (sd2 >= 0 && sd2 < nvB) pbk = ld_basis(P, ((s & ~(1 << bit)) | (sd2 << bit)) * N + ib);
                } else {
                    pbk = ld_basis(P, s * N + ib);
                }
                const double gk = ld_basis(P, s * N + ia) - pbk;
                if (gk == 0.0) continue;
                int off = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (cd.bit[a] >= 0) off += (loA[a] + ((s >> cd.bit[a]) & 1) - J[a] + 2) * mul[a];
                if ((unsigned)off < (unsigned)noff) acc[off * kRapThreads + tid] += Tg * gk;
            }
            // blocks held only by b
            if (bit >= 0) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int sdb = (s >> bit) & 1;
                    if (sdb >= nvB) continue;
                    bool okb = true;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        if (a != ax && cd.bit[a] >= 0 && ((s >> cd.bit[a]) & 1) >= nvA[a]) okb = false;
                    if (!okb) continue;
                    const int sda = sdb - delta;
                    if (sda >= 0 && sda < nvA[ax]) continue;  // also held by a: done above
                    const double gk = -ld_basis(P, s * N + ib);
                    if (gk == 0.0) continue;
                    int off = 0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        if (cd.bit[a] < 0) continue;
                        const int lb = a == ax ? loB : loA[a];
                        off += (lb + ((s >> cd.bit[a]) & 1) - J[a] + 2) * mul[a];
                    }
                    if ((unsigned)off < (unsigned)noff) acc[off * kRapThreads + tid] += Tg * gk;
                }
            }
        }
    }
    __syncthreads();
    for (int o = tid; o < noff; o += kRapThreads) {
        double sum = 0.0;
        for (int t = 0; t < kRapThreads; ++t) sum += acc[o * kRapThreads + t];
        int K[3], rem = o;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (cd.bit[a] < 0) {
                K[a] = J[a];
                continue;
            }
            K[a] = J[a] + (rem % 5) - 2;
            rem /= 5;
            if (K[a] < 0 || K[a] >= cd.m[a]) ok = false;
        }
        if (!ok) continue;
        const int kc = cd.cmap[K[0] + cd.m[0] * (K[1] + cd.m[1] * K[2])];
        if (kc >= 0) Ac[(long)j * Mp + kc] = sum;
    }
}

__global__ void k_pad_identity(double *A, int M, int Mp) {
    const int k = M + blockIdx.x * blockDim.x + threadIdx.x;
    if (k < Mp) A[(long)k * Mp + k] = 1.0;
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

void launch_symmetrize(Ctx &c, double *A, int M, int Mp) {
    hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(M, 16), cdiv(M, 16)), dim3(16, 16), 0, c.stream, A, M, Mp);
    if (Mp > M) hipLaunchKernelGGL(k_pad_identity, dim3(cdiv(Mp - M, 64)), dim3(64), 0, c.stream, A, M, Mp);
}

template <typename PS>
static void rap_dispatch(Ctx &c, Stage &s, const PS *P) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    int nbits = 0;
    for (int a = 0; a < 3; ++a) nbits += s.cart.bit[a] >= 0;
    int noff = 1;
    for (int b = 0; b < nbits; ++b) noff *= 5;
    const size_t lds = (size_t)noff * kRapThreads * sizeof(double);
    const dim3 grid(s.M), blk(kRapThreads);
    switch (s.ns) {
    case 1: hipLaunchKernelGGL((k_rap_cart<1, PS>), grid, blk, lds, c.stream, s.cart, g, P, c.bcdiag, s.Ac, s.Mp, noff); break;
    case 2: hipLaunchKernelGGL((k_rap_cart<2, PS>), grid, blk, lds, c.stream, s.cart, g, P, c.bcdiag, s.Ac, s.Mp, noff); break;
    case 4: hipLaunchKernelGGL((k_rap_cart<4, PS>), grid, blk, lds, c.stream, s.cart, g, P, c.bcdiag, s.Ac, s.Mp, noff); break;
    default: hipLaunchKernelGGL((k_rap_cart<8, PS>), grid, blk, lds, c.stream, s.cart, g, P, c.bcdiag, s.Ac, s.Mp, noff); break;
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
    launch_symmetrize(c, s.Ac, s.M, s.Mp);
}

__global__ void k_export_vals(long n, const uint16_t *__restrict__ in, double *__restrict__ out) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = (double)bf16_to_float(in[k]);
}

// Current basis values of a rectilinear stage as FP64 (device buffer).
void launch_export_cart(Ctx &c, Stage &s, double *d_vals) {
    const long n = (long)s.ns * c.N;
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_export_vals, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, s.Pbf, d_vals);
    else
        hipMemcpyAsync(d_vals, s.P64[s.cur], sizeof(double) * n, hipMemcpyDeviceToDevice, c.stream);
}

}  // namespace msrsb
