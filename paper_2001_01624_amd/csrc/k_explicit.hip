// Stages with explicit slots: static partitions whose blocks and supports
// are not boxes (the fault-cut stage: pieces of the general blocks separated
// by faults, paper section "Multiscale methods", partition type "Static").
//
// Layout: slot-major tables sb[s*N + i] = block held by slot s of cell i
// (ascending, -1 past the cell's last slot) and basis values P[s*N + i];
// per-block support lists (CSR over cells in ascending order, with the slot
// index of the block in that cell) for restriction and the Galerkin rows.
#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

template <typename PT>
__global__ void k_xinit(int N, int ns, const int32_t *__restrict__ sb, const int32_t *__restrict__ pblock,
                        PT *__restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int own = pblock[i];
    for (int s = 0; s < ns; ++s) P[(long)s * N + i] = (own >= 0 && sb[(long)s * N + i] == own) ? (PT)1 : (PT)0;
}

// Neighbour slot maps (once per stage; the structure does not change): the
// slot count of every cell, and for face q (axis q/2, +/- as q%2) and slot s
// of cell i the slot of the same block in the face neighbour's list, or none:
// byte map[(q ns + s) N + i] (255: none), or with at most kXNibSlots slots
// nibble s of the word nib[q N + i] (15: none).
__global__ void k_xmap_build(Fine g, int ns, const int32_t *__restrict__ sb, uint8_t *__restrict__ cnt,
                             uint8_t *__restrict__ map, uint64_t *__restrict__ nib) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    const long N = g.N;
    int c = 0;
    for (int s = 0; s < ns; ++s)
        if (sb[s * N + i] >= 0) c = s + 1;
    cnt[i] = (uint8_t)c;
    for (int q = 0; q < 6; ++q) {
        const int a = q >> 1;
        const int step = a == 0 ? 1 : (a == 1 ? g.nx : g.nxy);
        const int l = (q & 1) ? i + step : i - step;
        const bool in = (q & 1) ? l < g.N : i >= step;
        uint64_t w = 0;
        for (int s = 0; s < ns; ++s) {
            int u = 255;
            if (in && s < c) {
                const int bo = sb[s * N + i];
                for (int t = 0; t < ns; ++t) {
                    const int bl = sb[t * N + l];
                    if (bl < 0) break;
                    if (bl == bo) {
                        u = t;
                        break;
                    }
                }
            }
            if (nib) w |= (uint64_t)(u == 255 ? 15 : u) << (4 * s);
            else map[(size_t)(q * ns + s) * N + i] = (uint8_t)u;
        }
        if (nib) {
            for (int s = ns; s < 16; ++s) w |= (uint64_t)15 << (4 * s);
            nib[(size_t)q * N + i] = w;
        }
    }
}

void launch_xmap_build(Ctx &c, Stage &s) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    hipLaunchKernelGGL(k_xmap_build, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, s.ns, s.xsb, s.xcnt,
                       s.xnmap, s.xnib);
}

// One restricted-smoothing sweep (same definition as the rectilinear one):
// the neighbour's value of block j is read at the slot the neighbour slot map
// gives (each face adds to a slot at most once, faces in a fixed order).
// NIB: the packed map, one word per face, all six loaded before the first
// gather; else the byte map.
template <int NSX, typename PT, bool NIB>
__global__ __launch_bounds__(kBlock) void k_xsweep(Fine g, int ns, const uint8_t *__restrict__ cntv,
                                                   const uint8_t *__restrict__ nmap, const uint64_t *__restrict__ nib,
                                                   const PT *__restrict__ tx, const PT *__restrict__ ty,
                                                   const PT *__restrict__ tz, const PT *__restrict__ Pin,
                                                   PT *__restrict__ Pout, PT omega, double *__restrict__ part,
                                                   int *flag, const int *done) {
    __shared__ double lds[kBlock / 64];
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double chg = 0.0;
    if (i < g.N) {
        const long N = g.N;
        const int cn = cntv[i];
        PT p[NSX], acc[NSX];
#pragma unroll
        for (int s = 0; s < NSX; ++s) {
            p[s] = s < ns ? Pin[s * N + i] : (PT)0;
            acc[s] = (PT)0;
        }
        if (!(g.diag[i] > 0.0)) {
            for (int s = 0; s < ns; ++s) Pout[s * N + i] = (PT)0;
        } else {
            PT db = (PT)0;
            uint64_t wq[6];
            if (NIB) {
#pragma unroll
                for (int q = 0; q < 6; ++q) wq[q] = nib[(size_t)q * N + i];
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int a = q >> 1;
                const bool up = q & 1;
                const int step = a == 0 ? 1 : (a == 1 ? g.nx : g.nxy);
                const PT *Ta = a == 0 ? tx : (a == 1 ? ty : tz);
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
                if (NIB) {
#pragma unroll
                    for (int s = 0; s < NSX; ++s) {
                        const int u = (int)(wq[q] >> (4 * s)) & 15;
                        if (s < cn && u != 15) acc[s] += T * Pin[u * N + l];
                    }
                } else {
                    const uint8_t *mq = nmap + (size_t)q * ns * N + i;
#pragma unroll
                    for (int s = 0; s < NSX; ++s) {
                        if (s >= cn) break;
                        const int u = mq[(size_t)s * N];
                        if (u != 255) acc[s] += T * Pin[u * N + l];
                    }
                }
            }
            const PT idb = db > (PT)0 ? (PT)1 / db : (PT)0;
            PT pn[NSX];
            PT rs = (PT)0;
#pragma unroll
            for (int s = 0; s < NSX; ++s) {
                PT v = (PT)0;
                if (s < cn) v = db > (PT)0 ? p[s] - omega * (p[s] - acc[s] * idb) : p[s];
                pn[s] = v;
                rs += v;
            }
            if (!(rs > (PT)0)) {
                atomicOr(flag, 2);
                for (int s = 0; s < ns; ++s) Pout[s * N + i] = Pin[s * N + i];
            } else {
                const PT irs = (PT)1 / rs;
#pragma unroll
                for (int s = 0; s < NSX; ++s) {
                    if (s >= ns) break;
                    const PT v = pn[s] * irs;
                    chg = fmax(chg, fabs((double)v - (double)p[s]));
                    Pout[s * N + i] = v;
                }
            }
        }
    }
    const double m = block_max(chg, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Returns the number of per-workgroup maxima written to c.partial.
template <typename PT>
static int xsweep_dispatch(Ctx &c, Stage &s, const PT *tx, const PT *ty, const PT *tz, const PT *in, PT *out) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    const dim3 grid(cdiv(c.N, kBlock)), blk(kBlock);
    const PT om = (PT)c.opt.omega;
    const int *done = &c.status->done;
    double *part = c.partial;
#define MSRSB_XSW(NSX, NIB)                                                                                    \
    hipLaunchKernelGGL((k_xsweep<NSX, PT, NIB>), grid, blk, 0, c.stream, g, s.ns, s.xcnt, s.xnmap, s.xnib, tx, ty, \
                       tz, in, out, om, part, c.flag, done)
    if (s.xnib) {
        if (s.ns <= 8) MSRSB_XSW(8, true);
        else MSRSB_XSW(16, true);
    } else {
        if (s.ns <= 16) MSRSB_XSW(16, false);
        else MSRSB_XSW(kMaxXSlots, false);
    }
#undef MSRSB_XSW
    return (int)grid.x;
}

void launch_xinit(Ctx &c, Stage &s) {
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_xinit<float>, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, s.ns, s.xsb,
                           s.xpblock, s.P32[0]);
    else
        hipLaunchKernelGGL(k_xinit<double>, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, s.ns, s.xsb,
                           s.xpblock, s.P64[0]);
}

int launch_xsweep(Ctx &c, Stage &s, int in, int out) {
    if (c.opt.precision == MSRSB_MIXED)
        return xsweep_dispatch<float>(c, s, c.tx32, c.ty32, c.tz32, s.P32[in], s.P32[out]);
    return xsweep_dispatch<double>(c, s, c.tx, c.ty, c.tz, s.P64[in], s.P64[out]);
}

// The basis value of every support-list entry in list order: Pl[k] =
// P[slot[k] N + cell[k]] (after each run of sweeps), so that the
// restriction reads the values of a block contiguously.
template <typename PS>
__global__ void k_xlist(int n, long N, const int32_t *__restrict__ cell, const uint8_t *__restrict__ slot,
                        const PS *__restrict__ P, PS *__restrict__ Pl) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) Pl[k] = P[(long)slot[k] * N + cell[k]];
}

void launch_xlist(Ctx &c, Stage &s) {
    const int n = s.nxent;
    if (n <= 0) return;
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_xlist<uint16_t>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, (long)c.N,
                           s.xcell, s.xslot, s.Pbf, (uint16_t *)s.xplist);
    else
        hipLaunchKernelGGL(k_xlist<double>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, (long)c.N, s.xcell,
                           s.xslot, s.P64[s.cur], (double *)s.xplist);
}

// d_j = sum over the support list of block j of P_ij r_i, in two fixed-order
// passes: one workgroup per chunk of at most kXChunk list entries (a block
// whose support spans the grid is spread over many workgroups), then one
// thread per block adds its chunks in order.  The basis values come from the
// list-ordered copy (contiguous per block).
template <typename PS>
__global__ __launch_bounds__(kBlock) void k_xrestrict(const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ cblk,
                                                      const int32_t *__restrict__ cfirst,
                                                      const int32_t *__restrict__ cell, const PS *__restrict__ Pl,
                                                      const double *__restrict__ r, double *__restrict__ part,
                                                      const int *done) {
    __shared__ double lds[kBlock / 64];
    if (done && *done) return;
    const int ch = blockIdx.x, j = cblk[ch];
    const int k0 = ptr[j] + (ch - cfirst[j]) * kXChunk, k1 = min(k0 + kXChunk, ptr[j + 1]);
    double acc = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) acc += ld_basis(Pl, (long)k) * r[cell[k]];
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[ch] = s;
}

__global__ void k_xrestrict_finish(int M, const int32_t *__restrict__ cfirst, const double *__restrict__ part,
                                   double *__restrict__ d, const int *done) {
    if (done && *done) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double s = 0.0;
    for (int c = cfirst[j]; c < cfirst[j + 1]; ++c) s += part[c];
    d[j] = s;
}

template <typename PS>
__global__ __launch_bounds__(kBlock) void k_xprolong(int N, int ns, const int32_t *__restrict__ sb,
                                                     const PS *__restrict__ P, const double *__restrict__ pc,
                                                     double *__restrict__ x, const int *done) {
    if (done && *done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int s = 0; s < ns; ++s) {
        const int b = sb[(long)s * N + i];
        if (b < 0) break;
        acc += ld_basis(P, (long)s * N + i) * pc[b];
    }
    x[i] += acc;
}

void launch_xrestrict(Ctx &c, Stage &s, const double *r, const int *done) {
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_xrestrict<uint16_t>, dim3(s.nxch), dim3(kBlock), 0, c.stream, s.xptr, s.xcblk, s.xcfirst,
                           s.xcell, (const uint16_t *)s.xplist, r, s.xpart, done);
    else
        hipLaunchKernelGGL(k_xrestrict<double>, dim3(s.nxch), dim3(kBlock), 0, c.stream, s.xptr, s.xcblk, s.xcfirst,
                           s.xcell, (const double *)s.xplist, r, s.xpart, done);
    hipLaunchKernelGGL(k_xrestrict_finish, dim3(cdiv(s.M, kBlock)), dim3(kBlock), 0, c.stream, s.M, s.xcfirst, s.xpart,
                       s.dvec, done);
}

void launch_xprolong(Ctx &c, Stage &s, double *x, const int *done) {
    if (c.opt.precision == MSRSB_MIXED)
        hipLaunchKernelGGL(k_xprolong<uint16_t>, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, s.ns, s.xsb,
                           s.Pbf, s.pc, x, done);
    else
        hipLaunchKernelGGL(k_xprolong<double>, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, c.N, s.ns, s.xsb,
                           s.P64[s.cur], s.pc, x, done);
}

// Row j of A_c = P^T A P from the face form (see the rectilinear kernel):
// one wavefront walks the support list of block j; every face (a, b) with
// P_aj - P_bj != 0 is taken once (from a, and from b only when a is not in
// the support), and its contributions T g_j g_k are summed per column k by
// fixed-shape wave reductions committed in a fixed order.  A lane first adds
// up its cell's contributions to the columns of the cell's own slots (the
// boundary term and the six faces), so those take one reduction per slot
// and entry rather than one per face; columns that only a neighbour holds
// are committed face by face.
// One wavefront per chunk of `chunk` entries of a block's list; a
// block with several chunks sums each into a partial row of its own, added
// in chunk order by k_xrap_finish.
// LDSROW: the row is accumulated in LDS (Mp doubles) and stored once at the
// end; otherwise in its global row (rows too long for LDS).  The additions
// are the same, in the same order, either way.
template <int NSX, typename PS, bool LDSROW>
__global__ __launch_bounds__(64) void k_xrap(Fine g, int ns, const int32_t *__restrict__ sb,
                                             const int32_t *__restrict__ ptr, const int32_t *__restrict__ rcblk,
                                             const int32_t *__restrict__ rcfirst, const int32_t *__restrict__ rrow,
                                             const int32_t *__restrict__ cell,
                                             const PS *__restrict__ Pl, const PS *__restrict__ P,
                                             const double *__restrict__ bcdiag, double *__restrict__ Ac,
                                             double *__restrict__ rpart, int Mp, int chunk) {
    extern __shared__ double srow[];
    const int ch = blockIdx.x, j = rcblk[ch], lane = threadIdx.x;
    const long N = g.N;
    double *grow = rrow[ch] >= 0 ? rpart + (long)rrow[ch] * Mp : Ac + (long)j * Mp;
    double *row = LDSROW ? srow : grow;
    if (LDSROW) {
        for (int k = lane; k < Mp; k += 64) srow[k] = 0.0;
        __syncthreads();
    }
    const int k0 = ptr[j] + (ch - rcfirst[j]) * chunk, k1 = min(k0 + chunk, ptr[j + 1]);
    // each wavefront sums one row's contributions per column k with a
    // ballot over the lanes' columns and a wave sum per distinct column
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
        const int a = live ? cell[k] : 0;
        // a's slot list (blocks ascending, -1 past the last slot) and values,
        // loaded once for the six faces
        int la[NSX];
        double pa[NSX];
#pragma unroll
        for (int t = 0; t < NSX; ++t) {
            la[t] = t < ns ? sb[(long)t * N + a] : -1;
            pa[t] = t < ns ? ld_basis(P, (long)t * N + a) : 0.0;
        }
        const double Paj = live ? ld_basis(Pl, (long)k) : 0.0;
        // the lane's contributions to the columns of a's own slots, summed
        // over the boundary term and the six faces before one commit per slot
        double acc[NSX];
        // boundary term: bc_a P_aj P_ak over a's slots
        {
            const double bc = live ? bcdiag[a] : 0.0;
#pragma unroll
            for (int t = 0; t < NSX; ++t) acc[t] = live && bc > 0.0 && la[t] >= 0 ? bc * Paj * pa[t] : 0.0;
        }
        for (int q = 0; q < 6; ++q) {
            const int ax = q >> 1;
            const bool up = q & 1;
            const int step = ax == 0 ? 1 : (ax == 1 ? g.nx : g.nxy);
            const double *Ta = ax == 0 ? g.tx : (ax == 1 ? g.ty : g.tz);
            int b = -1;
            double T = 0.0;
            if (live) {
                if (up) {
                    T = Ta[a];
                    b = a + step;
                } else if (a >= step) {
                    b = a - step;
                    T = Ta[b];
                }
            }
            // b's slot list and values (b = a where there is no face: unused)
            const int bb = T != 0.0 ? b : a;
            int lb[NSX];
            double pb[NSX];
#pragma unroll
            for (int t = 0; t < NSX; ++t) {
                lb[t] = t < ns ? sb[(long)t * N + bb] : -1;
                pb[t] = t < ns ? ld_basis(P, (long)t * N + bb) : 0.0;
            }
            // value of block j at b, and whether b lies in the support
            double Pbj = 0.0;
            bool bin = false;
            if (T != 0.0) {
#pragma unroll
                for (int t = 0; t < NSX; ++t)
                    if (lb[t] == j) {
                        Pbj = pb[t];
                        bin = true;
                    }
            }
            // each face once: from a, unless b is also in the support and b < a
            const bool take = T != 0.0 && !(bin && b < a);
            const double gj = take ? Paj - Pbj : 0.0;
            const bool act = take && gj != 0.0;
            // columns: blocks of a (with b's value of the same block) into the
            // lane's sums, then blocks only of b
#pragma unroll
            for (int t = 0; t < NSX; ++t) {
                if (act && la[t] >= 0) {
                    double po = 0.0;
#pragma unroll
                    for (int u = 0; u < NSX; ++u)
                        if (lb[u] == la[t]) po = pb[u];
                    acc[t] += T * gj * (pa[t] - po);
                }
            }
#pragma unroll
            for (int t = 0; t < NSX; ++t) {
                if (t >= ns) break;
                int kb = -1;
                double v = 0.0;
                if (act && lb[t] >= 0) {
                    bool shared = false;
#pragma unroll
                    for (int u = 0; u < NSX; ++u)
                        if (la[u] == lb[t]) shared = true;
                    if (!shared) {  // blocks of both were taken with a's slots
                        kb = lb[t];
                        v = -T * gj * pb[t];
                    }
                }
                commit(kb, v);
            }
        }
#pragma unroll
        for (int t = 0; t < NSX; ++t) {
            if (t >= ns) break;
            commit(live && la[t] >= 0 ? la[t] : -1, acc[t]);
        }
    }
    if (LDSROW) {
        __syncthreads();
        for (int k = lane; k < Mp; k += 64) grow[k] = srow[k];
    }
}

// Rows of blocks with several chunks: A_c[j][k] = sum of the chunks' partial
// rows, in chunk order (one thread per column).
__global__ void k_xrap_finish(int M, int Mp, const int32_t *__restrict__ rcfirst, const int32_t *__restrict__ rrow,
                              const double *__restrict__ rpart, double *__restrict__ Ac) {
    const int j = blockIdx.y;
    const int c0 = rcfirst[j], c1 = rcfirst[j + 1];
    if (c1 - c0 < 2) return;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < M; k += gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int c = c0; c < c1; ++c) v += rpart[(long)rrow[c] * Mp + k];
        Ac[(long)j * Mp + k] = v;
    }
}

void launch_partial_rows_finish(Ctx &c, int M, int Mp, const int32_t *rcfirst, const int32_t *rrow,
                                const double *rpart, double *A) {
    hipLaunchKernelGGL(k_xrap_finish, dim3(cdiv(M, kBlock), M), dim3(kBlock), 0, c.stream, M, Mp, rcfirst, rrow, rpart,
                       A);
}

void launch_symmetrize(Ctx &c, double *A, int M, int Mp);

constexpr size_t kXRapLds = 65536;  // longest row accumulated in LDS: 8192 coarse columns

void launch_xrap(Ctx &c, Stage &s) {
    Fine g{c.nx, c.ny, c.nz, c.nx * c.ny, c.N, c.tx, c.ty, c.tz, c.diag};
    hipMemsetAsync(s.Ac, 0, sizeof(double) * (size_t)s.Mp * s.Mp, c.stream);
    if (s.nxrrow > 0) hipMemsetAsync(s.xrpart, 0, sizeof(double) * (size_t)s.nxrrow * s.Mp, c.stream);
    const size_t lds = sizeof(double) * (size_t)s.Mp;
#define MSRSB_XRAP1(NSX, PS, PP, L)                                                                             \
    hipLaunchKernelGGL((k_xrap<NSX, PS, L>), dim3(s.nxrch), dim3(64), L ? lds : 0, c.stream, g, s.ns, s.xsb,     \
                       s.xptr, s.xrcblk, s.xrcfirst, s.xrrow, s.xcell, (const PS *)s.xplist, PP, c.bcdiag, s.Ac,    \
                       s.xrpart, s.Mp, s.xrchunk)
#define MSRSB_XRAP(PS, PP, L)                                \
    {                                                        \
        if (s.ns <= 8) MSRSB_XRAP1(8, PS, PP, L);            \
        else if (s.ns <= 16) MSRSB_XRAP1(16, PS, PP, L);     \
        else MSRSB_XRAP1(kMaxXSlots, PS, PP, L);             \
    }
    const bool mixed = c.opt.precision == MSRSB_MIXED;
    if (lds <= kXRapLds) {
        if (mixed) MSRSB_XRAP(uint16_t, s.Pbf, true)
        else MSRSB_XRAP(double, s.P64[s.cur], true)
    } else {
        if (mixed) MSRSB_XRAP(uint16_t, s.Pbf, false)
        else MSRSB_XRAP(double, s.P64[s.cur], false)
    }
#undef MSRSB_XRAP
#undef MSRSB_XRAP1
    if (s.nxrrow > 0)
        hipLaunchKernelGGL(k_xrap_finish, dim3(cdiv(s.M, kBlock), s.M), dim3(kBlock), 0, c.stream, s.M, s.Mp,
                           s.xrcfirst, s.xrrow, s.xrpart, s.Ac);
    launch_symmetrize(c, s.Ac, s.M, s.Mp);
}

}  // namespace msrsb
