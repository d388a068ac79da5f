// Coarse factorisation and solve (section "Computational efficiency":
// inverting the coarse matrix by direct Gaussian elimination).
//
// A_c is SPD, so Gauss-Jordan elimination needs no pivoting: sweeping the
// pivots in order turns A_c into A_c^{-1} in place.  Each pivot of the sweep
// is a diagonal entry of a Schur complement of A_c (the square of the
// corresponding Cholesky diagonal), so a non-positive pivot means A_c is
// not SPD and is reported.  The sweep is blocked by T = kTile columns; for
// pivot block K with D = A[K,K]:
//   A[K,J] <- D^{-1} A[K,J]                      (row panel, J != K)
//   A[I,J] <- A[I,J] - A[I,K] (D^{-1} A[K,J])     (I != K, J != K)
//   A[I,K] <- -A[I,K] D^{-1},  A[K,K] <- D^{-1}.
// D^{-1} of the next pivot block is formed by the workgroup that updates
// that block, inside the update of the current step, so only the first
// block inversion is on its own on the critical path.  The tile products of
// the panels and the trailing update run on the FP64 matrix instructions.
// Each cycle then applies the inverse by a GEMV (one workgroup per row).
#include "batch.h"
#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

constexpr int T_ = kTile;     // 64
constexpr int kGJThreads = 256;
constexpr int kLd = T_ + 1;   // LDS row pitch (bank spread)

// In-place inversion of the T x T (64) block M in LDS by one workgroup of
// 256 threads: Gauss-Jordan blocked by 16 pivots.  For sub-block s (rows and
// columns o..o+15, o = 16 s):
//   1. D = M[s,s] is inverted element-wise by one wavefront (pivot row and
//      column by lane shuffles, no workgroup barrier per pivot);
//   2. W[s,:] = D^{-1} M[s,:] off the block, W[s,s] = D^{-1}; Cb = M[:,s];
//   3. M[i,j] <- M[i,j] - Cb[i,:] W[:,j] for rows i off the block (with 0 in
//      place of M[i,j] on the block columns), M[s,:] <- W[s,:].
// W is 16 x kLd and Cb 64 x 17 doubles of LDS scratch.
__device__ inline void gj_invert_lds(double (*M)[kLd], double (*W)[kLd], double (*Cb)[17], int *flag, bool general) {
    const int t = threadIdx.x;
#pragma unroll 1
    for (int sb = 0; sb < T_ / 16; ++sb) {
        const int o = 16 * sb;
        // 1. element-wise inverse of the 16 x 16 diagonal sub-block by the
        //    first wavefront: lane l owns row l/4, columns 4(l%4)..+3, and
        //    takes the pivot row and column from the owning lanes by shuffles
        if (t < 64) {
            const int r = t >> 2, cg = t & 3;
            double x[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) x[b] = M[o + r][o + 4 * cg + b];
#pragma unroll 4
            for (int k = 0; k < 16; ++k) {  // k & 3 is fixed within the unrolled body
                const double p = __shfl(x[k & 3], 4 * k + (k >> 2), 64);
                // SPD: every pivot is positive; a general matrix needs non-zero pivots
                const bool ok = general ? (p != 0.0 && isfinite(p)) : p > 0.0;
                if (t == 0 && !ok) atomicOr(flag, 1);
                const double ip = ok ? 1.0 / p : 0.0;
                const double dik = __shfl(x[k & 3], 4 * r + (k >> 2), 64);
                double rowk[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) rowk[b] = __shfl(x[b], 4 * k + cg, 64);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int c = 4 * cg + b;
                    const double rk = rowk[b] * ip;
                    double nx = c == k ? -dik * ip : x[b] - dik * rk;
                    if (r == k) nx = c == k ? ip : rk;
                    x[b] = nx;
                }
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) M[o + r][o + 4 * cg + b] = x[b];
        }
        __syncthreads();
        // 2. row panel W = D^{-1} M[s,:] (W[s,s] = D^{-1}), column copy Cb
        {
            const int r = t >> 4, j4 = (t & 15) * 4;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int q = 0; q < 16; ++q) {
                const double d = M[o + r][o + q];
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[b] += d * M[o + q][j4 + b];
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = j4 + b;
                W[r][j] = (j >= o && j < o + 16) ? M[o + r][j] : acc[b];
            }
            for (int e = t; e < T_ * 16; e += blockDim.x) Cb[e >> 4][e & 15] = M[e >> 4][o + (e & 15)];
            __syncthreads();
        }
        // 3. rows off the block: 3 rows x 4 columns per thread
        {
            const int g = t >> 4, j4 = (t & 15) * 4;
            double acc[3][4];
            int ri[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int rr = 3 * g + a;  // 0..47
                ri[a] = rr < o ? rr : rr + 16;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int j = j4 + b;
                    acc[a][b] = (j >= o && j < o + 16) ? 0.0 : M[ri[a]][j];
                }
            }
#pragma unroll 4
            for (int q = 0; q < 16; ++q) {
                double w[4], cv[3];
#pragma unroll
                for (int b = 0; b < 4; ++b) w[b] = W[q][j4 + b];
#pragma unroll
                for (int a = 0; a < 3; ++a) cv[a] = Cb[ri[a]][q];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] -= cv[a] * w[b];
            }
            __syncthreads();  // every read of M's old block column done
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) M[ri[a]][j4 + b] = acc[a][b];
            for (int e = t; e < 16 * T_; e += blockDim.x) M[o + (e >> 6)][e & 63] = W[e >> 6][e & 63];
            __syncthreads();
        }
    }
}

// acc = X * Y for T x T tiles staged in LDS with the FP64 16x16x4 matrix
// instruction: wavefront w of the four computes the 32 x 32 quadrant at rows
// 32 (w / 2), columns 32 (w % 2) as 2 x 2 blocks of 16 x 16, summing k in 16
// steps of 4.  Lane l supplies A[i][k] at i = l % 16, k = l / 16 and B[k][j]
// at j = l % 16, k = l / 16, and holds entry r of a block's result at row
// 4 r + l / 16, column l % 16 (mm_row / mm_col below).  One matrix
// instruction does 16 x 16 x 4 products from two operands per lane, so the
// LDS traffic per product is an eighth of the 4 x 4 register tiles'.
typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ inline int mm_row(int bi, int r) { return 32 * ((threadIdx.x >> 6) >> 1) + 16 * bi + 4 * r + ((threadIdx.x & 63) >> 4); }
__device__ inline int mm_col(int bj) { return 32 * ((threadIdx.x >> 6) & 1) + 16 * bj + (threadIdx.x & 15); }

__device__ inline void tile_mm_mfma(const double (*X)[kLd], const double (*Y)[kLd], dvec4 (&acc)[2][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dvec4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < T_; kk += 4) {
        const double a0 = X[r0 + li][kk + lk], a1 = X[r0 + 16 + li][kk + lk];
        const double b0 = Y[kk + lk][c0 + li], b1 = Y[kk + lk][c0 + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// T x T tile from global (leading dimension ld) into LDS: all 16 loads of a
// thread first, then the stores (256 threads).
__device__ inline void load_tile(double (*S)[kLd], const double *__restrict__ src, long ld) {
    double r[T_ * T_ / kGJThreads];
#pragma unroll
    for (int q = 0; q < T_ * T_ / kGJThreads; ++q) {
        const int e = threadIdx.x + kGJThreads * q;
        r[q] = src[(long)(e / T_) * ld + e % T_];
    }
#pragma unroll
    for (int q = 0; q < T_ * T_ / kGJThreads; ++q) {
        const int e = threadIdx.x + kGJThreads * q;
        S[e / T_][e % T_] = r[q];
    }
}

__device__ __forceinline__ void gj_diag_body(const double *__restrict__ A, int Mp, int k0, double *__restrict__ Dinv,
                                             int *flag, bool general) {
    __shared__ double Ms[T_][kLd], Ws[16][kLd], Cb[T_][17];
    load_tile(Ms, A + (long)k0 * Mp + k0, Mp);
    __syncthreads();
    gj_invert_lds(Ms, Ws, Cb, flag, general);
    for (int e = threadIdx.x; e < T_ * T_; e += blockDim.x) Dinv[e] = Ms[e / T_][e % T_];
}

__global__ __launch_bounds__(kGJThreads) void k_gj_diag(const double *__restrict__ A, int Mp, int k0,
                                                        double *__restrict__ Dinv, int *flag, bool general) {
    gj_diag_body(A, Mp, k0, Dinv, flag, general);
}

// Workgroup t: row panel A[K,t] <- D^{-1} A[K,t] and a copy C[t] = A[t,K]
// of the column panel (taken before the update).
__device__ __forceinline__ void gj_panel_body(int bid, int nblk, double *__restrict__ A, int Mp, int K,
                                              const double *__restrict__ Dinv, double *__restrict__ C) {
    __shared__ double Ds[T_][kLd], Bs[T_][kLd];
    const int t = bid;
    if (t == K) return;
    const int k0 = K * T_, c0 = t * T_;
    load_tile(Ds, Dinv, T_);
    load_tile(Bs, A + (long)k0 * Mp + c0, Mp);
    {
        double r[T_ * T_ / kGJThreads];
#pragma unroll
        for (int q = 0; q < T_ * T_ / kGJThreads; ++q) {
            const int e = threadIdx.x + kGJThreads * q;
            r[q] = A[(long)(c0 + e / T_) * Mp + k0 + e % T_];
        }
#pragma unroll
        for (int q = 0; q < T_ * T_ / kGJThreads; ++q) {
            const int e = threadIdx.x + kGJThreads * q;
            C[(long)(c0 + e / T_) * T_ + e % T_] = r[q];
        }
    }
    __syncthreads();
    dvec4 acc[2][2];
    tile_mm_mfma(Ds, Bs, acc);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) A[(long)(k0 + mm_row(bi, r)) * Mp + c0 + mm_col(bj)] = acc[bi][bj][r];
}

__global__ __launch_bounds__(kGJThreads) void k_gj_panel(double *__restrict__ A, int Mp, int K,
                                                         const double *__restrict__ Dinv, double *__restrict__ C) {
    gj_panel_body(blockIdx.x, gridDim.x, A, Mp, K, Dinv, C);
}

// Trailing update of step K over all tiles (I, J).  Workgroup 0 takes tile
// (K+1, K+1) and, after its update, inverts it into Dnext.
__device__ __forceinline__ void gj_update_body(int bid, int nblk, double *__restrict__ A, int Mp, int K, int nt,
                                               const double *__restrict__ Dinv, const double *__restrict__ C,
                                               double *__restrict__ Dnext, int *flag, bool general) {
    __shared__ double Cs[T_][kLd], Bs[T_][kLd];
    // tile of this workgroup: 0 -> (K+1, K+1) (when it exists), then the rest
    const int L = K + 1 < nt ? K + 1 : -1;
    int b = bid, I, J;
    if (L >= 0) {
        if (b == 0) {
            I = J = L;
        } else {
            const int lin = b - 1 + (b - 1 >= L * nt + L ? 1 : 0);  // skip (L, L)
            I = lin / nt;
            J = lin % nt;
        }
    } else {
        I = b / nt;
        J = b % nt;
    }
    const int r0 = I * T_, c0 = J * T_, k0 = K * T_;
    if (I == K) {
        if (J == K) {
            double r[T_ * T_ / kGJThreads];
#pragma unroll
            for (int q = 0; q < T_ * T_ / kGJThreads; ++q) r[q] = Dinv[threadIdx.x + kGJThreads * q];
#pragma unroll
            for (int q = 0; q < T_ * T_ / kGJThreads; ++q) {
                const int e = threadIdx.x + kGJThreads * q;
                A[(long)(k0 + e / T_) * Mp + k0 + e % T_] = r[q];
            }
        }
        return;
    }
    double old[2][2][4];
    if (J != K) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) old[bi][bj][r] = A[(long)(r0 + mm_row(bi, r)) * Mp + c0 + mm_col(bj)];
    }
    load_tile(Cs, C + (long)r0 * T_, T_);
    if (J == K) load_tile(Bs, Dinv, T_);
    else load_tile(Bs, A + (long)k0 * Mp + c0, Mp);
    __syncthreads();
    dvec4 acc[2][2];
    tile_mm_mfma(Cs, Bs, acc);
    if (J == K) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) A[(long)(r0 + mm_row(bi, r)) * Mp + c0 + mm_col(bj)] = -acc[bi][bj][r];
        return;
    }
    double nv[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                nv[bi][bj][r] = old[bi][bj][r] - acc[bi][bj][r];
                if (I != L || J != L) A[(long)(r0 + mm_row(bi, r)) * Mp + c0 + mm_col(bj)] = nv[bi][bj][r];
            }
    if (I == L && J == L) {
        // the next pivot block: stage the updated tile and invert it
        __syncthreads();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) Cs[mm_row(bi, r)][mm_col(bj)] = nv[bi][bj][r];
        __syncthreads();
        gj_invert_lds(Cs, Bs, reinterpret_cast<double (*)[17]>(&Bs[16][0]), flag, general);
        for (int e = threadIdx.x; e < T_ * T_; e += blockDim.x) Dnext[e] = Cs[e / T_][e % T_];
    }
}

__global__ __launch_bounds__(kGJThreads) void k_gj_update(double *__restrict__ A, int Mp, int K, int nt,
                                                          const double *__restrict__ Dinv,
                                                          const double *__restrict__ C, double *__restrict__ Dnext,
                                                          int *flag, bool general) {
    gj_update_body(blockIdx.x, gridDim.x, A, Mp, K, nt, Dinv, C, Dnext, flag, general);
}

void launch_coarse_inverse(Ctx &c, Stage &s) { launch_coarse_inverse_of(c, s.Ac, s.Ainv, s.Mp, false); }

// Ainv = A^{-1} for a padded Mp x Mp matrix (Mp a multiple of kTile).  Without
// pivoting: an SPD matrix has positive pivots (a non-positive one is flagged);
// a general one (general = true) needs non-zero leading principal minors.
void launch_coarse_inverse_of(Ctx &c, const double *Asrc, double *A, int Mp, bool general) {
    ProfScope ps(c, MSRSB_K_INVERSE);
    const int nt = Mp / T_;
    hipMemcpyAsync(A, Asrc, sizeof(double) * (size_t)Mp * Mp, hipMemcpyDeviceToDevice, c.stream);
    double *C = c.cbuf;                                       // Mp * kTile doubles
    double *Dbuf[2] = {c.cbuf + (size_t)c.cbuf_n * T_, c.cbuf + (size_t)(c.cbuf_n + T_) * T_};
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(kGJThreads), 0, c.stream, A, Mp, 0, Dbuf[0], c.flag, general);
    for (int K = 0; K < nt; ++K) {
        double *D = Dbuf[K & 1], *Dn = Dbuf[(K + 1) & 1];
        hipLaunchKernelGGL(k_gj_panel, dim3(nt), dim3(kGJThreads), 0, c.stream, A, Mp, K, D, C);
        hipLaunchKernelGGL(k_gj_update, dim3(nt * nt), dim3(kGJThreads), 0, c.stream, A, Mp, K, nt, D, C, Dn,
                           c.flag, general);
    }
}

// p_c = A_c^{-1} d: one workgroup per row.  Thread t adds the entries
// t, t + 256, ... of the row in order, then a fixed-order workgroup sum.  The
// entries of a thread are taken NPT at a time with every load issued before
// the first product (indices past the row clamped to an entry of the row and
// their terms multiplied by zero), so a row of up to 256 NPT entries costs one
// memory round trip; a loop with a run-time trip count below its unroll
// factor would wait on each load in turn.  Row j is stored at y[map[j]] when
// a map is given.
constexpr int kGemvThreads = 256;

template <int NPT>
__device__ __forceinline__ void gemv_body(int bid, int nblk, const double *__restrict__ A, int M, int Mp,
                                          const double *__restrict__ d, double *__restrict__ y,
                                          const int32_t *__restrict__ map, const int *done) {
    __shared__ double lds[kGemvThreads / 64];
    if (done && *done) return;
    const int row = bid;
    const double *a = A + (long)row * Mp;
    double s = 0.0;
    for (int k0 = threadIdx.x; k0 < M; k0 += NPT * kGemvThreads) {
        double av[NPT], dv[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int k = k0 + j * kGemvThreads;
            const int kc = k < M ? k : k0;
            av[j] = a[kc];
            dv[j] = d[kc];
        }
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const double m = k0 + j * kGemvThreads < M ? 1.0 : 0.0;
            s = fma(av[j], dv[j] * m, s);
        }
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) y[map ? map[row] : row] = s;
}

template <int NPT>
__global__ __launch_bounds__(kGemvThreads) void k_gemv(const double *__restrict__ A, int M, int Mp,
                                                       const double *__restrict__ d, double *__restrict__ y,
                                                       const int32_t *__restrict__ map, const int *done) {
    gemv_body<NPT>(blockIdx.x, gridDim.x, A, M, Mp, d, y, map, done);
}

void launch_coarse_solve(Ctx &c, Stage &s, const int *done) { launch_coarse_solve_with(c, s, s.Ainv, done); }

// p_c = Ainv d with the stage's coarse vectors (Ainv: the Galerkin inverse or
// another inverse of the stage's size).
// loads per thread of the coarse GEMV for M columns
static int gemv_npt(int M) {
    const int npt = cdiv(M, kGemvThreads);
    if (npt <= 4) return std::max(npt, 1);
    if (npt <= 6) return 6;
    if (npt <= 8) return 8;
    if (npt <= 9) return 9;
    if (npt <= 10) return 10;
    if (npt <= 12) return 12;
    return 16;
}

void launch_coarse_solve_with(Ctx &c, Stage &s, const double *Ainv, const int *done) {
    ProfScope ps(c, MSRSB_K_COARSE);
#define MSRSB_GEMV(NPT)                                                                                          \
    case NPT:                                                                                                    \
        hipLaunchKernelGGL(k_gemv<NPT>, dim3(s.M), dim3(kGemvThreads), 0, c.stream, Ainv, s.M, s.Mp, s.dvec, s.pc, \
                           s.pc_map, done);                                                                      \
        break
    switch (gemv_npt(s.M)) {
        MSRSB_GEMV(1); MSRSB_GEMV(2); MSRSB_GEMV(3); MSRSB_GEMV(4); MSRSB_GEMV(6);
        MSRSB_GEMV(8); MSRSB_GEMV(9); MSRSB_GEMV(10); MSRSB_GEMV(12); MSRSB_GEMV(16);
    default: break;
    }
#undef MSRSB_GEMV
}

// ------------------------------------------------------- batched launches ----
// p_c = A_c^-1 d for every member, one launch per loads-per-thread key
// (grid: one workgroup per coarse row).
int bat_member_gemv(const Stage &s, int *key) {
    *key = gemv_npt(s.M);
    return s.M;
}

template <int NPT>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_b(const BMember *D, BGroup gp, const int *act) {
    int m, lb, nb;
    if (!bat_locate(gp, act, m, lb, nb)) return;
    const BMember &d = D[m];
    gemv_body<NPT>(lb, nb, d.Ainv, d.M, d.Mp, d.dvec, d.pc, d.pc_map, &d.status->done);
}

void bat_coarse_solve(Batch &B) {
    for (const HGroup &h : B.gemv) {
        if (h.g.n == 0) continue;
        const dim3 grid(h.g.total), blk(kGemvThreads);
#define MSRSB_BGEMV(NPT)                                                                               \
    case NPT:                                                                                          \
        hipLaunchKernelGGL(k_gemv_b<NPT>, grid, blk, 0, B.stream, B.d_mem, h.g, B.d_act);            \
        break
        switch (h.key) {
            MSRSB_BGEMV(1); MSRSB_BGEMV(2); MSRSB_BGEMV(3); MSRSB_BGEMV(4); MSRSB_BGEMV(6);
            MSRSB_BGEMV(8); MSRSB_BGEMV(9); MSRSB_BGEMV(10); MSRSB_BGEMV(12); MSRSB_BGEMV(16);
        default: break;
        }
#undef MSRSB_BGEMV
    }
}

// Coarse inverses of every member: the copy, the first pivot block, then per
// step K one panel launch and one update launch over all members whose
// matrices have more than K tiles (the others' workgroups return).
void bat_member_inverse(const Stage &s, int grid[3]) {
    const int nt = s.Mp / T_;
    grid[0] = cdiv((long)s.Mp * s.Mp, 2048);  // 8 entries per thread
    grid[1] = nt;
    grid[2] = nt * nt;
}

#define BAT_LOCATE()                              \
    int m, lb, nb;                                \
    if (!bat_locate(gp, act, m, lb, nb)) return;  \
    const BMember &d = D[m]

__device__ inline double *bat_dbuf(const BMember &d, int i) { return d.cbuf + (size_t)(d.cbuf_n + i * T_) * T_; }

__global__ __launch_bounds__(kGJThreads) void k_gj_copy_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    (void)nb;
    static_assert(kGJThreads == 256, "2048 entries per workgroup");
    const long n = (long)d.Mp * d.Mp, e0 = (long)lb * 2048 + threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const long e = e0 + (long)q * kGJThreads;
        if (e < n) d.Ainv[e] = d.Ac[e];
    }
}

__global__ __launch_bounds__(kGJThreads) void k_gj_diag_b(const BMember *D, BGroup gp, const int *act) {
    BAT_LOCATE();
    (void)lb;
    (void)nb;
    gj_diag_body(d.Ainv, d.Mp, 0, bat_dbuf(d, 0), d.flag, false);
}

__global__ __launch_bounds__(kGJThreads) void k_gj_panel_b(const BMember *D, BGroup gp, const int *act, int K) {
    BAT_LOCATE();
    if (K >= d.Mp / T_) return;
    gj_panel_body(lb, nb, d.Ainv, d.Mp, K, bat_dbuf(d, K & 1), d.cbuf);
}

__global__ __launch_bounds__(kGJThreads) void k_gj_update_b(const BMember *D, BGroup gp, const int *act, int K) {
    BAT_LOCATE();
    const int nt = d.Mp / T_;
    if (K >= nt) return;
    gj_update_body(lb, nb, d.Ainv, d.Mp, K, nt, bat_dbuf(d, K & 1), d.cbuf, bat_dbuf(d, (K + 1) & 1), d.flag,
                   false);
}

#undef BAT_LOCATE

void bat_coarse_inverse(Batch &B) {
    for (const HGroup &h : B.gjcopy)
        hipLaunchKernelGGL(k_gj_copy_b, dim3(h.g.total), dim3(kGJThreads), 0, B.stream, B.d_mem, h.g, B.d_act);
    for (const HGroup &h : B.one)
        hipLaunchKernelGGL(k_gj_diag_b, dim3(h.g.total), dim3(kGJThreads), 0, B.stream, B.d_mem, h.g, B.d_act);
    for (int K = 0; K < B.max_tiles; ++K) {
        for (const HGroup &h : B.gjpanel)
            hipLaunchKernelGGL(k_gj_panel_b, dim3(h.g.total), dim3(kGJThreads), 0, B.stream, B.d_mem, h.g, B.d_act,
                               K);
        for (const HGroup &h : B.gjupdate)
            hipLaunchKernelGGL(k_gj_update_b, dim3(h.g.total), dim3(kGJThreads), 0, B.stream, B.d_mem, h.g, B.d_act,
                               K);
    }
}

}  // namespace msrsb
