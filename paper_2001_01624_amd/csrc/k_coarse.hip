// Coarse factorisation and solve (section "Computational efficiency":
// inverting the coarse matrix by direct Gaussian elimination).
//
// A_c is SPD, so Gauss-Jordan elimination needs no pivoting: sweeping the
// pivots in order turns A_c into A_c^{-1} in place.  Each pivot of the sweep
// is a diagonal entry of a Schur complement of A_c (the square of the
// corresponding Cholesky diagonal), so a non-positive pivot means A_c is
// not SPD and is reported.  The sweep is blocked by kTile columns:
//   1. D = A[K,K] is inverted in LDS (one workgroup),
//   2. row panel A[K,J] <- D^{-1} A[K,J] and a copy C of the column panel,
//   3. A[I,J] -= C[I] A[K,J];  A[I,K] <- -C[I] D^{-1};  A[K,K] <- D^{-1}.
// Each cycle then applies the inverse by a GEMV (one wavefront per row).
#include "dev_util.h"
#include "msrsb_internal.h"

namespace msrsb {

constexpr int T_ = kTile;

__global__ __launch_bounds__(256) void k_gj_diag(double *__restrict__ A, int Mp, int k0, double *__restrict__ Dinv,
                                                 int *flag) {
    __shared__ double D[T_][T_ + 1];
    __shared__ double col[T_];
    const int tid = threadIdx.x;
    for (int e = tid; e < T_ * T_; e += blockDim.x) D[e / T_][e % T_] = A[(long)(k0 + e / T_) * Mp + k0 + e % T_];
    __syncthreads();
    for (int k = 0; k < T_; ++k) {
        const double p = D[k][k];
        if (tid == 0 && !(p > 0.0)) atomicOr(flag, 1);
        const double ip = p > 0.0 ? 1.0 / p : 0.0;
        if (tid < T_) col[tid] = D[tid][k];
        __syncthreads();
        if (tid < T_ && tid != k) D[k][tid] *= ip;
        __syncthreads();
        for (int e = tid; e < T_ * T_; e += blockDim.x) {
            const int i = e / T_, j = e % T_;
            if (i != k && j != k) D[i][j] -= col[i] * D[k][j];
        }
        __syncthreads();
        if (tid < T_) {
            if (tid != k) D[tid][k] = -col[tid] * ip;
            else D[k][k] = ip;
        }
        __syncthreads();
    }
    for (int e = tid; e < T_ * T_; e += blockDim.x) Dinv[e] = D[e / T_][e % T_];
}

// Workgroup t: row panel tile (columns of tile t) and column-panel copy (rows of tile t).
__global__ __launch_bounds__(256) void k_gj_panel(double *__restrict__ A, int Mp, int K, const double *__restrict__ Dinv,
                                                  double *__restrict__ C) {
    __shared__ double Ds[T_][T_ + 1];
    __shared__ double Bs[T_][T_ + 1];
    const int t = blockIdx.x, tid = threadIdx.x;
    if (t == K) return;
    const int k0 = K * T_, c0 = t * T_;
    for (int e = tid; e < T_ * T_; e += blockDim.x) {
        const int i = e / T_, j = e % T_;
        Ds[i][j] = Dinv[e];
        Bs[i][j] = A[(long)(k0 + i) * Mp + c0 + j];
        C[(long)(c0 + i) * T_ + j] = A[(long)(c0 + i) * Mp + k0 + j];
    }
    __syncthreads();
    for (int e = tid; e < T_ * T_; e += blockDim.x) {
        const int i = e / T_, j = e % T_;
        double s = 0.0;
#pragma unroll 8
        for (int m = 0; m < T_; ++m) s += Ds[i][m] * Bs[m][j];
        A[(long)(k0 + i) * Mp + c0 + j] = s;
    }
}

__global__ __launch_bounds__(256) void k_gj_update(double *__restrict__ A, int Mp, int K, const double *__restrict__ Dinv,
                                                   const double *__restrict__ C) {
    __shared__ double Cs[T_][T_ + 1];
    __shared__ double Bs[T_][T_ + 1];
    const int I = blockIdx.y, J = blockIdx.x, tid = threadIdx.x;
    const int r0 = I * T_, c0 = J * T_, k0 = K * T_;
    if (I == K) {
        if (J == K)
            for (int e = tid; e < T_ * T_; e += blockDim.x) A[(long)(k0 + e / T_) * Mp + k0 + e % T_] = Dinv[e];
        return;
    }
    for (int e = tid; e < T_ * T_; e += blockDim.x) {
        const int i = e / T_, j = e % T_;
        Cs[i][j] = C[(long)(r0 + i) * T_ + j];
        Bs[i][j] = (J == K) ? Dinv[e] : A[(long)(k0 + i) * Mp + c0 + j];
    }
    __syncthreads();
    for (int e = tid; e < T_ * T_; e += blockDim.x) {
        const int i = e / T_, j = e % T_;
        double s = 0.0;
#pragma unroll 8
        for (int m = 0; m < T_; ++m) s += Cs[i][m] * Bs[m][j];
        double *dst = &A[(long)(r0 + i) * Mp + c0 + j];
        if (J == K) *dst = -s;
        else *dst -= s;
    }
}

void launch_coarse_inverse(Ctx &c, Stage &s) {
    ProfScope ps(c, MSRSB_K_INVERSE);
    const int nt = s.Mp / T_;
    double *A = s.Ainv;
    hipMemcpyAsync(A, s.Ac, sizeof(double) * (size_t)s.Mp * s.Mp, hipMemcpyDeviceToDevice, c.stream);
    double *Dinv = c.scal + 6000;            // kTile^2 doubles
    double *C = c.cbuf;                       // Mp * kTile doubles
    for (int K = 0; K < nt; ++K) {
        hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, c.stream, A, s.Mp, K * T_, Dinv, c.flag);
        hipLaunchKernelGGL(k_gj_panel, dim3(nt), dim3(256), 0, c.stream, A, s.Mp, K, Dinv, C);
        hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(256), 0, c.stream, A, s.Mp, K, Dinv, C);
    }
}

// p_c = A_c^{-1} d: one wavefront per row, fixed-order lane sums.
__global__ __launch_bounds__(256) void k_gemv(const double *__restrict__ A, int M, int Mp, const double *__restrict__ d,
                                              double *__restrict__ y, const int *done) {
    if (done && *done) return;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= M) return;
    const double *a = A + (long)row * Mp;
    double s = 0.0;
    for (int k = lane; k < M; k += 64) s += a[k] * d[k];
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

void launch_coarse_solve(Ctx &c, Stage &s, const int *done) {
    ProfScope ps(c, MSRSB_K_COARSE);
    hipLaunchKernelGGL(k_gemv, dim3(cdiv(s.M, 4)), dim3(256), 0, c.stream, s.Ainv, s.M, s.Mp, s.dvec, s.pc, done);
}

}  // namespace msrsb
