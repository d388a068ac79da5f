// Device helpers shared by the kernel files: fixed-order wave/block
// reductions (results never depend on timing), BF16 conversion and the
// Cartesian cell-coordinate helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msrsb {

// Sum over the 64 lanes of a wavefront; the tree shape is fixed, so the
// result is the same on every run.  Valid in lane 0.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Block-wide sum in a fixed order (waves in index order).  `lds` needs
// blockDim.x/64 doubles.  Valid in thread 0.
__device__ inline double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) s += lds[k];
    }
    __syncthreads();
    return s;
}

// Sum of p[0..n) by one workgroup in a fixed order: thread t adds
// p[t], p[t + blockDim], ... (loads unrolled), then block_sum.
__device__ inline double sum_partials(const double *__restrict__ p, int n, double *lds) {
    double s = 0.0;
#pragma unroll 8
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += p[k];
    return block_sum(s, lds);
}

// Sum of p[lane], p[lane + 64], ... (indices below n) in that order, as the
// plain strided loop adds them, with eight loads issued before their adds.
__device__ inline double lane_strided_sum(const double *__restrict__ p, int lane, int n) {
    double v = 0.0;
    for (int b0 = lane; b0 < n; b0 += 8 * 64) {
        double t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = p[min(b0 + 64 * q, n - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (b0 + 64 * q < n) v += t[q];
    }
    return v;
}

__device__ inline double block_max(double v, double *lds) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) s = fmax(s, lds[k]);
    }
    __syncthreads();
    return s;
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each
// with its own L2.  xcd_block renumbers them so that XCD x runs one
// contiguous range of logical blocks: stencil neighbours in the next row or
// layer are then read through the same L2.  The grid must be a multiple of
// kXcd (xcd_grid rounds up); logical ids past the real block count exit.
constexpr int kXcd = 8;
__device__ inline int xcd_block(int bid, int nblk) {
    const int per = nblk / kXcd;
    return (bid % kXcd) * per + bid / kXcd;
}
__device__ inline int xcd_block() { return xcd_block(blockIdx.x, gridDim.x); }
inline int xcd_grid(int nblocks) { return ((nblocks + kXcd - 1) / kXcd) * kXcd; }

// Traversal order of the stencil kernels: thread t visits the cell with x
// fastest, then z, then y.  Memory stays x-y-z; only the visiting order
// changes, so that the largest neighbour reuse distance is one x-z slice
// (nx*nz cells) rather than one x-y layer.  Returns -1 past the end.
__device__ inline int xzy_cell(int t, int nx, int ny, int nz) {
    const int nxz = nx * nz;
    const int y = t / nxz;
    if (y >= ny) return -1;
    const int r = t - y * nxz;
    const int z = r / nx, x = r - z * nx;
    return x + nx * (y + ny * z);
}

__device__ inline float bf16_to_float(uint16_t u) { return __uint_as_float(((uint32_t)u) << 16); }

// Round-to-nearest-even FP32 -> BF16 (finite inputs).
__device__ inline uint16_t float_to_bf16(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

template <typename T> __device__ inline double ld_basis(const T *p, long idx) { return (double)p[idx]; }
template <> __device__ inline double ld_basis<uint16_t>(const uint16_t *p, long idx) {
    return (double)bf16_to_float(p[idx]);
}

// Sum of V values (V a power of two <= 64) over the wavefront, by halving
// exchanges: afterwards every lane holds the total of value lane >> (6 - log2 V).
// Lane pairs add the same two operands, so the result does not depend on
// the lane that computes it.
template <int V>
__device__ inline double wave_transpose_sum(double (&v)[V], int lane) {
#pragma unroll
    for (int step = 0; step < 6; ++step) {
        const int o = 32 >> step;
        const int c = V >> step;
        if (c >= 2) {
            // lanes with bit o clear keep the lower half, the others the
            // upper half; both halves are exchanged and the kept one summed
            // (a select on sums, not on array slots, keeps v in registers)
            const bool up = lane & o;
#pragma unroll
            for (int k = 0; k < (c >> 1); ++k) {
                const double lo = v[k], hi = v[k + (c >> 1)];
                const double rlo = __shfl_xor(lo, o, 64), rhi = __shfl_xor(hi, o, 64);
                v[k] = up ? hi + rhi : lo + rlo;
            }
        } else {
            v[0] += __shfl_xor(v[0], o, 64);
        }
    }
    return v[0];
}

// Workgroup total of V per-thread values, written to out[0..nout): waves in
// order, each wave by wave_transpose_sum.
template <int V>
__device__ inline void group_sum_store(double (&v)[V], int nout, double *red, double *__restrict__ out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double t = wave_transpose_sum<V>(v, lane);
    if ((lane & ((64 / V) - 1)) == 0) red[wv * V + lane / (64 / V)] = t;
    __syncthreads();
    for (int q = threadIdx.x; q < nout; q += blockDim.x) {
        double sum = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w * V + q];
        out[q] = sum;
    }
    __syncthreads();
}

// Workgroup totals of V per-thread values left in red[nw*V + q] (nw = number
// of wavefronts; red holds (nw + 1) * V doubles): waves in order, each wave
// by wave_transpose_sum.  Ends with a barrier.
template <int V>
__device__ inline void group_sum_lds(double (&v)[V], double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    const double t = wave_transpose_sum<V>(v, lane);
    if ((lane & ((64 / V) - 1)) == 0) red[wv * V + lane / (64 / V)] = t;
    __syncthreads();
    if ((int)threadIdx.x < V) {
        double sum = 0.0;
        for (int w = 0; w < nw; ++w) sum += red[w * V + threadIdx.x];
        red[nw * V + threadIdx.x] = sum;
    }
    __syncthreads();
}

}  // namespace msrsb
