// The two-point seven-point stencil of the fine operator A = D - T, shared
// by the fine-grid kernels and the fused residual-restriction kernel so that
// both evaluate (A x)_i with the same operations in the same order.
#pragma once

#include "msrsb_internal.h"

namespace msrsb {

// The six faces of cell i in the order -x, +x, -y, +y, -z, +z: neighbour
// index (clamped to i outside the grid) and transmissibility (0 there).  All
// loads depend on i alone, so a kernel can issue every load before its first
// use.
template <typename TT>
__device__ inline void cell_faces(const Fine &g, int i, const TT *__restrict__ tx, const TT *__restrict__ ty,
                                  const TT *__restrict__ tz, int l[6], TT t[6]) {
    const int step[3] = {1, g.nx, g.nxy};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const TT *Ta = a == 0 ? tx : (a == 1 ? ty : tz);
        const bool dn = i >= step[a], up = i + step[a] < g.N;
        l[2 * a] = dn ? i - step[a] : i;
        l[2 * a + 1] = up ? i + step[a] : i;
        const TT td = Ta[l[2 * a]], tu = Ta[i];
        t[2 * a] = dn ? td : (TT)0;
        t[2 * a + 1] = up ? tu : (TT)0;
    }
}

// (A x)_i for an active cell with diagonal d; the off-diagonal terms are
// subtracted in face order (faces outside the grid have t = 0).
__device__ inline double ax_row(const Fine &g, const double *__restrict__ x, int i, double d) {
    int l[6];
    double t[6], xl[6];
    cell_faces(g, i, g.tx, g.ty, g.tz, l, t);
    const double xi = x[i];
#pragma unroll
    for (int q = 0; q < 6; ++q) xl[q] = x[l[q]];
    double s = d * xi;
#pragma unroll
    for (int q = 0; q < 6; ++q) s -= t[q] * xl[q];
    return s;
}

// r_i = b_i - (A x)_i on an active cell, 0 on an inactive one.
__device__ inline double residual_cell(const Fine &g, const double *__restrict__ b, const double *__restrict__ x,
                                       int i) {
    const double d = g.diag[i], bi = b[i];
    const double ax = ax_row(g, x, i, d);
    return d > 0.0 ? bi - ax : 0.0;
}

}  // namespace msrsb
