// Device helpers shared by the rectilinear-stage kernels (sweeps, transfer
// operators, Galerkin product): cell coordinates and the implicit slot ->
// block map of a cell with per-axis first block lo and support count nv.
#pragma once

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

}  // namespace msrsb
