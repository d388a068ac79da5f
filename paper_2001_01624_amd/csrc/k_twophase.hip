// Two-phase (water/oil) fully implicit model and the two-stage CPR
// preconditioner (sections "Model equations", "Discrete equations",
// "Preconditioning: the constrained pressure residual (CPR) method" and
// "Description of the solution procedure").
//
// Unknowns per cell: pressure p and water saturation s; vectors of the full
// system interleave them per cell in box numbering, v[2i] (water equation /
// pressure) and v[2i+1] (oil equation / saturation); inactive cells hold 0.
// The Jacobian is kept by rows of 2x2 blocks: the diagonal block of cell i
// and the blocks of its six neighbours (-x, +x, -y, +y, -z, +z), zero where
// no face exists.
#include "dev_util.h"
#include "msrsb_internal.h"
#include "twophase.h"

namespace msrsb {

struct TpGeom {
    int nx, ny, nz, nxy, N;
    const double *T0[3];          // single-phase face transmissibilities (+x, +y, +z)
    const uint8_t *act;
};

__device__ inline void mob(double s, const TpFluid &f, double *lw, double *lo, double *dlw, double *dlo) {
    const double so = 1.0 - s;
    *lw = pow(s, f.n_w) / f.mu_w;
    *lo = pow(so, f.n_o) / f.mu_o;
    *dlw = f.n_w == 1.0 ? 1.0 / f.mu_w : f.n_w * pow(s, f.n_w - 1.0) / f.mu_w;
    *dlo = f.n_o == 1.0 ? -1.0 / f.mu_o : -f.n_o * pow(so, f.n_o - 1.0) / f.mu_o;
}

// Neighbour q of cell i (0: -x, 1: +x, 2: -y, 3: +y, 4: -z, 5: +z) and the
// face's single-phase T (0 when there is no face).
__device__ inline int nbr(const TpGeom &g, int i, int q, double *T) {
    const int a = q >> 1;
    const int step = a == 0 ? 1 : (a == 1 ? g.nx : g.nxy);
    if (q & 1) {
        *T = g.T0[a][i];
        return i + step;
    }
    if (i < step) {
        *T = 0.0;
        return i;
    }
    *T = g.T0[a][i - step];
    return i - step;
}

// Residual, Jacobian rows and the IMPES pressure operator (face coefficients
// T lambda_t(up)/2 on the +x/+y/+z faces, well terms WI lambda_t/2).
__global__ void k_tp_assemble(TpGeom g, TpFluid f, double dt, const double *__restrict__ p,
                              const double *__restrict__ s, const double *__restrict__ s_old,
                              const double *__restrict__ pv, const double *__restrict__ q,
                              const int32_t *__restrict__ bcptr, const int32_t *__restrict__ bcidx,
                              const double *__restrict__ wi, const double *__restrict__ pbh, double *__restrict__ R,
                              double *__restrict__ Jd, double *__restrict__ Jo, double *__restrict__ teff,
                              double *__restrict__ bceff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    if (!g.act[i]) {
        R[2 * i] = R[2 * i + 1] = 0.0;
        for (int e = 0; e < 4; ++e) Jd[4 * i + e] = 0.0;
        for (int qq = 0; qq < 6; ++qq)
            for (int e = 0; e < 4; ++e) Jo[((long)qq * g.N + i) * 4 + e] = 0.0;
        for (int a = 0; a < 3; ++a) teff[(long)a * g.N + i] = 0.0;
        return;
    }
    double lw, lo, dlw, dlo;
    mob(s[i], f, &lw, &lo, &dlw, &dlo);
    const double acc = pv[i] / dt, ds = s[i] - s_old[i];
    double rw = acc * ds - q[i], ro = -acc * ds;
    double d00 = 0.0, d01 = acc, d10 = 0.0, d11 = -acc;
    for (int qq = 0; qq < 6; ++qq) {
        double T;
        const int l = nbr(g, i, qq, &T);
        double o00 = 0.0, o01 = 0.0, o10 = 0.0, o11 = 0.0;
        if (T != 0.0) {
            const double dp = p[i] - p[l];
            // the face (a, b), a < b, takes a's mobility when p_a >= p_b
            const bool iup = (qq & 1) ? p[i] >= p[l] : p[i] > p[l];
            double mw = lw, mo = lo;
            double lwl, lol, dlwl, dlol;
            mob(s[l], f, &lwl, &lol, &dlwl, &dlol);
            if (!iup) {
                mw = lwl;
                mo = lol;
            }
            rw += T * mw * dp;
            ro += T * mo * dp;
            d00 += T * mw;
            d10 += T * mo;
            o00 = -T * mw;
            o10 = -T * mo;
            if (iup) {
                d01 += T * dlw * dp;
                d11 += T * dlo * dp;
            } else {
                o01 = T * dlwl * dp;
                o11 = T * dlol * dp;
            }
            if (qq & 1) teff[(long)(qq >> 1) * g.N + i] = 0.5 * T * (mw + mo);
        } else if (qq & 1) {
            teff[(long)(qq >> 1) * g.N + i] = 0.0;
        }
        double *o = Jo + ((long)qq * g.N + i) * 4;
        o[0] = o00;
        o[1] = o01;
        o[2] = o10;
        o[3] = o11;
    }
    for (int k = bcptr[i]; k < bcptr[i + 1]; ++k) {
        const int c = bcidx[k];
        const double w = wi[c], dpc = p[i] - pbh[c];
        rw += w * lw * dpc;
        ro += w * lo * dpc;
        d00 += w * lw;
        d10 += w * lo;
        d01 += w * dlw * dpc;
        d11 += w * dlo * dpc;
        bceff[c] = 0.5 * w * (lw + lo);
    }
    R[2 * i] = rw;
    R[2 * i + 1] = ro;
    Jd[4 * i] = d00;
    Jd[4 * i + 1] = d01;
    Jd[4 * i + 2] = d10;
    Jd[4 * i + 3] = d11;
}

__device__ inline bool inv2(const double *m, double *r) {
    const double det = m[0] * m[3] - m[1] * m[2];
    if (!(det != 0.0) || !isfinite(det)) return false;
    const double id = 1.0 / det;
    r[0] = m[3] * id;
    r[1] = -m[1] * id;
    r[2] = -m[2] * id;
    r[3] = m[0] * id;
    return true;
}

__device__ inline bool is_red(const TpGeom &g, int i) {
    return ((i % g.nx) + (i / g.nx) % g.ny + i / g.nxy) % 2 == 0;
}

// Red-black block ILU(0), red cells first: a red pivot is its diagonal block;
// every neighbour of a black cell is red, so its pivot is
// S = D_b - sum_l J_bl D_l^{-1} J_lb (the ILU(0) Schur complement keeps only
// the diagonal blocks: black cells are not coupled to each other).  Stored
// inverted.  flag |= 1 on a singular pivot.
__global__ void k_tp_ilu_red(TpGeom g, const double *__restrict__ Jd, double *__restrict__ Pinv, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N || !is_red(g, i)) return;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.act[i] && !inv2(Jd + 4 * i, r)) atomicOr(flag, 1);
    for (int e = 0; e < 4; ++e) Pinv[4 * i + e] = r[e];
}

__global__ void k_tp_ilu_black(TpGeom g, const double *__restrict__ Jd, const double *__restrict__ Jo,
                               double *__restrict__ Pinv, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N || is_red(g, i)) return;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.act[i]) {
        double S[4] = {Jd[4 * i], Jd[4 * i + 1], Jd[4 * i + 2], Jd[4 * i + 3]};
        for (int qq = 0; qq < 6; ++qq) {
            double T;
            const int l = nbr(g, i, qq, &T);
            if (T == 0.0) continue;
            const double *A = Jo + ((long)qq * g.N + i) * 4;             // J_il
            const double *B = Jo + ((long)(qq ^ 1) * g.N + l) * 4;       // J_li
            const double *Di = Pinv + 4 * l;                              // D_l^{-1}
            // A Di B
            const double t00 = A[0] * Di[0] + A[1] * Di[2], t01 = A[0] * Di[1] + A[1] * Di[3];
            const double t10 = A[2] * Di[0] + A[3] * Di[2], t11 = A[2] * Di[1] + A[3] * Di[3];
            S[0] -= t00 * B[0] + t01 * B[2];
            S[1] -= t00 * B[1] + t01 * B[3];
            S[2] -= t10 * B[0] + t11 * B[2];
            S[3] -= t10 * B[1] + t11 * B[3];
        }
        if (!inv2(S, r)) atomicOr(flag, 1);
    }
    for (int e = 0; e < 4; ++e) Pinv[4 * i + e] = r[e];
}

// y = (L U)^{-1} v: black cells y_b = S_b^{-1} (v_b - sum_l J_bl D_l^{-1} v_l),
// then red cells y_r = D_r^{-1} (v_r - sum_b J_rb y_b).
__global__ void k_tp_solve_black(TpGeom g, const double *__restrict__ Jo, const double *__restrict__ Pinv,
                                 const double *__restrict__ v, double *__restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N || is_red(g, i)) return;
    double z0 = v[2 * i], z1 = v[2 * i + 1];
    for (int qq = 0; qq < 6; ++qq) {
        double T;
        const int l = nbr(g, i, qq, &T);
        if (T == 0.0) continue;
        const double *D = Pinv + 4 * l;
        const double u0 = D[0] * v[2 * l] + D[1] * v[2 * l + 1], u1 = D[2] * v[2 * l] + D[3] * v[2 * l + 1];
        const double *A = Jo + ((long)qq * g.N + i) * 4;
        z0 -= A[0] * u0 + A[1] * u1;
        z1 -= A[2] * u0 + A[3] * u1;
    }
    const double *S = Pinv + 4 * i;
    y[2 * i] = S[0] * z0 + S[1] * z1;
    y[2 * i + 1] = S[2] * z0 + S[3] * z1;
}

__global__ void k_tp_solve_red(TpGeom g, const double *__restrict__ Jo, const double *__restrict__ Pinv,
                               const double *__restrict__ v, double *__restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N || !is_red(g, i)) return;
    double z0 = v[2 * i], z1 = v[2 * i + 1];
    for (int qq = 0; qq < 6; ++qq) {
        double T;
        const int l = nbr(g, i, qq, &T);
        if (T == 0.0) continue;
        const double *A = Jo + ((long)qq * g.N + i) * 4;
        z0 -= A[0] * y[2 * l] + A[1] * y[2 * l + 1];
        z1 -= A[2] * y[2 * l] + A[3] * y[2 * l + 1];
    }
    const double *D = Pinv + 4 * i;
    y[2 * i] = D[0] * z0 + D[1] * z1;
    y[2 * i + 1] = D[2] * z0 + D[3] * z1;
}

// out = J x, or out = v - J (x_p, 0) when v is given (the residual of the
// pressure predictor's correction: x holds pressures only, [N]).
template <bool PRES>
__global__ void k_tp_matvec(TpGeom g, const double *__restrict__ Jd, const double *__restrict__ Jo,
                            const double *__restrict__ x, const double *__restrict__ v, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N) return;
    double y0, y1;
    if (PRES) {
        y0 = Jd[4 * i] * x[i];
        y1 = Jd[4 * i + 2] * x[i];
    } else {
        y0 = Jd[4 * i] * x[2 * i] + Jd[4 * i + 1] * x[2 * i + 1];
        y1 = Jd[4 * i + 2] * x[2 * i] + Jd[4 * i + 3] * x[2 * i + 1];
    }
    for (int qq = 0; qq < 6; ++qq) {
        double T;
        const int l = nbr(g, i, qq, &T);
        if (T == 0.0) continue;
        const double *A = Jo + ((long)qq * g.N + i) * 4;
        if (PRES) {
            y0 += A[0] * x[l];
            y1 += A[2] * x[l];
        } else {
            y0 += A[0] * x[2 * l] + A[1] * x[2 * l + 1];
            y1 += A[2] * x[2 * l] + A[3] * x[2 * l + 1];
        }
    }
    if (PRES) {
        out[2 * i] = v[2 * i] - y0;
        out[2 * i + 1] = v[2 * i + 1] - y1;
    } else {
        out[2 * i] = y0;
        out[2 * i + 1] = y1;
    }
}

// pressure residual of the IMPES weights (1/2, 1/2)
__global__ void k_tp_pres_rhs(int N, const double *__restrict__ v, double *__restrict__ vp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) vp[i] = 0.5 * (v[2 * i] + v[2 * i + 1]);
}

__global__ void k_tp_add_pres(int N, const double *__restrict__ dp, double *__restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[2 * i] += dp[i];
}

// Newton update: p += dp, s = clamp(s + ds, 0, 1) on active cells
__global__ void k_tp_update(TpGeom g, const double *__restrict__ dx, double *__restrict__ p, double *__restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.N || !g.act[i]) return;
    p[i] += dx[2 * i];
    s[i] = fmin(1.0, fmax(0.0, s[i] + dx[2 * i + 1]));
}

// ---- vector kernels of the GMRES on the full system (fixed-order sums) ----

// part[j * gridDim + block] = block's share of V_j . w, j < k
__global__ __launch_bounds__(kBlock) void k_tp_multidot(long n, const double *__restrict__ V, int k,
                                                        const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double lds[kBlock / 64];
    for (int j = 0; j < k; ++j) {
        double a = 0.0;
        for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
            a += V[(long)j * n + t] * w[t];
        a = block_sum(a, lds);
        if (threadIdx.x == 0) part[(long)j * gridDim.x + blockIdx.x] = a;
    }
}

__global__ __launch_bounds__(kBlock) void k_tp_finish(int nb, const double *__restrict__ part,
                                                      double *__restrict__ h) {
    __shared__ double lds[kBlock / 64];
    const double s = sum_partials(part + (long)blockIdx.x * nb, nb, lds);
    if (threadIdx.x == 0) h[blockIdx.x] = s;
}

// w += sign * sum_j V_j h_j (h on the device)
__global__ void k_tp_multiaxpy(long n, const double *__restrict__ V, int k, const double *__restrict__ h,
                               double sign, double *__restrict__ w) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        double a = w[t];
        for (int j = 0; j < k; ++j) a += sign * V[(long)j * n + t] * h[j];
        w[t] = a;
    }
}

__global__ void k_tp_scale(long n, const double *__restrict__ a, double f, double *__restrict__ b) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t] * f;
}

// ---- launchers ----

static TpGeom geom(TpCtx &t) {
    TpGeom g;
    const Ctx &c = *t.ms;
    g.nx = c.nx; g.ny = c.ny; g.nz = c.nz; g.nxy = c.nx * c.ny; g.N = c.N;
    for (int a = 0; a < 3; ++a) g.T0[a] = t.T0 + (size_t)a * c.N;
    g.act = t.act;
    return g;
}

void tp_launch_assemble(TpCtx &t, double dt, const double *p, const double *s, const double *s_old, const double *q) {
    Ctx &c = *t.ms;
    TpGeom g = geom(t);
    hipLaunchKernelGGL(k_tp_assemble, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, t.fluid, dt, p, s, s_old,
                       t.pv, q, c.bcptr, c.bcidx, t.WI0, c.bc_value, t.R, t.Jd, t.Jo, t.teff, t.bceff);
}

void tp_launch_ilu(TpCtx &t, int *flag) {
    Ctx &c = *t.ms;
    TpGeom g = geom(t);
    hipLaunchKernelGGL(k_tp_ilu_red, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, t.Jd, t.Pinv, flag);
    hipLaunchKernelGGL(k_tp_ilu_black, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, t.Jd, t.Jo, t.Pinv,
                       flag);
}

void tp_launch_matvec(TpCtx &t, const double *x, double *out) {
    Ctx &c = *t.ms;
    TpGeom g = geom(t);
    hipLaunchKernelGGL(k_tp_matvec<false>, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, t.Jd, t.Jo, x,
                       nullptr, out);
}

// y = CPR^{-1} v (v and y distinct [2N] vectors)
void tp_launch_cpr(TpCtx &t, const double *v, double *y) {
    Ctx &c = *t.ms;
    TpGeom g = geom(t);
    const dim3 grid(cdiv(c.N, kBlock)), blk(kBlock);
    hipLaunchKernelGGL(k_tp_pres_rhs, grid, blk, 0, c.stream, c.N, v, t.vp);
    ms_precondition(c, t.vp, t.dp);  // stage 1: the multiscale pressure predictor
    hipLaunchKernelGGL(k_tp_matvec<true>, grid, blk, 0, c.stream, g, t.Jd, t.Jo, t.dp, v, t.r2);
    hipLaunchKernelGGL(k_tp_solve_black, grid, blk, 0, c.stream, g, t.Jo, t.Pinv, t.r2, y);  // stage 2: ILU(0)
    hipLaunchKernelGGL(k_tp_solve_red, grid, blk, 0, c.stream, g, t.Jo, t.Pinv, t.r2, y);
    hipLaunchKernelGGL(k_tp_add_pres, grid, blk, 0, c.stream, c.N, t.dp, y);
}

void tp_launch_update(TpCtx &t, const double *dx, double *p, double *s) {
    Ctx &c = *t.ms;
    TpGeom g = geom(t);
    hipLaunchKernelGGL(k_tp_update, dim3(cdiv(c.N, kBlock)), dim3(kBlock), 0, c.stream, g, dx, p, s);
}

// h[0..k) = V[0..k)^T w (device), fixed order
void tp_launch_dots(TpCtx &t, const double *V, int k, const double *w, double *h) {
    Ctx &c = *t.ms;
    const long n = 2L * c.N;
    hipLaunchKernelGGL(k_tp_multidot, dim3(kTpRed), dim3(kBlock), 0, c.stream, n, V, k, w, t.part);
    hipLaunchKernelGGL(k_tp_finish, dim3(k), dim3(kBlock), 0, c.stream, kTpRed, t.part, h);
}

void tp_launch_multiaxpy(TpCtx &t, const double *V, int k, const double *h, double sign, double *w) {
    Ctx &c = *t.ms;
    const long n = 2L * c.N;
    hipLaunchKernelGGL(k_tp_multiaxpy, dim3(std::min<long>(cdiv(n, kBlock), 8192)), dim3(kBlock), 0, c.stream, n, V, k,
                       h, sign, w);
}

void tp_launch_scale(TpCtx &t, const double *a, double f, double *b) {
    Ctx &c = *t.ms;
    const long n = 2L * c.N;
    hipLaunchKernelGGL(k_tp_scale, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, c.stream, n, a, f, b);
}

}  // namespace msrsb
