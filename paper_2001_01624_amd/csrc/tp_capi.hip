// C entry points of the two-phase CPR solver (msrsb_tp_*): context set-up,
// assembly (with the pressure context's operator replaced by the IMPES
// pressure block and its bases updated locally), the two-stage
// preconditioner, GMRES on the full system and the Newton update.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dev_util.h"
#include "msrsb_internal.h"
#include "twophase.h"

using namespace msrsb;

struct msrsb_tp_ctx : public TpCtx {};

static double *tp_alloc(TpCtx &t, size_t n) {
    double *p = (double *)ctx_alloc(*t.ms, 8 * std::max<size_t>(n, 1));
    if (p) t.bufs.push_back(p);
    return p;
}

// Host copy of a device scalar array on the pressure context's stream.
static int tp_read(TpCtx &t, void *dst, const void *src, size_t bytes) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, t.ms->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t.ms->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "two-phase read");
    return MSRSB_OK;
}

extern "C" {

void msrsb_tp_destroy(msrsb_tp_ctx *t) {
    if (!t) return;
    if (t->ms) {
        (void)hipStreamSynchronize(t->ms->stream);
        for (void *p : t->bufs) ctx_free(*t->ms, p);
    }
    delete t;
}

int msrsb_tp_create(msrsb_ctx *ms, const double *pore_volume, const msrsb_fluid *fluid, int restart,
                    msrsb_tp_ctx **out) {
    if (!out) return MSRSB_E_INVAL;
    *out = nullptr;
    if (!ms || !pore_volume || !fluid || restart < 1 || restart > 200) {
        set_error("bad two-phase arguments (restart in [1, 200])");
        return MSRSB_E_INVAL;
    }
    if (!(fluid->mu_w > 0.0 && fluid->mu_o > 0.0 && fluid->n_w >= 1.0 && fluid->n_o >= 1.0)) {
        set_error("viscosities must be positive and Corey exponents >= 1");
        return MSRSB_E_INVAL;
    }
    Ctx &c = *reinterpret_cast<Ctx *>(ms);
    const size_t N = c.N;
    for (size_t i = 0; i < N; ++i)
        if (!(pore_volume[i] >= 0.0) || !std::isfinite(pore_volume[i]) || (c.h_active[i] && !(pore_volume[i] > 0.0))) {
            set_error("pore volume %zu must be positive on active cells and finite", i);
            return MSRSB_E_INVAL;
        }
    msrsb_tp_ctx *t = new msrsb_tp_ctx();
    t->ms = &c;
    t->fluid = {fluid->mu_w, fluid->mu_o, fluid->n_w, fluid->n_o};
    t->restart = restart;
    auto fail = [&](int rc) {
        msrsb_tp_destroy(t);
        return rc;
    };
    const size_t m = restart;
    t->T0 = tp_alloc(*t, 3 * N);
    t->WI0 = tp_alloc(*t, std::max(c.n_bc, 1));
    t->pv = tp_alloc(*t, N);
    t->act = (uint8_t *)tp_alloc(*t, (N + 7) / 8);
    t->R = tp_alloc(*t, 2 * N);
    t->Jd = tp_alloc(*t, 4 * N);
    t->Jo = tp_alloc(*t, 24 * N);
    t->Pinv = tp_alloc(*t, 4 * N);
    t->teff = tp_alloc(*t, 3 * N);
    t->bceff = tp_alloc(*t, std::max(c.n_bc, 1));
    t->vp = tp_alloc(*t, N);
    t->dp = tp_alloc(*t, N);
    t->r2 = tp_alloc(*t, 2 * N);
    t->V = tp_alloc(*t, (m + 1) * 2 * N);
    t->Z = tp_alloc(*t, m * 2 * N);
    t->w = tp_alloc(*t, 2 * N);
    t->part = tp_alloc(*t, (size_t)kTpRed * (m + 2));
    t->h = tp_alloc(*t, m + 2);
    for (void *p : {(void *)t->T0, (void *)t->WI0, (void *)t->pv, (void *)t->act, (void *)t->R, (void *)t->Jd,
                    (void *)t->Jo, (void *)t->Pinv, (void *)t->teff, (void *)t->bceff, (void *)t->vp, (void *)t->dp,
                    (void *)t->r2, (void *)t->V, (void *)t->Z, (void *)t->w, (void *)t->part, (void *)t->h})
        if (!p) return fail(MSRSB_E_NOMEM);
    // the pressure context's current operator is the single-phase one
    const double *src3[3] = {c.tx, c.ty, c.tz};
    hipError_t e = hipSuccess;
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(t->T0 + a * N, src3[a], 8 * N, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess && c.n_bc > 0)
        e = hipMemcpyAsync(t->WI0, c.bc_trans, 8 * (size_t)c.n_bc, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t->pv, pore_volume, 8 * N, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t->act, c.h_active.data(), N, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return fail(hip_fail(e, "two-phase set-up"));
    *out = t;
    return MSRSB_OK;
}

int msrsb_tp_assemble(msrsb_tp_ctx *t, double dt, const double *d_p, const double *d_s, const double *d_s_old,
                      const double *d_q, int basis_sweeps, double *d_res, double *res_norm) {
    if (!t || !d_p || !d_s || !d_s_old || !(dt > 0.0) || basis_sweeps < 0) {
        set_error("bad two-phase assembly arguments");
        return MSRSB_E_INVAL;
    }
    Ctx &c = *t->ms;
    for (auto &s : c.stages)
        if (!s.has_basis) {
            set_error("the pressure context's bases must exist before assembly");
            return MSRSB_E_STATE;
        }
    tp_launch_assemble(*t, dt, d_p, d_s, d_s_old, d_q ? d_q : c.src);
    // the IMPES pressure block into the pressure context, bases updated locally
    int rc = set_operator_device(c, t->teff, t->bceff);
    if (rc) return rc;
    if ((rc = refresh_bases(c, basis_sweeps))) return rc;
    int *flag = c.flag;
    hipMemsetAsync(flag, 0, sizeof(int), c.stream);
    tp_launch_ilu(*t, flag);
    tp_launch_dots(*t, t->R, 1, t->R, t->h);
    double nr = 0.0;
    int hflag = 0;
    if ((rc = tp_read(*t, &nr, t->h, sizeof(double))) || (rc = tp_read(*t, &hflag, flag, sizeof(int)))) return rc;
    if (hflag & 1) {
        set_error("singular 2x2 pivot in the full-system ILU(0)");
        return MSRSB_E_SINGULAR;
    }
    if (d_res && hipMemcpyAsync(d_res, t->R, 16 * (size_t)c.N, hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
        return hip_fail(hipGetLastError(), "residual copy");
    if (res_norm) *res_norm = std::sqrt(nr);
    t->assembled = true;
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "two-phase assembly");
    return MSRSB_OK;
}

int msrsb_tp_apply(msrsb_tp_ctx *t, int op, const double *d_in, double *d_out) {
    if (!t || !d_in || !d_out || d_in == d_out || (op != 0 && op != 1)) {
        set_error("bad two-phase apply arguments");
        return MSRSB_E_INVAL;
    }
    if (!t->assembled) {
        set_error("apply before assembly");
        return MSRSB_E_STATE;
    }
    if (op == 0) tp_launch_matvec(*t, d_in, d_out);
    else tp_launch_cpr(*t, d_in, d_out);
    hipError_t e = hipStreamSynchronize(t->ms->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "two-phase apply");
    return MSRSB_OK;
}

// GMRES(m) on J dx = -R with the two-stage CPR as right preconditioner
// (Arnoldi by classical Gram-Schmidt with a second pass; Givens rotations
// and the small least-squares problem on the host).
int msrsb_tp_solve(msrsb_tp_ctx *t, double *d_dx, double rtol, int max_iters, int *iters, double *relres) {
    if (!t || !d_dx || !(rtol >= 0.0) || max_iters < 0) {
        set_error("bad two-phase solve arguments");
        return MSRSB_E_INVAL;
    }
    if (!t->assembled) {
        set_error("solve before assembly");
        return MSRSB_E_STATE;
    }
    Ctx &c = *t->ms;
    const long n = 2L * c.N;
    const int m = t->restart;
    hipMemsetAsync(d_dx, 0, 8 * (size_t)n, c.stream);
    double nb2 = 0.0;
    int rc;
    tp_launch_dots(*t, t->R, 1, t->R, t->h);
    if ((rc = tp_read(*t, &nb2, t->h, sizeof(double)))) return rc;
    const double nb = nb2 > 0.0 ? std::sqrt(nb2) : 1.0;
    int its = 0;
    double rel = 0.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hcol(m + 2), one{-1.0};
    double *minus_one = t->h + m + 1;
    if (hipMemcpyAsync(minus_one, one.data(), sizeof(double), hipMemcpyHostToDevice, c.stream) != hipSuccess)
        return hip_fail(hipGetLastError(), "constant upload");
    for (;;) {
        // r = -R - J dx into V(0)
        tp_launch_matvec(*t, d_dx, t->V);
        tp_launch_scale(*t, t->V, -1.0, t->V);
        tp_launch_multiaxpy(*t, t->R, 1, minus_one, 1.0, t->V);  // V0 = -J dx - R
        double beta2 = 0.0;
        tp_launch_dots(*t, t->V, 1, t->V, t->h);
        if ((rc = tp_read(*t, &beta2, t->h, sizeof(double)))) return rc;
        const double beta = std::sqrt(beta2);
        rel = beta / nb;
        if (rel <= rtol || its >= max_iters || beta == 0.0) break;
        tp_launch_scale(*t, t->V, 1.0 / beta, t->V);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && its < max_iters; ++j) {
            double *vj = t->V + (long)j * n, *zj = t->Z + (long)j * n;
            tp_launch_cpr(*t, vj, zj);
            tp_launch_matvec(*t, zj, t->w);
            // two Gram-Schmidt passes; the coefficients of both add up
            std::fill(hcol.begin(), hcol.end(), 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<double> hp(j + 1);
                tp_launch_dots(*t, t->V, j + 1, t->w, t->h);
                tp_launch_multiaxpy(*t, t->V, j + 1, t->h, -1.0, t->w);
                if ((rc = tp_read(*t, hp.data(), t->h, sizeof(double) * (j + 1)))) return rc;
                for (int i = 0; i <= j; ++i) hcol[i] += hp[i];
            }
            double w2 = 0.0;
            tp_launch_dots(*t, t->w, 1, t->w, t->h);
            if ((rc = tp_read(*t, &w2, t->h, sizeof(double)))) return rc;
            hcol[j + 1] = std::sqrt(w2);
            if (hcol[j + 1] > 0.0) tp_launch_scale(*t, t->w, 1.0 / hcol[j + 1], t->V + (long)(j + 1) * n);
            // Givens rotations
            for (int i = 0; i < j; ++i) {
                const double a = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
                hcol[i] = a;
            }
            const double r = std::hypot(hcol[j], hcol[j + 1]);
            cs[j] = r > 0.0 ? hcol[j] / r : 1.0;
            sn[j] = r > 0.0 ? hcol[j + 1] / r : 0.0;
            hcol[j] = r;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
            ++its;
            k = j + 1;
            if (std::fabs(g[j + 1]) / nb <= rtol || r == 0.0 || hcol[j + 1] == 0.0) break;
        }
        // dx += Z y with H y = g (upper triangular)
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
            y[i] = H[(size_t)i * m + i] != 0.0 ? s / H[(size_t)i * m + i] : 0.0;
        }
        if (hipMemcpyAsync(t->h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c.stream) != hipSuccess)
            return hip_fail(hipGetLastError(), "coefficient upload");
        tp_launch_multiaxpy(*t, t->Z, k, t->h, 1.0, d_dx);
        if (hipStreamSynchronize(c.stream) != hipSuccess) return hip_fail(hipGetLastError(), "solution update");
    }
    if (iters) *iters = its;
    if (relres) *relres = rel;
    if (!(rel <= rtol)) {
        set_error("two-phase GMRES: tolerance %g not met after %d iterations (%g)", rtol, its, rel);
        return MSRSB_E_NOCONV;
    }
    return MSRSB_OK;
}

int msrsb_tp_update(msrsb_tp_ctx *t, const double *d_dx, double *d_p, double *d_s) {
    if (!t || !d_dx || !d_p || !d_s) {
        set_error("bad two-phase update arguments");
        return MSRSB_E_INVAL;
    }
    tp_launch_update(*t, d_dx, d_p, d_s);
    hipError_t e = hipStreamSynchronize(t->ms->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "two-phase update");
    return MSRSB_OK;
}

}  // extern "C"
