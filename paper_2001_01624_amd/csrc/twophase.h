// Two-phase context of the CPR preconditioner (internal).
#pragma once

#include "msrsb_internal.h"

namespace msrsb {

struct TpFluid {
    double mu_w, mu_o, n_w, n_o;
};

constexpr int kTpRed = 1024;  // fixed grid of the full-system dot products

struct TpCtx {
    Ctx *ms = nullptr;            // the pressure context (not owned)
    TpFluid fluid{};
    int restart = 30;
    int basis_sweeps = 0;
    bool assembled = false;
    // device: single-phase faces and well indices (the pressure context's
    // operator is replaced by the IMPES one), active mask, pore volumes
    double *T0 = nullptr, *WI0 = nullptr, *pv = nullptr;
    uint8_t *act = nullptr;
    // residual [2N], Jacobian rows (diagonal [4N], neighbours [6][N][4]),
    // block ILU(0) pivots inverted [4N], IMPES coefficients [3N] + [n_bc]
    double *R = nullptr, *Jd = nullptr, *Jo = nullptr, *Pinv = nullptr, *teff = nullptr, *bceff = nullptr;
    // CPR work: pressure rhs and correction [N], stage-2 residual [2N]
    double *vp = nullptr, *dp = nullptr, *r2 = nullptr;
    // GMRES: basis [(m+1) 2N], preconditioned vectors [m 2N], w [2N],
    // partial dots, device coefficients
    double *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr, *h = nullptr;
    std::vector<void *> bufs;
};

void tp_launch_assemble(TpCtx &t, double dt, const double *p, const double *s, const double *s_old, const double *q);
void tp_launch_ilu(TpCtx &t, int *flag);
void tp_launch_matvec(TpCtx &t, const double *x, double *out);
void tp_launch_cpr(TpCtx &t, const double *v, double *y);
void tp_launch_update(TpCtx &t, const double *dx, double *p, double *s);
void tp_launch_dots(TpCtx &t, const double *V, int k, const double *w, double *h);
void tp_launch_multiaxpy(TpCtx &t, const double *V, int k, const double *h, double sign, double *w);
void tp_launch_scale(TpCtx &t, const double *a, double f, double *b);

}  // namespace msrsb
