// Batched launches over the members of an ensemble (several independent
// contexts driven in lockstep).  A batched launch runs, for every member of
// a group, exactly the workgroups that member's own launch would run: the
// kernel maps its workgroup id to (member, workgroup id within the member's
// own grid) and calls the same kernel body with the member's arguments.  So
// every member computes what it computes alone, bit for bit, and one launch
// serves the whole ensemble.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msrsb_internal.h"

namespace msrsb {

// One member as the batched kernels see it (device array, one entry per
// member).  Pointers are the member context's own buffers; pw/pt are the
// working-precision operator and basis (FP32 / BF16 in mixed precision).
struct BMember {
    Fine g;                        // FP64 operator
    CartDev cd;                    // the member's rectilinear stage
    int M, Mp, ns;
    int G, GA;                     // reduction grid, pass-A grid of the Arnoldi step
    // sweep geometry of the batched sweep: x tiles, row groups, z chunks and
    // their length, workgroups
    int s_nxt, s_ngy, s_nzc, s_zc, s_nblk, check_blocks;
    // z-line ILU(0) register path
    int l_hx, l_ncol, l_cw, l_nch, l_L;
    long l_S;
    const void *wtx, *wty, *wtz;   // face T in the working precision
    const void *lpack;
    void *lpe;
    void *P[2];                    // sweep buffers (FP64 or FP32)
    int cur;                       // the one holding the final basis
    const void *Pt;                // basis the transfers read (FP64 or BF16)
    uint16_t *Pbf;
    double *rpart, *dvec, *pc;
    const int32_t *pc_map;
    double *Ac, *Ainv, *rap_part;  // coarse operator, its inverse, Galerkin partial sums
    double *cbuf;                  // inverse panel and pivot-block buffers
    long cbuf_n;
    const double *bcrhs;
    double *b, *src, *x, *r, *tmp, *V, *Z;
    float *Vf;
    double *partial, *scal;
    Status *status;
    unsigned long long *maxbits;
    int *flag;
    const double *q;               // source of the current solve
};

// Vectors of a member named by the host: kind | (index << 4).
enum : int { BV_B = 0, BV_X = 1, BV_R = 2, BV_TMP = 3, BV_U = 4, BV_Z = 5, BV_V0 = 6 };
__host__ __device__ constexpr int bvsel(int kind, int j) { return kind | (j << 4); }

// BV_U: the DCGS2 candidate u_j (V(j & 1) with an FP32 basis, V(j) with an
// FP64 one); BV_Z: the stored preconditioned candidate Z(j).
__device__ inline double *bvec(const BMember &d, int sel) {
    const int kind = sel & 15, j = sel >> 4;
    const long N = d.g.N;
    switch (kind) {
    case BV_B: return d.b;
    case BV_X: return d.x;
    case BV_R: return d.r;
    case BV_TMP: return d.tmp;
    case BV_U: return d.V + (d.Vf ? (long)(j & 1) : (long)j) * N;
    case BV_Z: return d.Z + (long)j * N;
    default: return d.V;
    }
}

// The members of one batched launch and the workgroup range of each:
// member mem[k] owns workgroups start[k] .. start[k+1]-1.  With one
// workgroup per member (direct) the lookup is the workgroup id itself.
struct BGroup {
    int n, total, direct;
    const int32_t *start;   // [n+1]
    const int32_t *mem;     // [n]
};

// Member and member-local workgroup of this workgroup; false if that member
// has left the batch (act[m] == 0).  nb = the member's own grid size.
__device__ inline bool bat_locate(const BGroup &gp, const int *act, int &m, int &lb, int &nb) {
    const int b = blockIdx.x;
    int k;
    if (gp.direct) {
        k = b;
    } else {
        int lo = 0, hi = gp.n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (gp.start[mid] <= b) lo = mid;
            else hi = mid;
        }
        k = lo;
    }
    m = gp.mem[k];
    lb = b - gp.start[k];
    nb = gp.start[k + 1] - gp.start[k];
    return act[m] != 0;
}

// Host side of a batch: the members, their device descriptors and the
// launch groups of every batched kernel.
struct Batch;

struct HGroup {
    BGroup g{};
    int key = 0;            // template key the group's members share
    size_t lds = 0;         // dynamic LDS of the launch (largest member's)
};

// launch groups of one kernel: members split by the template key
using Groups = std::vector<HGroup>;

struct Batch {
    hipStream_t stream = nullptr;
    int device = 0;
    int n = 0;
    bool mixed = false;
    int restart = 0;
    bool has_basis = false;
    std::vector<Ctx *> mem;
    std::vector<BMember> h_mem;
    BMember *d_mem = nullptr;
    int *d_act = nullptr, *h_act = nullptr;       // members still taking part
    Status *d_st = nullptr, *h_st = nullptr;      // gathered statuses
    int *d_flag = nullptr, *h_flag = nullptr;     // gathered error flags
    int32_t *d_tab = nullptr;                     // every group's start/mem lists
    // launch groups
    Groups one, cells, red, passa, lilu, rrows, gather, gemv, prolong, sweep, init, bf16, nofuse;
    Groups rapbox, rapgather, pad, gjcopy, gjpanel, gjupdate;
    int max_tiles = 0;             // largest coarse inverse (64-wide tiles)
};

// ---- batched launchers (each kernel file) ----
// k_fine.hip
void bat_source_update(Batch &B);
void bat_begin_solve(Batch &B);
void bat_restart_residual(Batch &B, double rtol, int max_iters);
void bat_dgmres_step(Batch &B, int j, double rtol, int max_iters, bool final_);
void bat_solution_update(Batch &B);
void bat_gather_status(Batch &B);
bool bat_member_fine(const Ctx &c, BMember &d);
// k_lineilu.hip: x = S r (assign) for the selected vectors
void bat_lilu_assign(Batch &B, int rsel, int xsel);
int bat_member_lilu(const Ctx &c, BMember &d);
// k_transfer.hip
void bat_residual_restrict(Batch &B, int bsel, int xsel);
void bat_prolong(Batch &B, int xsel);
void bat_member_transfer(const Ctx &c, const Stage &s, int grid[3], int key[3], size_t *lds);
// Galerkin operator: grids of the box pass, the gather and the identity
// padding (key: split-axis mask)
void bat_member_rap(const Stage &s, int grid[3], int *key);
void bat_rap(Batch &B);
// k_coarse.hip
void bat_coarse_solve(Batch &B);
int bat_member_gemv(const Stage &s, int *key);
// coarse inverse: grids of the copy, a panel step and an update step
void bat_member_inverse(const Stage &s, int grid[3]);
void bat_coarse_inverse(Batch &B);
// k_sweep.hip
void bat_sweep_begin(Batch &B, int max_sweeps);
void bat_sweep_pair(Batch &B, int k, int npair, double omega, double tol, int max_sweeps);
void bat_to_bf16(Batch &B);
int bat_member_sweep(const Ctx &c, const Stage &s, BMember &d, int *key);

}  // namespace msrsb
