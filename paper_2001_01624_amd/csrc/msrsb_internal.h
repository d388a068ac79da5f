// Internal declarations of the MI355X MsRSB library: context layout and the
// launchers each kernel file provides.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/msrsb.h"

namespace msrsb {

constexpr int kBlock = 256;        // threads per workgroup of the streaming kernels
constexpr int kRedBlocks = 2048;   // fixed grid of the norm/dot kernels (deterministic order)
constexpr int kTile = 64;          // coarse inverse tile / panel width
constexpr int kMaxRestart = 64;
constexpr int kMaxXSlots = 32;   // slots per cell of an explicit (fault-cut) stage
constexpr int kXNibSlots = 15;   // explicit stages up to this many slots keep packed neighbour maps
constexpr int kMaxXBlocks = 32768;  // blocks of an explicit stage (dense coarse operator)
constexpr int kXChunk = 2048;    // support-list entries per restriction workgroup (explicit stages)
constexpr int kXRapChunk = 8192; // support-list entries per Galerkin-row wavefront (at most)
constexpr int kXRapChunkMin = 1024;  // shortest Galerkin-row chunk of an explicit stage
// bytes of Galerkin partial rows an explicit stage of `entries` support
// entries and Mp padded blocks may hold: what the longest chunks need, or
// 16 bytes per entry (room for the shorter chunks) if that is more
inline size_t xrap_part_bytes(size_t entries, long Mp) {
    const size_t b = (2 * entries / kXRapChunk + 1) * (size_t)Mp * 8;
    return b > 16 * entries ? b : 16 * entries;
}

// Geometry of the fine box as the kernels see it.
struct Fine {
    int nx, ny, nz, nxy;
    int N;
    const double *tx, *ty, *tz;   // face T to the +x/+y/+z neighbour
    const double *diag;           // A_ii (0 marks an inactive cell)
};

// Rectilinear stage tables (device).  For axis d with n_d cells and m_d
// blocks: blk[i] = floor(i m/n); lo[i] = first block whose 1-D support holds
// i; nv[i] in {1,2} = how many consecutive blocks from lo hold it;
// slo/shi[J] = inclusive 1-D support range of block J.
struct CartDev {
    int n[3], m[3];
    int bit[3];                   // slot bit of axis d, -1 if m_d == 1
    int ns;                       // slots per cell = 2^(#axes with m_d > 1)
    const int32_t *lo[3], *nv[3], *slo[3], *shi[3];
    const int32_t *be[3];         // block start per axis (m+1 entries)
    const int32_t *split[3];      // per block: first cell whose first support block is the block itself
    const int32_t *pack[3];       // per cell: lo | (nv==2)<<20 | (lo[c]-lo[c-1])<<21 | (lo[c+1]-lo[c])<<22
    const uint64_t *xmask;        // per run of 64 x cells: bits 20, 21, 22 of pack[0] as three masks
    const int32_t *cmap;          // Cartesian block -> compact id (-1 dropped)
    const int32_t *present;       // compact id -> Cartesian block
};

struct Stage {
    int kind = 0;                 // 0 general (Cartesian), 2 explicit slots (fault cut or graph), 3 dynamic
    bool graph = false;           // explicit-slot stage built from a caller's block vector
    int M = 0, Mp = 0;            // blocks; padded to a multiple of kTile
    int ns = 1;                   // slots per cell
    // Cartesian tables
    CartDev cart{};
    int32_t *d_tab = nullptr;     // one allocation holding every table
    std::vector<int32_t> h_present;
    std::vector<int32_t> h_tab;   // host copy of the tables (export, checks)
    int tab_off[3][7] = {};       // offsets of lo/nv/slo/shi/be/split/pack per axis in h_tab
    int32_t *gbase = nullptr;     // [m0*m1*m2+1] active cells before each Cartesian block
    // basis values, slot-major [ns*N]
    double *P64[2] = {nullptr, nullptr};
    float *P32[2] = {nullptr, nullptr};
    uint16_t *Pbf = nullptr;      // BF16 storage (mixed precision)
    int cur = 0;                  // buffer holding the current basis
    bool has_basis = false;
    int sweeps = 0;
    double change = 0.0;
    // dynamic (constant basis)
    int32_t *dblock = nullptr;    // [N] block per cell (-1 inactive)
    int32_t *dptr = nullptr;      // [M+1] CSR of cells per block
    int32_t *dcells = nullptr;    // [n_active]
    // coarse operator and its inverse (Mp x Mp, row-major), coarse vectors
    double *Ac = nullptr, *Ainv = nullptr;
    double *dvec = nullptr, *pc = nullptr;
    // rectilinear stages hold p_c per Cartesian block (zero on dropped
    // blocks); the coarse solve writes entry j at pc_map[j]
    const int32_t *pc_map = nullptr;
    // restriction partial sums per (layer, dual interval, slot); Galerkin
    // partial sums per dual box
    double *rpart = nullptr;
    double *rap_part = nullptr;
    int zwide = 0;                // widest dual z-interval (layers)
    // explicit-slot stage (fault cut): slot tables, piece of each cell,
    // per-block support lists (cells ascending, with the block's slot there)
    int parent = -1;
    int32_t *xsb = nullptr, *xpblock = nullptr, *xptr = nullptr, *xcell = nullptr;
    // per cell: its slot count, and for each of its six faces and each of its
    // slots the slot of the same block in the face neighbour's list (255: none)
    uint8_t *xcnt = nullptr, *xnmap = nullptr;
    // the same maps packed four bits per slot, one word per cell and face
    // (15: none), for stages of at most kXNibSlots slots (xnmap is then null)
    uint64_t *xnib = nullptr;
    // the basis value of every support-list entry, in list order (working
    // precision of the transfers: BF16 or FP64), rebuilt after each sweep run
    void *xplist = nullptr;
    int nxent = 0;                // support-list entries
    uint8_t *xslot = nullptr;
    // the support lists cut into chunks of at most kXChunk entries (restriction)
    // and kXRapChunk entries (Galerkin rows): block of each chunk, first chunk
    // of each block; Galerkin chunks of blocks with more than one chunk sum
    // into partial rows (xrrow: row of each chunk, -1 = straight into A_c)
    int nxch = 0, nxrch = 0, nxrrow = 0;
    int xrchunk = kXRapChunk;     // entries per Galerkin-row chunk
    int32_t *xcblk = nullptr, *xcfirst = nullptr;
    int32_t *xrcblk = nullptr, *xrcfirst = nullptr, *xrrow = nullptr;
    double *xpart = nullptr, *xrpart = nullptr;
    // finite-volume mode: the stage's own blocks as cell lists, position of
    // each cell in its list, explicit slot table of a rectilinear stage
    // (-1 = slot unused), the operator R_fv A P and its inverse, Galerkin-style
    // chunk tables over the own-cell lists; fv_version is the basis version
    // the operator was built from
    bool fv_ready = false;
    int fv_version = -1, fv_maxcells = 0;
    int32_t *fvblock = nullptr, *fvptr = nullptr, *fvcells = nullptr, *fvloc = nullptr, *fvsb = nullptr;
    int nfvrch = 0, nfvrrow = 0;
    int32_t *fvrcblk = nullptr, *fvrcfirst = nullptr, *fvrrow = nullptr;
    double *fvrpart = nullptr, *Afv = nullptr, *Afvinv = nullptr;
    int version = 0;              // incremented whenever the basis or the operator changes
    std::vector<int32_t> h_xsb, h_xpblock;
};

struct Status {                   // device-side solver status (one struct per context)
    int done;                     // 1: converged or finished -> later kernels return
    int iters;                    // iterations completed
    int flag;                     // error bits (1: singular pivot, 2: row sum <= 0)
    int jcur;                     // GMRES: inner index of the next Arnoldi step
    int skip2;                    // GMRES: 1 = second Gram-Schmidt pass not needed (or done)
    double relres;
    double bnorm;
    double change_bits_dummy;
};

struct Ctx {
    hipStream_t stream = nullptr;
    // launch timing of one kernel class (msrsb_profile_begin/end)
    int prof_class = -1;
    std::vector<hipEvent_t> prof_ev;  // pairs: start, stop
    int prof_used = 0;
    int device = 0;
    msrsb_options opt{};
    int nx = 0, ny = 0, nz = 0, N = 0, n_active = 0;
    // host copies needed later (dynamic stages, export)
    std::vector<uint8_t> h_active;
    std::vector<uint8_t> h_fault;   // [3N] or empty
    std::vector<int32_t> h_bc_cell;
    std::vector<double> h_bc_trans, h_bc_value;
    int n_bc = 0;
    // device operator
    double *tx = nullptr, *ty = nullptr, *tz = nullptr;   // FP64
    float *tx32 = nullptr, *ty32 = nullptr, *tz32 = nullptr;
    double *diag = nullptr, *b = nullptr, *src = nullptr;
    double *bcdiag = nullptr, *bcrhs = nullptr;
    double *dtil = nullptr;       // red-black ILU(0) pivots
    float *dtil32 = nullptr, *diag32 = nullptr;
    // z-line red-black ILU(0): inverse pivots and Tz_{k-1} / p_{k-1} per cell
    double *ldinv = nullptr, *lcz = nullptr;
    float *ldinv32 = nullptr, *lcz32 = nullptr;
    // its register path's colour-packed factors [colour][1/p, cz, Tz/p][slot] and
    // corrections [colour][slot], in the working precision (null: not used)
    void *lpack = nullptr, *lpe = nullptr;
    int32_t *bc_cell = nullptr;
    double *bc_trans = nullptr, *bc_value = nullptr;
    int32_t *bcptr = nullptr, *bcidx = nullptr;  // connections grouped by cell ([N+1], [n_bc])
    // work vectors [N]
    double *r = nullptr, *e = nullptr, *tmp = nullptr, *z = nullptr, *u = nullptr;
    double *partial = nullptr;    // [kRedBlocks * (2 * kMaxRestart + 2)]
    double *cbuf = nullptr;       // coarse inverse column panel [cbuf_n * kTile], then 2 kTile^2 block inverses
    long cbuf_n = 0;
    double *scal = nullptr;       // small device scalars / GMRES Hessenberg state
    Status *status = nullptr;     // device
    Status *h_status = nullptr;   // pinned host mirror
    unsigned long long *maxbits = nullptr;  // device max |change| bit pattern
    int *flag = nullptr;          // device error flag
    // GMRES Krylov basis [(restart+1) * N]; with an FP32 basis (Vf, mixed
    // precision and the DCGS2 path) V holds only the two candidate vectors
    // u_j [2 * N] and Vf the basis [restart * N]
    double *V = nullptr;
    double *Z = nullptr;          // DCGS2: preconditioned candidates M^-1 u_j, one per column
    float *Vf = nullptr;
    std::vector<Stage> stages;    // general + static
    std::vector<Stage> dyn;       // dynamic, newest first
    std::vector<void *> allocs;   // every device allocation (freed at destroy)
    std::vector<size_t> alloc_bytes;  // their sizes (the caller's allocator is told them)
    msrsb_allocator ua{};         // caller's device allocator (ua.alloc == NULL: the library's pool)
    // set-up arena: one allocation that the set-up's buffers are carved from
    // (256-byte aligned); later allocations, and any that do not fit, are
    // allocations of their own
    char *arena = nullptr;
    size_t arena_size = 0, arena_off = 0;
    bool arena_open = false;
};

// Brackets the launches of one kernel class with HIP events when that class
// is being timed.
// For launches timed by the dispatch itself (hipExtLaunchKernelGGL): the
// next event pair of class cls, or null events when that class is not being
// profiled.
inline void prof_pair(Ctx &c, int cls, hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    if (c.prof_class == cls && c.prof_used + 2 <= (int)c.prof_ev.size()) {
        *e0 = c.prof_ev[c.prof_used];
        *e1 = c.prof_ev[c.prof_used + 1];
        c.prof_used += 2;
    }
}

struct ProfScope {
    Ctx &c;
    bool on;
    ProfScope(Ctx &cc, int cls) : c(cc), on(cc.prof_class == cls && cc.prof_used + 2 <= (int)cc.prof_ev.size()) {
        if (on) (void)hipEventRecord(c.prof_ev[c.prof_used], c.stream);
    }
    ~ProfScope() {
        if (on) {
            (void)hipEventRecord(c.prof_ev[c.prof_used + 1], c.stream);
            c.prof_used += 2;
        }
    }
};

// ---- error helpers (capi.hip) ----
void set_error(const char *fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char *what);

// ---- fine-grid kernels (k_fine.hip) ----
void launch_assemble(Ctx &c);
void launch_source_update(Ctx &c, const double *d_source);
void launch_ilu_factor(Ctx &c);
void launch_residual(Ctx &c, const double *b, const double *x, double *r, bool norm, const int *done);
void launch_matvec(Ctx &c, const double *x, double *y, bool norm, const int *done);
void launch_smooth(Ctx &c, const double *r, double *x, const int *done, bool assign = false);
void launch_lilu_factor(Ctx &c);
void launch_lilu_apply(Ctx &c, const double *r, double *x, const int *done, bool assign);
int lilu_reg_chunks(int nz);                          // 0: columns too tall for the register path
size_t lilu_slots(int nx, int ny, int nz);            // packed slots of one colour
void launch_dgmres_step(Ctx &c, const double *z, double *w, const double *u, int j, double rtol, int max_iters,
                        bool final_);
constexpr int kDcgsMax = 31;  // largest restart served by the DCGS2 kernels
// c.scal regions of the DCGS2 solution update: the triangle T with
// M^-1 Q = Z T^-1 (column-major, ld kDcgsMax + 1) and the coefficients T^-1 y
constexpr int kScalT = 13000, kScalW = 14100;
void launch_zero_inactive(Ctx &c, double *x);
void launch_norm_finish(Ctx &c, double *out_sq, const int *done);
void launch_check(Ctx &c, double rtol, int max_iters, int count);
void launch_gmres_begin(Ctx &c, double rtol, int max_iters);
void launch_begin_solve(Ctx &c, const double *b, double *x);
void launch_symmetrize(Ctx &c, double *A, int M, int Mp);
size_t rap_part_doubles(int ns, int nbox);
void *ctx_alloc(Ctx &c, size_t bytes);
void ctx_free(Ctx &c, void *p);
void launch_fluxes(Ctx &c, const double *p, double *face, double *bcf);
// GMRES helpers
void launch_multidot(Ctx &c, const double *V, int k, const double *w, double *h_out, const int *done);
void launch_multiaxpy(Ctx &c, const double *V, int k, const double *h, double *w, double sign, bool norm,
                      const int *done);
void launch_multiaxpy(Ctx &c, const float *V, int k, const double *h, double *w, double sign, bool norm,
                      const int *done);
void launch_gmres_start(Ctx &c, const double *r, double *v0, int restart);
void launch_gmres_step(Ctx &c, int j, double rtol, int max_iters, int restart);
void launch_gmres_scale(Ctx &c, const double *w, double *v, int j);
void launch_gmres_solve_small(Ctx &c, int restart, bool zform = false);
void launch_axpy(Ctx &c, double *x, const double *z, const int *done);
void launch_reorth_check(Ctx &c, int k);
void launch_arnoldi(Ctx &c, const double *z, double *w, int j, double rtol, int max_iters, int restart);

// ---- basis kernels (k_sweep.hip, k_transfer.hip) ----
int launch_sweeps(Ctx &c, Stage &s, int max_sweeps, double tol, bool warm, int *sweeps, double *change);
void launch_restrict(Ctx &c, Stage &s, const double *r, const int *done);
void launch_residual_restrict(Ctx &c, Stage &s, const double *b, const double *x, const int *done);
void launch_prolong(Ctx &c, Stage &s, double *x, const int *done);
void launch_rap(Ctx &c, Stage &s);
void launch_export_cart(Ctx &c, Stage &s, double *d_vals);
void launch_export_bf16(Ctx &c, const uint16_t *d_in, long n, double *d_out);

// ---- coarse kernels (k_coarse.hip) ----
void launch_coarse_inverse(Ctx &c, Stage &s);
void launch_coarse_solve(Ctx &c, Stage &s, const int *done);

// ---- explicit-slot stage kernels (k_explicit.hip) ----
void launch_xinit(Ctx &c, Stage &s);
void launch_xmap_build(Ctx &c, Stage &s);
int launch_xsweep(Ctx &c, Stage &s, int in, int out);
void launch_xrestrict(Ctx &c, Stage &s, const double *r, const int *done);
void launch_xprolong(Ctx &c, Stage &s, double *x, const int *done);
void launch_xrap(Ctx &c, Stage &s);
void launch_xlist(Ctx &c, Stage &s);

// ---- finite-volume restriction and flux reconstruction (k_fv.hip) ----
constexpr int kFvMaxCells = 8192;  // cells of one block in the local solves (LDS-resident direction)
void launch_fv_rap(Ctx &c, Stage &s);
void launch_fv_restrict(Ctx &c, Stage &s, const double *b);
int launch_fv_local(Ctx &c, Stage &s, const double *pms, double *pf, double rtol, int max_iters, int *iters_max);
void launch_fv_faces(Ctx &c, Stage &s, const double *pms, const double *pf, double *face);
void launch_fv_imbalance(Ctx &c, const double *face, const double *pf, unsigned long long *maxbits);
void launch_coarse_inverse_of(Ctx &c, const double *A, double *Ainv, int Mp, bool general);
void launch_coarse_solve_with(Ctx &c, Stage &s, const double *Ainv, const int *done);

// ---- two-phase CPR hooks (capi.hip) ----
void ms_precondition(Ctx &c, const double *r, double *x);
int set_operator_device(Ctx &c, const double *d_t3, const double *d_bc);
int refresh_bases(Ctx &c, int sweeps);

// ---- dynamic basis kernels (k_dyn.hip) ----
int build_dynamic_stage(Ctx &c, const double *dp, Stage &out, int *count);
void launch_dyn_restrict(Ctx &c, Stage &s, const double *r, const int *done);
void launch_dyn_prolong(Ctx &c, Stage &s, double *x, const int *done);
void launch_dyn_rap(Ctx &c, Stage &s);

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace msrsb

// the public context handle is the context itself
struct msrsb_ctx : public msrsb::Ctx {};
