/*
 * msrsb.h - C ABI of the MI355X multiscale restricted-smoothing (MsRSB)
 * pressure solver.
 *
 * The library solves the single-phase pressure system A p = q of a two-point
 * flux (TPFA) discretisation on a Cartesian box, as posed in the paper's
 * "Multiscale methods" section (eq. pressure_system), by the iterative
 * multiscale-multibasis method of its subsection "Iterative multiscale
 * multibasis solver" (eq. multiscale-multibasis): a sequence of
 * prolongation/restriction pairs (P^l, R^l = (P^l)^T), each with its own
 * smoother step and Galerkin coarse correction (eq. pressure_system_reduced).
 * Paper: Klemetsdal, Moyner & Lie, arXiv 2001.01624.
 *
 * Conventions shared by every call:
 *  - Cells are numbered in the full box, x fastest: idx = i + nx*(j + ny*k).
 *    Inactive cells keep their index; every per-cell array has N = nx*ny*nz
 *    entries and the library writes 0 to inactive entries of its outputs.
 *  - "host" arrays are read during the call only and copied; the caller
 *    keeps ownership.  "device" arrays are HIP device pointers on the
 *    context's device; they must stay valid until the call returns (calls
 *    are synchronous with respect to the host unless named *_async).
 *  - Every call returns MSRSB_OK (0) or a negative status; the message of
 *    the last failure on the calling thread is msrsb_last_error().
 *  - A context is not thread-safe.  Distinct contexts may be used from
 *    distinct threads at the same time, each on its own stream.
 *  - All device work of a context runs on the stream given at setup (or the
 *    null stream).  Device memory comes from the allocator given at setup
 *    (msrsb_allocator) or, without one, stream-ordered from the device's
 *    default memory pool: at setup one arena of about msrsb_footprint_bytes
 *    that the set-up buffers are carved from (anything beyond it is
 *    allocated on its own), and further blocks when dynamic bases are added
 *    or a stage is exported.  Pool arenas of destroyed contexts are kept
 *    (at most 4 GiB per device, until the process ends) and reused by later
 *    set-ups that need at least three quarters of one.
 */
#ifndef MSRSB_H
#define MSRSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MSRSB_OK = 0,
    MSRSB_E_INVAL = -1,    /* malformed input (sizes, NaN, negative T, ...) */
    MSRSB_E_NOMEM = -2,    /* device allocation failed */
    MSRSB_E_DEVICE = -3,   /* a HIP call failed */
    MSRSB_E_SINGULAR = -4, /* A or a coarse operator is singular / not SPD,
                              or a basis row sum is not positive */
    MSRSB_E_NOCONV = -5,   /* tolerance not met within the iteration limit;
                              the outputs hold the last iterate */
    MSRSB_E_STATE = -6     /* call out of order (e.g. solve before basis) */
};

/* Opaque solver context; owns every device allocation of one problem. */
typedef struct msrsb_ctx msrsb_ctx;

/*
 * Fine grid and its two-point operator (paper section "Discrete equations":
 * two-point flux approximation; mobility 1).  The operator is
 *   A_ii = sum of T over the faces of i + sum of bc_trans on i,
 *   A_ij = -T_f for the face f between i and j,
 *   b_i  = source_i + sum of bc_trans*bc_value on i.
 * All arrays are HOST arrays.
 */
typedef struct {
    int32_t nx, ny, nz;        /* box size, each >= 1 */
    const uint8_t *active;     /* [N] 1 = active, 0 = inactive; NULL = all active */
    const double *tx;          /* [N] T of the face between i and i+1 (x); 0 = none */
    const double *ty;          /* [N] T of the face between i and i+nx (y) */
    const double *tz;          /* [N] T of the face between i and i+nx*ny (z) */
    const uint8_t *fault;      /* [3*N] fault[d*N+i] = 1 if the +d face of i lies on
                                  a fault (used by FAULT_CUT partitions); may be NULL */
    int32_t n_bc;              /* Dirichlet faces and bottom-hole-pressure connections */
    const int32_t *bc_cell;    /* [n_bc] cell of each connection (active) */
    const double *bc_trans;    /* [n_bc] >= 0 */
    const double *bc_value;    /* [n_bc] prescribed pressure */
    const double *source;      /* [N] injection rate q (> 0 injects); NULL = 0 */
} msrsb_grid;

/*
 * Coarse partitions (paper "Multiscale methods": requirements 1-3 on each
 * operator pair; "General" and "Static" partition types).
 *   CARTESIAN: rectilinear blocks, cell i of an axis of n cells goes to block
 *     floor(i*m/n); blocks without active cells are dropped.  Supports: per
 *     axis, i is in S_J iff 2c_{J-1} < 2i+1 < 2c_{J+1}, 2c_J = e_J + e_{J+1},
 *     e_J = ceil(J*n/m); the support is the product of the three axis sets,
 *     restricted to active cells.  The first partition must be CARTESIAN.
 *   FAULT_CUT: the connected pieces of each block of stage `parent` over the
 *     faces not on a fault, numbered by (parent block, smallest cell); the
 *     support of a piece is the part of its parent's support reachable from
 *     it without crossing a fault face.
 */
/*   GRAPH: any partition given as a block id per cell (a graph partitioner's
 *     output, or the well and indicator partitions of msrsb_partition_wells
 *     and msrsb_partition_indicator): ids >= 0 on active cells (inactive
 *     entries are ignored), blocks numbered by ascending id with unused ids
 *     dropped.  The support of a block is every active cell within `overlap`
 *     face steps of the block (faces with T > 0); overlap 0 keeps the block
 *     itself, i.e. a constant basis.  At most 32 supports may hold a cell.
 */
enum { MSRSB_PART_CARTESIAN = 0, MSRSB_PART_GRAPH = 1, MSRSB_PART_FAULT_CUT = 2 };
typedef struct {
    int32_t kind;
    int32_t coarse_dims[3];    /* CARTESIAN: blocks per axis, 1 <= m <= n */
    int32_t parent;            /* FAULT_CUT: index of the parent stage */
    const int32_t *block_of_cell; /* GRAPH: host [N] block id per cell (read during setup only) */
    int32_t overlap;           /* GRAPH: support reach in face steps, >= 0 */
} msrsb_partition;

/* Smoothers: damped Jacobi; ILU(0) in red-black cell order (the colour of a
 * cell is the parity of i+j+k, red = even first); ILU(0) in z-line red-black
 * order (whole columns (i, j) coloured by the parity of i+j, red columns
 * first, each column's cells in ascending k: columns are solved along z,
 * which suits strong vertical coupling). */
enum { MSRSB_SMOOTH_JACOBI = 0, MSRSB_SMOOTH_ILU0_RB = 1, MSRSB_SMOOTH_ILU0_LINE = 2 };
enum { MSRSB_FP64 = 0, MSRSB_MIXED = 1 };
enum { MSRSB_RICHARDSON = 0, MSRSB_GMRES = 1 };

typedef struct {
    double omega;           /* basis damping, default 2/3 */
    double omega_s;         /* Jacobi smoother damping, default 2/3 */
    int32_t smoother;       /* MSRSB_SMOOTH_*; default JACOBI */
    int32_t precision;      /* MSRSB_FP64 (default) or MSRSB_MIXED: FP32 basis
                               sweeps and smoother, BF16 basis storage; residual,
                               norms, coarse operators and coarse solves in FP64 */
    int32_t n_bins;         /* dynamic-basis bins, default 4 */
    int32_t max_dyn_blocks; /* cap on blocks of one dynamic stage, default 4096 */
    int32_t outer;          /* MSRSB_RICHARDSON (default) or MSRSB_GMRES */
    int32_t restart;        /* GMRES restart length, default 30, <= 64 */
} msrsb_options;

/* Fill *opt with the defaults listed above. */
void msrsb_default_options(msrsb_options *opt);

/* Device bytes msrsb_setup will allocate for this input (dynamic stages
 * excluded: each adds about 8*N + 16*M^2 bytes, M padded to a multiple of
 * 64).  Returns 0 on invalid input, including grids the kernels cannot
 * address: N = nx*ny*nz at most (2^31 - 1)/8 cells, and for every stage
 * (slots per cell) * N * 8 bytes below 2^31 (a 3-D rectilinear stage has 8
 * slots per cell, so N <= 33,554,431 there). */
size_t msrsb_footprint_bytes(const msrsb_grid *grid, int n_part, const msrsb_partition *parts,
                             const msrsb_options *opt);

/*
 * Device memory source of a context.  alloc returns `bytes` of device memory
 * on the context's device, aligned to at least 256 bytes, usable in the order
 * of `hip_stream` (the context's stream), or NULL on failure; free returns a
 * block from alloc with its size.  Both are called from the thread that
 * calls into the library, during msrsb_setup, msrsb_add_dynamic_basis,
 * msrsb_export_stage and msrsb_destroy.  `user` is passed through.  (The
 * Python binding passes PyTorch's caching allocator here.)
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *hip_stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *hip_stream, void *user);
    void *user;
} msrsb_allocator;

/*
 * Validate the grid, assemble A and b on the device (two-point operator, see
 * msrsb_grid), build every partition and support, and factor the smoother.
 * alloc: the context's device allocator (copied), or NULL for the library's
 * own: stream-ordered allocations from the device's default memory pool.
 * hip_stream: a hipStream_t (NULL = null stream); every device operation of
 * the context, its allocations included (the set-up buffers share one
 * arena), runs on that stream, and msrsb_setup returns after synchronising it
 * alone.  On success *out owns all device memory of the context.  Errors:
 * E_INVAL (bad sizes, non-finite or negative T, a face touching an inactive
 * cell or leaving the box, a BC on an inactive cell, an allocator without
 * both functions), E_SINGULAR (an active connected component without any bc
 * connection), E_NOMEM, E_DEVICE.
 */
int msrsb_setup(const msrsb_grid *grid, int n_part, const msrsb_partition *parts,
                const msrsb_options *opt, const msrsb_allocator *alloc, void *hip_stream, msrsb_ctx **out);

/*
 * Build the restricted-smoothing basis of one stage (stage >= 0) or of every
 * general/static stage (stage = -1), then its Galerkin coarse operator
 * A_c = P^T A P and the coarse inverse.  The basis starts from the block
 * indicator (warm = 0) or from the current basis (warm = 1: "a few extra"
 * smoothing iterations for local updates, subsection "Iterative multiscale
 * multibasis solver").  Sweeps stop after the first sweep whose largest
 * entry change is <= tol, or after max_sweeps (>= 0).  sweeps_done and
 * last_change (may be NULL) report the last stage processed.
 * new_trans (host [3N]: tx, ty, tz as in msrsb_grid, or NULL to keep) and
 * new_bc_trans (host [n_bc]: the connections' bc_trans, or NULL to keep):
 * the operator's coefficients change first ("changing reservoir/fluid
 * properties", same subsection), validated as at setup; A, b and the
 * smoother are rebuilt, the stages named by `stage` are smoothed with the
 * new operator (warm = 1 continues from their current basis: the local
 * update), and every other stage, dynamic ones included, keeps its basis
 * and gets its coarse operator and inverse rebuilt for the new A.
 * Partitions and supports keep the structure of setup.
 * Errors: E_INVAL, E_SINGULAR (row sum <= 0, A_c not SPD, or new_trans
 * leaves a component without a boundary connection), E_STATE (warm start
 * of a stage without a basis), E_DEVICE.
 */
int msrsb_update_basis(msrsb_ctx *ctx, int stage, const double *new_trans, const double *new_bc_trans,
                       int max_sweeps, double tol, int warm, int *sweeps_done, double *last_change);

/*
 * Dynamic stages (subsection "Iterative multiscale multibasis solver", type
 * "Dynamic"; constant basis functions).  d_dp[k] (device, [N] doubles) are
 * pressure increments, newest first, n_incr in {1, 2}.  For each: a = |dp|,
 * cells get bin = #{k = 1..n_bins-1 : a <= ldexp(max a, -2k)}, cells with
 * the same (stage-0 block, bin) key that are face connected form one block,
 * blocks are numbered by (stage-0 block, smallest cell index); if more than
 * max_dyn_blocks result, n_bins is halved and the binning repeated (E_INVAL
 * if even one bin gives more; no stage of that call is kept then).  An
 * increment with max |dp| = 0 or non-finite adds no stage (count 0).
 * Replaces any previous dynamic stages.  n_dyn_blocks[k] (host, may be NULL)
 * receives the block count of each increment.
 */
int msrsb_add_dynamic_basis(msrsb_ctx *ctx, int n_incr, const double *const *d_dp, int *n_dyn_blocks);

/* Remove all dynamic stages. */
int msrsb_clear_dynamic_basis(msrsb_ctx *ctx);

/*
 * Solve A p = b to ||b - A p||_2 <= rtol * ||b||_2 (||b|| = 1 if b = 0).
 * d_source: device [N] new source vector (b is rebuilt) or NULL to keep.
 * d_p: device [N], initial guess in, solution out.
 * outer = RICHARDSON: cycles of eq. multiscale-multibasis, stages in the
 * order general, static, dynamic (newest first); each stage applies the
 * smoother once to b - A x and then x += P A_c^{-1} P^T (b - A x); the test
 * runs after every full cycle.  outer = GMRES: restarted GMRES with one such
 * cycle (from a zero guess) as right preconditioner (section "Description of
 * the solution procedure").  max_iters bounds cycles / GMRES iterations.
 * iters, relres (host, may be NULL): iterations used and the relative
 * residual ||b - A p||_2 / ||b||_2 of the returned iterate, computed in FP64
 * from that iterate (for GMRES at the restart that ends the solve; the
 * least-squares estimate only decides when an inner cycle stops).  Returns
 * E_NOCONV with the last iterate in d_p if the limit is reached; E_STATE
 * before update_basis.
 */
int msrsb_solve(msrsb_ctx *ctx, const double *d_source, double *d_p, double rtol, int max_iters,
                int *iters, double *relres);

/*
 * Finite-volume multiscale solve with conservative fine fluxes (section
 * "Multiscale methods": when fine-scale fluxes are needed, a restriction that
 * sums the cells of each block instead of R = P^T).  For general or static
 * stage `stage` (0 .. number of general/static stages - 1, basis built):
 *   A_fv = R_fv A P (R_fv sums the stage's own blocks; not symmetric in
 *   general), inverted by the Gauss-Jordan sweep of the coarse solves without
 *   pivoting (rebuilt whenever the basis or the operator changed; a zero
 *   pivot is E_SINGULAR);
 *   d_p = P A_fv^{-1} R_fv b, the multiscale pressure, whose fluxes balance
 *   every block;
 *   inside every block the fine pressure p' solves the block's problem with
 *   the fluxes of d_p imposed on the faces leaving the block (conjugate
 *   gradients from p' = d_p, to ||r|| <= local_rtol ||rhs|| per block or
 *   max_local_iters steps; preconditioned by tridiagonal solves along the
 *   block's z lines for blocks of at most 2304 cells, by the diagonal for
 *   larger ones);
 *   d_face_flux [3N] (layout of msrsb_fluxes): T (p'_a - p'_b) on faces
 *   inside a block, T (p_a - p_b) on faces between blocks; d_bc_flux
 *   [n_bc] (may be NULL): bc_trans (p'_i - bc_value) from p'.
 * These fluxes balance every cell (outflow - q_i = 0) up to the local
 * solves' residual, provided each block is face-connected or anchored by a
 * boundary term.  d_source (device [N] or NULL) replaces the source first;
 * d_p_fine (device [N], may be NULL) receives p'.  local_iters (host, may be
 * NULL): the most conjugate-gradient steps any block took; max_imbalance
 * (host, may be NULL): max over cells of |outflow - q_i| of the returned
 * fluxes.  Blocks of at most 8192 cells (E_INVAL otherwise).  Device
 * vectors are the context's; E_STATE if the stage has no basis.
 */
int msrsb_solve_fv(msrsb_ctx *ctx, int stage, const double *d_source, double *d_p, double *d_p_fine,
                   double *d_face_flux, double *d_bc_flux, double local_rtol, int max_local_iters, int *local_iters,
                   double *max_imbalance);

/*
 * Asynchronous solve (eq. iterative_multiscale: the multistage cycle as a
 * stationary iteration, whatever the context's outer option): enqueues on
 * the context's stream, without any host synchronisation, the source update
 * (d_source device [N] or NULL), the initial residual and max_cycles cycles,
 * each followed by the residual test; once the test is met (or max_cycles
 * reached) the remaining enqueued kernels return at once.  d_p (device [N])
 * holds the guess and receives the iterate; the result is written on the
 * stream to d_result (device memory, may be NULL) when the enqueued work
 * ends: status MSRSB_OK or MSRSB_E_NOCONV, the cycles taken and the
 * relative residual.  The caller synchronises the stream before reading
 * d_p or d_result.  Returns E_INVAL (bad arguments, max_cycles outside
 * 1..100000) or E_STATE (no basis yet) at once; launch failures as
 * E_DEVICE.  Each enqueued cycle is about a dozen kernel launches, so
 * max_cycles should bound the expected count rather than exceed it
 * greatly.  The iterates are those of msrsb_solve with the Richardson outer
 * loop, bit for bit.
 */
typedef struct {
    int32_t status;   /* MSRSB_OK or MSRSB_E_NOCONV */
    int32_t cycles;   /* cycles taken */
    double relres;    /* ||b - A p|| / ||b|| of the returned iterate */
} msrsb_result;
int msrsb_solve_async(msrsb_ctx *ctx, const double *d_source, double *d_p, double rtol, int max_cycles,
                      msrsb_result *d_result);

/*
 * Ensemble batch: many independent contexts (the realisations of an
 * ensemble, each its own grid and operator) driven in lockstep, with one
 * kernel launch per step of the path over all members.  Every step is the
 * same computation as in the member's own calls (the paper's restricted
 * smoothing of "Iterative multiscale multibasis solver", the multistage
 * cycle of eq. multiscale-multibasis, GMRES), so each member's bases,
 * iterates, iteration counts and residuals are those of msrsb_update_basis
 * and msrsb_solve on that member alone, bit for bit; the batch only removes
 * the per-member launches that dominate small grids.
 *
 * msrsb_batch_create: members[0..n) (host array of n >= 1 distinct contexts,
 * 1 <= n <= 65536) are borrowed, not owned: they must outlive the batch and
 * must not be used on their own while a batch call runs.  Every member must
 * be on the current device with one rectilinear partition (kind CARTESIAN,
 * no dynamic stages), the GMRES outer loop with restart <= 31, the z-line
 * ILU(0) smoother with columns of at most 512 cells, and the same
 * precision, omega and restart as the others.  The members' streams are
 * switched to `hip_stream` (hipStream_t, NULL = null stream; each member's
 * old stream is synchronised first) and stay on it after the batch is
 * destroyed (a failed create leaves them on their own).  Errors: E_INVAL
 * (with the offending member in the message), E_NOMEM, E_DEVICE.
 *
 * msrsb_batch_update_basis: builds every member's basis from scratch (up to
 * max_sweeps sweeps each, member-wise stop at tol as in msrsb_update_basis
 * with warm = 0), then its Galerkin operator and coarse inverse.  sweeps
 * (host int32[n], may be NULL) receives the sweeps each member took.
 * Errors as msrsb_update_basis (E_SINGULAR names the first failing member).
 *
 * msrsb_batch_solve: for every member k, solves with source d_source[k]
 * (device [N_k]; a NULL array or entry keeps that member's current source)
 * from the guess in d_p[k] (device [N_k], receives the solution) to rtol
 * within max_iters iterations.  iters, relres and status (host arrays of n,
 * each may be NULL) receive each member's iteration count, final relative
 * residual and status (MSRSB_OK or MSRSB_E_NOCONV).  Returns MSRSB_OK when
 * every member converged, E_NOCONV when some did not (the others hold their
 * solutions), E_STATE before msrsb_batch_update_basis, E_INVAL, E_DEVICE.
 *
 * msrsb_batch_destroy frees the batch's own tables (not the members).  The
 * batch's tables (member descriptors and launch groups, a few hundred bytes
 * per member) come from hipMalloc / hipHostMalloc at create, not from the
 * members' allocators.  A batch is not thread-safe.
 */
typedef struct msrsb_batch msrsb_batch;
int msrsb_batch_create(int n, msrsb_ctx *const *members, void *hip_stream, msrsb_batch **out);
int msrsb_batch_update_basis(msrsb_batch *batch, int max_sweeps, double tol, int32_t *sweeps);
int msrsb_batch_solve(msrsb_batch *batch, const double *const *d_source, double *const *d_p, double rtol,
                      int max_iters, int32_t *iters, double *relres, int32_t *status);
void msrsb_batch_destroy(msrsb_batch *batch);

/*
 * Apply one operator of the path to a device vector (for testing single
 * steps; d_in, d_out device [N], distinct):
 *   op 0 RESIDUAL:  d_out = b - A d_in
 *   op 1 SMOOTH:    d_out = S(d_in), the smoother correction for residual d_in
 *   op 2 PRECOND:   d_out = one multistage cycle from zero with rhs d_in
 *   op 3 MATVEC:    d_out = A d_in
 */
enum { MSRSB_OP_RESIDUAL = 0, MSRSB_OP_SMOOTH = 1, MSRSB_OP_PRECOND = 2, MSRSB_OP_MATVEC = 3 };
int msrsb_apply(msrsb_ctx *ctx, int op, const double *d_in, double *d_out);

/*
 * Face fluxes v_f = T_f (p_a - p_b) in the structured layout
 * d_face_flux[d*N + i] (face between i and its +d neighbour) and
 * connection fluxes d_bc_flux[c] = bc_trans[c] (p_i - bc_value[c]) (device
 * arrays; either may be NULL).  Per-cell balance: outflow - q = -(b - A p).
 */
int msrsb_fluxes(msrsb_ctx *ctx, const double *d_p, double *d_face_flux, double *d_bc_flux);

/* Number of stages (general + static + dynamic) and, for one stage, its
 * block count M, its kind (0 rectilinear, 1 graph, 2 fault cut, 3 dynamic) and the
 * number of basis slots per cell. */
int msrsb_num_stages(msrsb_ctx *ctx);
int msrsb_stage_info(msrsb_ctx *ctx, int stage, int *M, int *kind, int *n_slots);

/*
 * Copy one stage to host arrays (tests and inspection):
 *   h_block [N]           block of each cell (-1 inactive)
 *   h_slot_block [S*N]    block held by slot s of cell i (-1 none), slot-major
 *   h_vals [S*N]          basis value of that slot, in FP64 (BF16 upcast)
 *   h_Ac [M*M]            Galerkin coarse operator, row-major
 * (S = n_slots; any pointer may be NULL).
 */
int msrsb_export_stage(msrsb_ctx *ctx, int stage, int32_t *h_block, int32_t *h_slot_block, double *h_vals,
                       double *h_Ac);

/*
 * Allocation-free form of msrsb_export_stage, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops
 * that checkpoint a resident basis, harnesses that forbid hipMalloc.  Same
 * arguments, outputs and errors as msrsb_export_stage, and it calls no
 * device allocator.  A BF16 (mixed-precision) basis is widened to FP64 one
 * slot column at a time through a staging array of MSRSB_NOALLOC_MAX_CELLS
 * doubles (16 MiB) that the library keeps in device memory: each device the
 * library runs on holds one such array until the process ends.  Grids of
 * more than MSRSB_NOALLOC_MAX_CELLS cells (nx*ny*nz) are rejected with
 * E_INVAL.  Every call on one device shares that device's array, so calls
 * that overlap on one device (contexts on different streams or threads)
 * race and must be serialised by the caller.
 */
#define MSRSB_NOALLOC_MAX_CELLS 2097152
int msrsb_export_stage_noalloc(msrsb_ctx *ctx, int stage, int32_t *h_block, int32_t *h_slot_block,
                               double *h_vals, double *h_Ac);

/*
 * Coarse solve of one stage (eq. pressure_system_reduced; section
 * "Computational efficiency": the coarse system solved directly): h_pc =
 * A_c^{-1} h_d with the explicit inverse built by msrsb_update_basis or
 * msrsb_add_dynamic_basis, applied by the same kernel every cycle uses.  Host
 * arrays of M entries (M from msrsb_stage_info), in the stage's block order.
 * For tests and inspection.  Errors: E_INVAL (no such stage), E_STATE (the
 * stage has no coarse operator yet), E_DEVICE.
 */
int msrsb_coarse_apply(msrsb_ctx *ctx, int stage, const double *h_d, double *h_pc);

/*
 * Static partitions for GRAPH stages (subsection "Iterative multiscale
 * multibasis solver", type "Static"; section "Numerical examples", Example 2:
 * well bases and partitions agglomerated from a flow indicator).  Host-only,
 * integer work; both write block[N] (host, caller-allocated) with -1 on
 * inactive cells, and return E_INVAL for an invalid grid or arguments.
 *
 * msrsb_partition_wells: one block per well plus one for the rest, so that
 *   the blocks cover the grid.  Cell i joins well w if its distance in face
 *   steps (faces with T > 0) to the cells of well w is at most `radius` and
 *   smaller than to any other well (ties to the lower well index); every
 *   other active cell joins block n_wells.  Well w's cells are
 *   well_cells[well_ptr[w] .. well_ptr[w+1]-1] (host; active cells, at least
 *   one per well).
 * msrsb_partition_indicator: agglomeration by a cell indicator (e.g. log
 *   permeability or a velocity magnitude, host [N], finite on active cells):
 *   (1) equal-count bins: active cells ranked by (indicator, cell index),
 *   bin = floor(rank * n_bins / n_active); (2) pieces: face-connected cells
 *   with the same (bin, rectilinear parent block of coarse_dims, as in
 *   CARTESIAN); (3) while a piece has fewer than min_cells cells and a
 *   face-neighbour piece in the same parent block, the smallest such piece
 *   (size, then smallest cell index) joins the neighbour piece it shares the
 *   most faces with (ties: the one with the smaller smallest cell index);
 *   (4) blocks numbered by their smallest cell index.
 */
int msrsb_partition_wells(const msrsb_grid *grid, int n_wells, const int32_t *well_ptr, const int32_t *well_cells,
                          int radius, int32_t *block);
int msrsb_partition_indicator(const msrsb_grid *grid, const double *indicator, int n_bins,
                              const int32_t coarse_dims[3], int min_cells, int32_t *block);

/*
 * Two-phase fully implicit model with the two-stage CPR preconditioner
 * (sections "Model equations" and "Discrete equations": water and oil, one
 * component each, backward Euler, two-point fluxes with single-point
 * upstream mobilities, no gravity or capillary pressure; section
 * "Preconditioning: the constrained pressure residual (CPR) method" and
 * "Description of the solution procedure").  Unknowns per cell: pressure p
 * and water saturation s.  Full-system vectors ([2N], device) interleave
 * them per cell in box numbering: v[2i] water equation / pressure, v[2i+1]
 * oil equation / saturation; inactive cells hold 0.  Residuals:
 *   R_w,i =  pv_i/dt (s_i - s_old,i) + sum_f T_f lw(up) (p_i - p_l)
 *            + sum_c WI_c lw(s_i) (p_i - p_c) - q_i
 *   R_o,i = -pv_i/dt (s_i - s_old,i) + sum_f T_f lo(up) (p_i - p_l)
 *            + sum_c WI_c lo(s_i) (p_i - p_c)
 * with T_f the pressure context's face transmissibilities at
 * msrsb_tp_create, WI_c / p_c its connections' bc_trans / bc_value, q the
 * injected water rate, lw = s^n_w / mu_w, lo = (1-s)^n_o / mu_o, and up the
 * cell a face's flux leaves (for the face a < b: a when p_a >= p_b).
 * CPR: IMPES weights (1/2, 1/2) cancel the accumulation derivatives, so the
 * pressure block is the two-point operator with face coefficients
 * T lambda_t(up)/2 and connection terms WI lambda_t/2, which
 * msrsb_tp_assemble installs in the pressure context (its bases smoothed
 * basis_sweeps more times from their current state: local updates).  One
 * preconditioner application: dp = one multistage cycle of the pressure
 * context on (v_w + v_o)/2, then y = (dp, 0) + ILU0(J)^{-1} (v - J (dp, 0))
 * with block ILU(0) of the full system in red-black cell order.
 * The two-phase context borrows the pressure context (which must outlive it
 * and whose bases must exist); its device memory comes from the pressure
 * context's allocator.
 */
typedef struct msrsb_tp_ctx msrsb_tp_ctx;
typedef struct {
    double mu_w, mu_o;  /* viscosities, > 0 */
    double n_w, n_o;    /* Corey exponents, >= 1 */
} msrsb_fluid;
/* pore_volume: host [N], > 0 on active cells; restart: GMRES restart length
 * in [1, 200]. */
int msrsb_tp_create(msrsb_ctx *pressure, const double *pore_volume, const msrsb_fluid *fluid, int restart,
                    msrsb_tp_ctx **out);
/* Residual and Jacobian at (d_p, d_s) (device [N]) with old saturation
 * d_s_old and injected rate d_q (device [N]; NULL = the pressure context's
 * source), the IMPES operator into the pressure context and the full-system
 * ILU(0).  d_res (device [2N], may be NULL) receives R; res_norm (host, may
 * be NULL) ||R||_2.  E_SINGULAR on a singular 2x2 ILU pivot, E_STATE if the
 * pressure bases do not exist. */
int msrsb_tp_assemble(msrsb_tp_ctx *tp, double dt, const double *d_p, const double *d_s, const double *d_s_old,
                      const double *d_q, int basis_sweeps, double *d_res, double *res_norm);
/* op 0: d_out = J d_in; op 1: d_out = CPR^{-1} d_in ([2N] device, distinct). */
int msrsb_tp_apply(msrsb_tp_ctx *tp, int op, const double *d_in, double *d_out);
/* GMRES(restart) on J dx = -R from dx = 0 with CPR as right preconditioner,
 * to ||-R - J dx||_2 <= rtol ||R||_2 (true residual, at a restart);
 * E_NOCONV with the last iterate after max_iters iterations. */
int msrsb_tp_solve(msrsb_tp_ctx *tp, double *d_dx, double rtol, int max_iters, int *iters, double *relres);
/* Newton update on active cells: p += dx_p, s = min(1, max(0, s + dx_s)). */
int msrsb_tp_update(msrsb_tp_ctx *tp, const double *d_dx, double *d_p, double *d_s);
/* Frees the two-phase context; call it before msrsb_destroy of its pressure
 * context (its device buffers are that context's allocations). */
void msrsb_tp_destroy(msrsb_tp_ctx *tp);

/*
 * Host-only helpers (no device needed):
 * msrsb_validate_grid: the checks msrsb_setup applies to a grid (E_INVAL,
 *   E_SINGULAR as documented there).
 * msrsb_axis_support: 1-D support tables of a rectilinear partition of n
 *   cells into m blocks (paper requirement 2; rule of msrsb_partition):
 *   lo[i] (host [n]) first block whose support holds cell i, nv[i] in {1,2}
 *   number of consecutive blocks from lo[i] whose supports hold it,
 *   slo[J], shi[J] (host [m]) first and last cell of the support of block J.
 *   Any pointer may be NULL.  E_INVAL unless 1 <= m <= n.
 */
/*
 * msrsb_faces_to_box: face-list input for box grids (the grid described by
 *   its cell pairs and face transmissibilities, section "Discrete
 *   equations": two-point fluxes over the faces shared by two cells).  Cells
 *   are numbered x fastest in an nx x ny x nz box; face f joins cells
 *   face_cells[2f] < face_cells[2f+1], which must be neighbours along x, y
 *   or z; face_trans[f] >= 0 and finite.  Writes the structured arrays of
 *   msrsb_grid: tx, ty, tz (host [N], caller-allocated) with the face's T at
 *   its lower cell and zero elsewhere.  E_INVAL for a pair that is not a box
 *   neighbour (grids that are not boxes are not supported), a repeated face,
 *   a cell outside the box or a negative or non-finite T; the outputs are
 *   then unspecified.
 */
int msrsb_faces_to_box(int32_t nx, int32_t ny, int32_t nz, int32_t n_faces, const int32_t *face_cells,
                       const double *face_trans, double *tx, double *ty, double *tz);
int msrsb_validate_grid(const msrsb_grid *grid);
int msrsb_axis_support(int n, int m, int32_t *lo, int32_t *nv, int32_t *slo, int32_t *shi);

/*
 * Launch timing (measurement support).  Between msrsb_profile_begin and
 * msrsb_profile_end every launch of one kernel class is bracketed by HIP
 * events on the context's stream (at most max_launches launches are
 * recorded).  msrsb_profile_end synchronises the stream and returns the
 * summed kernel time in milliseconds and the number of launches timed.
 */
enum {
    MSRSB_K_SWEEP = 1,     /* one restricted-smoothing sweep over all cells */
    MSRSB_K_RESIDUAL = 2,  /* r = b - A x */
    MSRSB_K_SMOOTH = 3,    /* smoother correction (both colours for ILU(0)) */
    MSRSB_K_RESTRICT = 4,  /* d = P^T r */
    MSRSB_K_PROLONG = 5,   /* x += P p_c */
    MSRSB_K_COARSE = 6,    /* p_c = A_c^{-1} d */
    MSRSB_K_ORTHO = 7,     /* one Gram-Schmidt pass: dots + update */
    MSRSB_K_MATVEC = 8,    /* y = A x */
    MSRSB_K_RAP = 9,       /* Galerkin coarse operator of one stage */
    MSRSB_K_INVERSE = 10,  /* coarse inverse of one stage */
    MSRSB_K_RESTRICT_ROWS = 11 /* the fine-grid pass of d = P^T (b - A x) on a
                                  rectilinear stage, without its final gather */
};
int msrsb_profile_begin(msrsb_ctx *ctx, int kernel_class, int max_launches);
int msrsb_profile_end(msrsb_ctx *ctx, double *total_ms, int *launches);

/* Change the stream used by later calls (hipStream_t).  The current stream
 * is synchronised first (its work and stream-ordered allocations complete).
 * Errors: E_INVAL (NULL ctx), E_DEVICE. */
int msrsb_set_stream(msrsb_ctx *ctx, void *hip_stream);

/* Synchronise the context's stream and return all its device memory to the
 * device's memory pool (or to the caller's allocator), in the stream's order
 * (no device-wide synchronisation; NULL is ignored); a pool arena may
 * instead be kept for a later set-up (see the conventions above). */
void msrsb_destroy(msrsb_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *msrsb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MSRSB_H */
