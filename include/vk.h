/*
 * vk.h -- C ABI of the MI355X (gfx950) Vanka / geometric-multigrid / GMRES
 * solver for the Newton systems of dG(k)-in-time, Q2/P1disc-in-space
 * Navier-Stokes slabs (Anselmann & Bause, "Efficiency of local Vanka smoother
 * geometric multigrid preconditioning for space-time finite element methods
 * to the Navier-Stokes equations", Sec. 3).
 *
 * Conventions
 *   - Array arguments are DEVICE pointers unless marked (host).
 *   - The caller owns every array it passes (level matrices, transfer
 *     matrices, cell maps, workspace, vectors) and keeps them alive and
 *     unchanged until vk_destroy; the context stores the pointers, not copies.
 *     The values of a level matrix may change between vanka_setup calls (a
 *     new Newton linearisation); its structure (row pointers, columns) and the
 *     cell maps may not, since setup keeps plans made from them (grouped CSR,
 *     patch entry maps, the coarse block structure) until the next
 *     vk_set_level or vk_set_workspace.
 *   - Apart from one 4 KiB status block and a 64 KiB pinned host staging
 *     buffer for small reads (both allocated by vk_create), the library
 *     allocates no memory: all scratch lives in the caller-provided workspace
 *     (vk_workspace_bytes / vk_set_workspace).
 *   - All work is enqueued on the stream given to vk_create.  Calls are
 *     asynchronous except those returning host outputs (vanka_setup's singular
 *     check, gmres_solve's counts), which synchronise that stream.
 *   - Every call returns a vk_status; nothing throws across the ABI.
 *     vk_last_error returns a message for the last failure on a context.
 *   - Calls on one context must not overlap (one host thread at a time).
 *   - Floating point: matrices, vectors, residuals, Krylov vectors, patch
 *     factorisations and the coarse direct solve are FP64.  Only the stored
 *     patch inverses follow vk_prec (FP32/BF16 storage is applied with FP32
 *     accumulation and the product is added in FP64).
 */
#ifndef VK_H
#define VK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VK_OK = 0,
  VK_ERR_ARG = 1,        /* invalid argument or malformed input (message says which) */
  VK_ERR_HIP = 2,        /* a HIP runtime call or kernel launch failed */
  VK_ERR_SINGULAR = 3,   /* a zero pivot in a patch (or coarse) factorisation */
  VK_ERR_NOCONV = 4,     /* gmres_solve reached max_iter before the tolerance */
  VK_ERR_BREAKDOWN = 5,  /* GMRES produced a non-finite value */
  VK_ERR_WORKSPACE = 6,  /* workspace missing or smaller than vk_workspace_bytes */
  VK_ERR_STATE = 7       /* call order violated (e.g. smoothing before setup) */
} vk_status;

/* Storage of the patch inverses A_K = J_K^{-1}. */
typedef enum { VK_F64 = 0, VK_F32 = 1, VK_BF16 = 2 } vk_prec;

/* Smoother update rule.
 * VK_ADDITIVE: the averaged element-wise Vanka iteration of Sec. 3, Eq. 3.4
 *   and 3.5a-d: every cell applies S_K to the same iterate d^{j-1}, the local
 *   results are summed and divided by the number of cells sharing a DoF.
 * VK_MULT_COLOURED: the "overwriting successively" alternative the paper
 *   mentions after Eq. 3.5, in cell-coloured order: colour by colour, every
 *   cell of the colour computes its local defect from the iterate left by the
 *   previous colour and adds omega J_K^{-1} R_K (b - J d) to its DoFs. */
typedef enum { VK_ADDITIVE = 0, VK_MULT_COLOURED = 1 } vk_mode;

/* Compressed sparse rows, FP64 values, int64 row pointers, int32 columns.
 * Columns must be strictly increasing within each row and lie in [0, n_cols). */
typedef struct {
  int64_t n_rows;
  int64_t n_cols;
  int64_t nnz;
  const int64_t* row_ptr;  /* n_rows + 1 entries, row_ptr[0] = 0, row_ptr[n_rows] = nnz */
  const int32_t* col;      /* nnz */
  const double* val;       /* nnz */
} vk_csr;

typedef struct vk_ctx vk_ctx;

/* Create a context for an n_levels hierarchy (level 0 = coarsest T_0,
 * level n_levels-1 = finest T_L, Sec. 2).  hip_stream may be NULL (default
 * stream).  Allocates the 4 KiB device status block. */
vk_status vk_create(vk_ctx** ctx, int32_t n_levels, void* hip_stream);
void vk_destroy(vk_ctx* ctx);
/* Message of the last failure on ctx; with ctx == NULL, of the last failed
 * vk_create in the process. */
const char* vk_last_error(const vk_ctx* ctx);

/* Describe level l.
 *   J          level matrix J_l (the Newton Jacobian of Eq. 3.3 on T_l), square.
 *   P, R       prolongation T_{l-1} -> T_l (n_l x n_{l-1}) and restriction
 *              (n_{l-1} x n_l); both NULL on level 0.
 *   cell_dofs  n_cells x n_K row-major int32: dof(K, mu^) of Sec. 3, the
 *              global DoFs of cell K for all k+1 Radau nodes.  Ignored (may
 *              be NULL) on level 0, which is solved directly.
 *   colour_cells  device int32[n_cells]: the cells sorted by colour;
 *   colour_ptr    (host) int32[n_colours + 1]: colour c owns
 *              colour_cells[colour_ptr[c] .. colour_ptr[c+1]).  Cells of one
 *              colour must share no DoF (the caller's contract; the additive
 *              sweep relies on it for a race-free scatter, the multiplicative
 *              sweep for its update order).
 * Validates sizes on the host; validates CSR structure and DoF ranges on the
 * device (one synchronisation).  Returns VK_ERR_ARG on malformed input. */
vk_status vk_set_level(vk_ctx* ctx, int32_t l, const vk_csr* J, const vk_csr* P, const vk_csr* R,
                       int32_t n_cells, int32_t n_K, const int32_t* cell_dofs,
                       const int32_t* colour_cells, const int32_t* colour_ptr, int32_t n_colours);

/* ---- several independent systems in one context (batching) -------------
 * A batch of independent systems is described level by level from the finest
 * down: level L - d of the context holds, for every system s, its level
 * L_s - d (block-diagonal concatenation).  Cells are given in groups of equal
 * patch width (one group per k); systems whose coarsest level is reached at
 * this depth are listed as diagonal blocks solved directly (their rows carry no
 * cells); level 0 holds only blocks.  Every stage of the V-cycle then runs as
 * one launch over all systems. */
typedef struct {
  int32_t n_cells;
  int32_t n_K;
  const int32_t* cell_dofs;     /* device, n_cells x n_K, level-global DoF numbers */
  const int32_t* colour_cells;  /* device, n_cells, cells sorted by colour */
  const int32_t* colour_ptr;    /* host, n_colours + 1 */
  int32_t n_colours;
} vk_cell_group;

/* General form of vk_set_level: n_groups cell groups (levels >= 1) and
 * n_blocks directly solved diagonal blocks, rows [block_rows[b],
 * block_rows[b+1]) (host array, n_blocks + 1 entries, at most 9216 rows per
 * block).  A block must not be coupled to rows outside it (checked at setup).
 * vk_set_level(l = 0) is one block covering the level; vk_set_level(l >= 1) one
 * group and no blocks. */
vk_status vk_set_level_groups(vk_ctx* ctx, int32_t l, const vk_csr* J, const vk_csr* P, const vk_csr* R,
                              int32_t n_groups, const vk_cell_group* groups, int32_t n_blocks,
                              const int64_t* block_rows);

/* Split the finest level into n_seg independent systems, rows
 * [seg_rows[i], seg_rows[i+1]) (host array).  Call after setting the finest
 * level and before vk_set_workspace; default: one segment. */
vk_status vk_set_segments(vk_ctx* ctx, int32_t n_seg, const int64_t* seg_rows);

/* GMRES for every segment at once (Sec. 3 method per system, each with its own
 * Krylov space, Givens rotations and stopping test), Arnoldi steps in
 * lockstep: one V-cycle over all systems per step, converged systems idle.
 * Outputs (host, n_seg entries each): iters, true_rel_res; *all_converged
 * (host, may be NULL).  Returns VK_ERR_NOCONV if a system missed the
 * tolerance. */
vk_status gmres_solve_batched(vk_ctx* ctx, const double* b, double* x, int32_t restart, int32_t max_iter,
                              double rtol, double atol, int32_t nu_pre, int32_t nu_post, int32_t* iters,
                              double* true_rel_res, int32_t* all_converged);

/* Bytes of device workspace needed for patch inverses stored in `prec`, GMRES
 * restart length `restart` and the current levels.  Host-only query. */
size_t vk_workspace_bytes(const vk_ctx* ctx, vk_prec prec, int32_t restart);

/* Hand the workspace to the context (device memory, 256-byte aligned, at
 * least vk_workspace_bytes(prec, restart) bytes).  The context keeps the
 * pointer; previous setup results are invalidated. */
vk_status vk_set_workspace(vk_ctx* ctx, void* dev, size_t bytes, vk_prec prec, int32_t restart);

/* Vanka setup (Sec. 3, the paragraph after Eq. 3.4): for every cell K of every
 * level l >= 1 gather J_K = J_l restricted to dof(K, .) x dof(K, .), entries
 * not stored in J_l being zero, invert it in FP64 by Gauss-Jordan elimination
 * with partial pivoting (first row of maximal |pivot|, the LU pivot sequence;
 * the matrix-core kernel of the 170-wide patches counts candidates within a
 * relative 2^-13 of the largest as tied) and store A_K in `prec`; compute 1/p_mu, p_mu = number of cells containing
 * DoF mu (Eq. 3.5b); and form the FP64 inverse of J_0 for the coarsest-level
 * direct solve (blocked Gauss-Jordan with partial pivoting: the largest |pivot|
 * up to a relative 2^-38, the lowest row among those).  omega is the
 * under-relaxation of Eq. 3.4 (the paper uses 0.7).
 * The patch inversions run on an internal stream restricted to 7/8 of the
 * CUs (when the runtime supports CU masks), the finest level first; the
 * context's stream waits for the finest level's, and vanka_setup synchronises
 * for them only.  On a zero pivot in a finest-level patch it returns
 * VK_ERR_SINGULAR with *bad_level / *bad_cell (host, may be NULL) naming the
 * level and the first failing cell.  The coarser levels' inversions keep
 * running beside the next solve's finest-level sweeps: the first call that
 * smooths on such a level orders itself after its inversions, and a zero
 * pivot there is reported by the next call that reads the library's status
 * once every level has been waited for (gmres_solve and gmres_solve_batched
 * at their convergence checks, vcycle, vanka_smooth, vanka_smooth_noalloc,
 * vk_get_patch_inverses, vk_autotune): VK_ERR_SINGULAR naming the level and
 * cell in the message, after which setup must run again.  Without the
 * internal stream every level is checked by vanka_setup.  The internal stream
 * is a blocking stream: work on the legacy default stream waits for it, so
 * the overlap needs the context's stream to be another stream.  The inversion of the
 * directly solved blocks (the coarse matrix) keeps running on a second internal
 * stream and overlaps the start of the next solve; the first call that applies
 * a block (vcycle, gmres_solve, gmres_solve_batched, vk_get_coarse_inverse)
 * orders itself after it and reports a singular or coupled block there
 * (VK_ERR_SINGULAR / VK_ERR_ARG, after which setup must run again). */
vk_status vanka_setup(vk_ctx* ctx, double omega, vk_mode mode, int32_t* bad_level, int32_t* bad_cell);

/* `sweeps` Vanka iterations on level l >= 1 for J_l d = b (Eq. 3.5, or the
 * multiplicative variant selected at setup).  b, d: n_l FP64.  d is updated in
 * place; d_is_zero != 0 declares d = 0 on entry (d is then cleared by the
 * library and the first defect is b itself, as in the pre-smoothing d^0 = 0). */
vk_status vanka_smooth(vk_ctx* ctx, int32_t l, const double* b, double* d, int32_t sweeps,
                       int32_t d_is_zero);

/* vanka_smooth for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): the same sweeps with the same kernels and
 * results, but the per-call scratch (the defect b - J d, the per-cell products y_K and, in the
 * multiplicative mode, the per-cell local defects of one colour) lives in a fixed device array of
 * the library (64 MiB, one per GPU, held until the process ends) instead of the context's
 * workspace.  The call allocates nothing and makes no allocating library call.  Levels whose
 * scratch exceeds 64 MiB (8 n_l + n_cells n_K (8 for FP64 inverses, else 4) + 8 n_K x the largest
 * colour's cell count, each part rounded up to 256 bytes) are rejected with VK_ERR_ARG.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (from
 * different contexts, streams or threads) race and must be serialised by the caller.  Nothing is
 * assumed about the array's contents at entry.  Arguments, errors and stream as vanka_smooth.
 * Like the other direct entry points, the first call after vanka_setup waits on the host for the
 * coarser levels' patch inversions still running on the internal setup stream and reads their
 * status words there (nothing is enqueued on the context's stream for it); a caller that captures
 * a graph should make one call, or any other direct entry point, before capturing. */
vk_status vanka_smooth_noalloc(vk_ctx* ctx, int32_t l, const double* b, double* d, int32_t sweeps,
                               int32_t d_is_zero);

/* One V-cycle x = V(b) on the finest level from the zero initial guess
 * (Sec. 3): nu_pre sweeps from d = 0, defect restriction, recursion, direct
 * solve on T_0, prolongation of the correction, nu_post sweeps.  b, x: n_L FP64;
 * x may not alias b. */
vk_status vcycle(vk_ctx* ctx, const double* b, double* x, int32_t nu_pre, int32_t nu_post);

/* Restarted GMRES(restart) for J_L x = b, right-preconditioned by one V-cycle
 * per Arnoldi step (Sec. 3; [S03]).  x holds the initial guess on entry and the
 * iterate on exit.  Stops when the residual estimate is <= max(rtol ||b||, atol)
 * (Sec. 4 uses an absolute GMRES tolerance; relative 1e-8 is the default of the
 * tests), after max_iter Arnoldi steps summed over restarts, or on a happy
 * breakdown.  Orthogonalisation: classical Gram-Schmidt applied twice.
 * restart must not exceed the value given to vk_set_workspace.
 * Outputs (host): *iters Arnoldi steps, *true_rel_res = ||b - J x|| / ||b||
 * recomputed at the end, history[0..*iters] residual estimates (the initial
 * residual first) if history != NULL (max_iter + 1 entries).
 * b = 0 returns x = 0 and *iters = 0.  Returns VK_ERR_NOCONV if max_iter was
 * reached with the tolerance unmet (x is the last iterate). */
vk_status gmres_solve(vk_ctx* ctx, const double* b, double* x, int32_t restart, int32_t max_iter,
                      double rtol, double atol, int32_t nu_pre, int32_t nu_post, int32_t* iters,
                      double* true_rel_res, double* history);

/* ---- inspection helpers used by tests and the benchmark ----------------- */

/* y = alpha * J_l x + beta * z (z may alias y; beta = 0 ignores z). */
vk_status vk_spmv(vk_ctx* ctx, int32_t l, double alpha, const double* x, double beta,
                  const double* z, double* y);

/* Copy the stored inverses of cells [cell0, cell0 + n) of level l into out
 * (device, FP64, n x n_K x n_K row-major), widening FP32/BF16 storage. */
vk_status vk_get_patch_inverses(vk_ctx* ctx, int32_t l, int32_t cell0, int32_t n, double* out);

/* Copy the FP64 inverse of the coarsest matrix J_0 (row-major n_0 x n_0). */
vk_status vk_get_coarse_inverse(vk_ctx* ctx, double* out);

/* Per-launch tuning of the patch kernels: cells per 256-thread workgroup
 * (1, 2, 4 or 8; 0 = library default chosen from n_K and vk_prec). */
vk_status vk_set_patch_tile(vk_ctx* ctx, int32_t l, int32_t cells_per_block);

/* Stored bytes per patch inverse on level l (including padding) and the
 * leading dimension used (the inverse is stored column by column). */
vk_status vk_patch_layout(const vk_ctx* ctx, int32_t l, int64_t* bytes_per_cell, int32_t* ld);

/* Implementation of the averaged additive sweep (both compute Eq. 3.5):
 * VK_SWEEP_DOF_GATHER (default): one launch computes y_K = A_K R_K r for all
 *   cells, a second forms z_mu = sum over the cells containing mu of their y
 *   entry (ascending cell order) and d_mu += omega z_mu / p_mu.  Deterministic;
 *   needs no colouring.
 *   The per-DoF cell lists are read at a fixed width (4 or 8 entries) when no
 *   DoF lies in more than 8 cells, else through offsets.
 * VK_SWEEP_COLOURED_SCATTER: one launch per colour, each cell adding
 *   omega y_K / p to its DoFs directly (cells of a colour share no DoF).
 * VK_SWEEP_DOF_GATHER_OFFSETS: as VK_SWEEP_DOF_GATHER, always through the
 *   offsets (the same sums in the same order; for comparison). */
typedef enum {
  VK_SWEEP_DOF_GATHER = 0,
  VK_SWEEP_COLOURED_SCATTER = 1,
  VK_SWEEP_DOF_GATHER_OFFSETS = 2
} vk_sweep_variant;
vk_status vk_set_sweep_variant(vk_ctx* ctx, int32_t variant);

/* Patch inversion kernel used by vanka_setup: 0 (default) keeps the patch
 * matrix in registers where a kernel for the patch width is compiled: blocked
 * Gauss-Jordan on the FP64 matrix cores for n_K = 170 (16 x 16 tiles over a
 * 704-thread workgroup, rank-4 panel updates), its patches gathered through a
 * patch entry map (per cell and patch entry the entry's offset in its CSR row,
 * 2 bytes each, kept in the workspace and built at the first vanka_setup after
 * vk_set_level or vk_set_workspace); one row per lane for n_K = 42, 63, spread
 * over a 512-thread workgroup with vector FP64 for n_K = 84, 85, 105, 120,
 * 180; inverts other patches wider than 88 (up to 512) with the blocked
 * kernels of the directly solved blocks, one block per cell, and the rest in
 * LDS; 1 always uses the LDS / global-memory kernel; 2 is 0 without the
 * matrix-core kernel (n_K = 170 on the vector unit); 3 is 0 with the n_K = 170
 * patches gathered by a search of their CSR rows instead of the map.  All
 * compute the Gauss-Jordan inverse with the same partial pivoting; setup must
 * run again after a change. */
vk_status vk_set_setup_variant(vk_ctx* ctx, int32_t variant);

/* Pivot choice of the directly solved blocks' Gauss-Jordan inversion (the
 * coarsest level's direct solve, Sec. 3).  0 (default): blocks wider than 4096
 * rows take the pivots of each 16-column panel by tournament (each 512-row leaf
 * proposes the rows its own partial pivoting chose, and one workgroup picks the
 * panel's pivots from the proposals), narrower blocks as 1; 1: partial pivoting
 * over all unused rows, column by column; 2: the tournament for every block.
 * All compute the same inverse up to rounding, and all report a block whose
 * panel has no nonzero pivot.  Setup must run again after a change. */
vk_status vk_set_coarse_pivoting(vk_ctx* ctx, int32_t mode);

/* Storage read by the products with a level's J (the sweeps' defects r = b - J d,
 * the V-cycle residuals and GMRES's J z; Sec. 3).  1 (default): on levels with at
 * least 4 Mi nonzeros, a grouped CSR planned on the host at the first vanka_setup
 * after vk_set_level or vk_set_workspace: up to four consecutive rows whose
 * columns agree entry by entry up to a shift of 0 or 1 per entry (the velocity
 * components of one node, the pressure modes of one cell) share one column
 * list, so one 4-byte column word serves up to four 8-byte values; the values
 * are J's CSR values as given.  The autotuner then times it against CSR.
 * 4, 8, 16, 32 or 64: the grouped CSR with that many lanes per row group on
 * every level that has one (the autotuner then times only that count against
 * CSR; 1 returns the choice to the library).  0: CSR everywhere.  All compute
 * the same products up to summation order; VK_ERR_ARG for any other value. */
vk_status vk_set_spmv_format(vk_ctx* ctx, int32_t grouped);

/* 0 if level `level`'s J products use CSR, else the lanes per row group of the
 * grouped CSR in use; -1 for an invalid call. */
int32_t vk_spmv_format(vk_ctx* ctx, int32_t level);

/* The algorithmic bytes of one product with level `level`'s J in the storage in
 * use: CSR 12 nnz + 8 (n + 1) + 24 n; grouped CSR 8 nnz + 4 (column words) +
 * 20 per group + 24 n (x, z read, y written once).  -1 for an invalid call. */
double vk_spmv_bytes(vk_ctx* ctx, int32_t level);

/* Direct solver of a level whose directly solved rows form one block wider
 * than 4096 unknowns (the coarsest level's direct solve, Sec. 3).  0 (default):
 * where the block's sparsity allows it, a block-tridiagonal factorisation:
 * breadth-first level sets of the symmetrised pattern, grouped into blocks of
 * at least 256 and at most 2048 unknowns, are eliminated in order (each
 * Schur-complement block inverted densely by Gauss-Jordan with partial
 * pivoting inside the block); the solve runs forward and back over the blocks.
 * The plan is made on the host at the first vanka_setup after vk_set_level or
 * vk_set_workspace (the pattern is copied to the host once).  Blocks without
 * such a structure, and every block under mode 1, get the dense inverse.  Both
 * compute J_0^{-1} b up to rounding; a singular block is reported by the first
 * solve either way.  vk_get_coarse_inverse needs the dense inverse.  Setup must
 * run again after a change. */
vk_status vk_set_coarse_solver(vk_ctx* ctx, int32_t mode);

/* After vanka_setup: the number of blocks of level `level`'s block-tridiagonal
 * factorisation (0 when its directly solved blocks are inverted densely, -1 for
 * an invalid call), and in *setup_flops (if not null) the algorithmic flop
 * count of one factorisation or inversion (2 sum s_i^3 + 4 sum s_i^2 s_(i+1),
 * or 2 sum m_b^3 for dense inverses of blocks of m_b rows). */
int32_t vk_coarse_plan(vk_ctx* ctx, int32_t level, double* setup_flops);

/* Autotuner: after vanka_setup, times each level's SpMV kernels (J, P, R)
 * with 4, 8, 16, 32 and 64 lanes per row (also 1 and 2 for matrices with
 * fewer than 16 entries per row on average, such as the transfers P) and the patch GEMV with 1, 2, 4 and
 * 8 cells per workgroup (`reps` launches each, HIP events) and keeps the
 * fastest for the context; on levels with one cell group the GEMV tiles are
 * then timed again inside V-cycles from the finest level (three rounds of
 * `reps` V-cycles per tile, every launch timed), which decides.  Results change only in floating-point summation
 * order.  Overwrites the level scratch vectors and clears the timing
 * records; waits for the block inversion; synchronises the stream.
 * A later vk_set_workspace resets the choices (vk_set_patch_tile overrides). */
vk_status vk_autotune(vk_ctx* ctx, int32_t reps);

/* ---- hipGraph replay --------------------------------------------------------
 * With graphs enabled, gmres_solve and gmres_solve_batched record each Arnoldi
 * step (V-cycle, J z, two Gram-Schmidt passes, norm, Givens update, scaling; one
 * graph per step index j) the first time it runs and replay the recorded graph
 * on the context's stream afterwards; vcycle records one graph per (b, x,
 * nu_pre, nu_post).  Any call that changes what a graph has baked in (levels,
 * segments, workspace, vanka_setup, tiles, autotuning, sweep variant, timing)
 * makes the next step record again.  A step that starts while the last
 * vanka_setup's coarse inversion is still running runs eagerly (so it overlaps
 * the inversion).  Results equal the eager launches bit for bit (the same
 * kernels with the same arguments run in the same order).
 * Recording needs a second stream, created by the first enable.  While timing
 * is enabled, launches are eager.  vk_graph_stats returns the number of
 * recordings and replays since vk_create. */
vk_status vk_set_graphs(vk_ctx* ctx, int32_t enable);
vk_status vk_graph_stats(const vk_ctx* ctx, int64_t* captures, int64_t* launches);

/* ---- per-launch timing (benchmarks) --------------------------------------
 * With timing enabled, the library brackets launches of the kernel classes
 * below with a pair of HIP events on the stream the launch runs on (a pool of
 * 16384 pairs; launches beyond it are not recorded).  The patch GEMV takes the
 * events in its launch (hipExtLaunchKernel), so its pair holds the kernel's own
 * start and end; the other classes are bracketed by event records.
 * vk_timing_enable(ctx, 1, l) clears earlier records and records launches on
 * level l only (l = -1: all levels); enable = 0 stops recording.
 * vk_timing_kinds restricts recording to the classes whose bit (1 << kind) is
 * set in `mask` and to one of every `every` (>= 1) such launches (default: all
 * classes, every launch); recording slows the stream, so a benchmark records a
 * sample of what it reads.  vk_timing_read synchronises the streams and returns
 * the number of recorded launches of class `kind` on level l (l = -1: all
 * levels) and their summed duration in milliseconds. */
typedef enum {
  VK_KERNEL_PATCH_APPLY = 0,    /* gather - patch GEMV - scatter, one colour */
  VK_KERNEL_SPMV = 1,           /* level defect b - J d */
  VK_KERNEL_PATCH_SETUP = 2,    /* patch gather + Gauss-Jordan inverse */
  VK_KERNEL_PATCH_RESIDUAL = 3, /* multiplicative mode local defects */
  VK_KERNEL_PATCH_GEMV = 4,     /* y_K = A_K r_K for all cells (additive, DoF gather) */
  VK_KERNEL_DOF_GATHER = 5,     /* d += omega z / p from the y_K (additive, DoF gather) */
  VK_KERNEL_SWEEP = 6,          /* one whole additive sweep that starts with its defect b - J d
                                   (SpMV, patch GEMVs, DoF gather; Eq. 3.5); the first sweep from
                                   d = 0, which has no defect to form, is not recorded */
  VK_KERNEL_BLOCK_INVERT = 7    /* the inversion of one level's directly solved blocks (setup) */
} vk_kernel_kind;
vk_status vk_timing_enable(vk_ctx* ctx, int32_t enable, int32_t level);
vk_status vk_timing_kinds(vk_ctx* ctx, uint32_t mask, int32_t every);
vk_status vk_timing_read(vk_ctx* ctx, int32_t kind, int32_t l, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* VK_H */
