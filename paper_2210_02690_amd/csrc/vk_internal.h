// Internal declarations shared by the HIP translation units of libvk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include <string>
#include <vector>

#include "vk.h"

#define VK_NT 256  // threads per workgroup for the patch kernels

// Largest patch width kept entirely in LDS during setup (FP64 n_K x n_K plus
// small vectors must fit the 64 KiB a workgroup may always allocate).
#define VK_LDS_SETUP_MAX_NK 88
#define VK_MAX_NK 512
#define VK_MAX_RESTART 64
// blocked Gauss-Jordan of the directly solved blocks: outer block width, widest inner panel
#define VK_GJ_NBO 256  // widest outer block of the blocked Gauss-Jordan inversion (buffer sizes)
// outer block width with tournament panels on levels of a few blocks: each outer pass reads and
// writes the whole block once, so wider outer blocks halve those passes (3D coarse inversion
// 85.8 -> 81.0 ms beside the patch inversions, 128 -> 256)
#define VK_TOURNEY_NBO 256
#define VK_GJ_NBI_MAX 16
// blocks wider than this choose their pivots by tournament by default (below it the single-workgroup
// panels, which run a level's blocks side by side, are as fast)
#define VK_TOURNEY_MIN_N 4096

// ---- wavefront reductions through DPP (row shifts, then row broadcasts);
// the result of lane 63 is returned to every lane ----
template <int CTRL, int RM>
__device__ inline double dpp_move(double v, double ident) {
  const int2 a = __builtin_bit_cast(int2, v), b = __builtin_bit_cast(int2, ident);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(b.x, a.x, CTRL, RM, 0xF, false);
  r.y = __builtin_amdgcn_update_dpp(b.y, a.y, CTRL, RM, 0xF, false);
  return __builtin_bit_cast(double, r);
}

// Workgroup i of a launch runs on XCD i mod 8 (round-robin dispatch over the 8 dies, each with
// its own L2).  xcd_block(i, n) gives XCD x the contiguous block range [x q + min(x, r), ...)
// (q = n / 8, r = n mod 8; a bijection of [0, n)), so neighbouring blocks, which share the cache
// lines at their boundaries, sit behind the same L2.
__device__ inline unsigned xcd_block(unsigned b, unsigned n) {
  const unsigned q = n >> 3, r = n & 7u, x = b & 7u, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// maximum over the 64 lanes, returned to every lane (NaN lanes are ignored)
__device__ inline double wave_max(double v) {
  const double id = -__builtin_inf();
  v = fmax(v, dpp_move<0x111, 0xF>(v, id));
  v = fmax(v, dpp_move<0x112, 0xF>(v, id));
  v = fmax(v, dpp_move<0x114, 0xF>(v, id));
  v = fmax(v, dpp_move<0x118, 0xF>(v, id));
  v = fmax(v, dpp_move<0x142, 0xA>(v, id));
  v = fmax(v, dpp_move<0x143, 0xC>(v, id));
  const int2 a = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(a.x, 63);
  r.y = __builtin_amdgcn_readlane(a.y, 63);
  return __builtin_bit_cast(double, r);
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ inline int wave_min(int v) {
  const int id = INT_MAX;
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xA, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, 63);
}


// A set of cells of one patch width on one level (one system, or all systems
// of a batch with the same k).
struct vk_group {
  int32_t n_cells = 0, n_K = 0;
  const int32_t* cell_dofs = nullptr;
  const int32_t* colour_cells = nullptr;
  std::vector<int32_t> colour_ptr;  // host copy
  int32_t n_colours = 0;
  int32_t max_colour_cells = 0;
  int32_t cpb_override = 0;
  int32_t cpb_tuned = 0;      // picked by vk_autotune for the patch GEMV
  // carved from the workspace
  void* inv = nullptr;        // stored patch inverses
  int32_t ld = 0;             // leading dimension (rows, padded)
  int64_t cell_stride = 0;    // elements per cell
  int64_t y_off = 0;          // first flat (cell, local) index of the group on its level
  // patch entry map of the matrix-core inversion (patch.hip, patch_map_kernel): per cell, per
  // accumulator element of its 16 x 16 tiles, the entry's offset in its CSR row (0xFFFF: not
  // stored); planned once per pattern and workspace
  uint16_t* pmap = nullptr;
  bool pmap_ok = false;
};

// Buffers of the blocked patch inversion: up to `cap` doubles of dense blocks (the setup scratch),
// and per-row / per-block arrays for up to `rows_cap` rows and `blocks_cap` blocks.
struct vk_blocked_ws {
  double* a = nullptr;        // dense blocks (aliases the setup scratch)
  int64_t cap = 0;            // doubles
  int64_t rows_cap = 0, blocks_cap = 0;
  int32_t* q = nullptr;       // pivot rows, per row
  int32_t* used = nullptr;    // pivot records, per row
  double* gi = nullptr;       // blocks_cap x VK_GJ_NBI_MAX x 64 (64-column outer blocks)
  double* go = nullptr;       // 64 x rows_cap
  int64_t* rows = nullptr;    // blocks_cap + 1 block offsets
  int64_t* woff = nullptr;    // blocks_cap dense-matrix offsets
};

// Grouped CSR of a level's J (sparse.hip, spmv_g_kernel): planned on the host once per pattern and
// workspace for levels with at least VK_GCSR_MIN_NNZ entries; the arrays live in workspace space
// reserved for them (gcol at most VK_GCSR_MAX_FRAC of nnz; a pattern that needs more keeps CSR).
#define VK_GCSR_MIN_NNZ (4 << 20)
#define VK_GCSR_MAX_FRAC 2  // column words reserved: nnz / 2
struct vk_gcsr {
  bool planned = false, active = false;
  int64_t n_groups = 0;
  int64_t cap_words = 0, cap_groups = 0;  // reserved space
  int32_t* g_row = nullptr;               // n_groups + 1 first rows
  int64_t* g_coff = nullptr;              // n_groups + 1 column-list offsets
  int64_t* g_v0 = nullptr;                // n_groups first value offsets (row_ptr of the first row)
  uint32_t* gcol = nullptr;               // column words
};

// Block-tridiagonal factorisation of a level's single wide directly solved block (coarse_bt.hip):
// the plan (level-set blocks, permutation) is made once per pattern and workspace; the buffers are
// carved from the level's dense-inverse buffer.
#define VK_BT_MIN_BLOCK 256   // consecutive level sets are grouped into blocks of at least this size
#define VK_BT_MAX_BLOCK 2048  // widest block the factorisation accepts
struct vk_bt {
  bool planned = false;  // a plan was attempted for the current pattern and workspace
  bool active = false;   // the block is solved through the factorisation
  int nb = 0;
  int64_t smax = 0;
  double flops = 0.0;                     // algorithmic flop count of one factorisation
  int c = 0;                              // the middle block: both chains end there
  std::vector<int64_t> off, oD, oU, oL;   // block offsets (new order); element offsets of D_i, U_i, L_i
  double *D = nullptr, *Dinv = nullptr, *U = nullptr, *X = nullptr, *Lc = nullptr, *Y = nullptr;
  double *bp = nullptr, *y = nullptr, *xp = nullptr, *w = nullptr;  // solve vectors (w: 2 smax)
  int32_t *perm = nullptr, *iperm = nullptr;                         // new -> old, old -> new
  int64_t *d_off = nullptr, *d_oD = nullptr, *d_oU = nullptr, *d_oL = nullptr;
  // elimination steps: step k inverts the left chain's block pa[k] and the right chain's pb[k]
  // (-1: none) in one launch sequence; the last step the middle block.  Per step, device row
  // offsets (3) and dense-block offsets (2) of the pair
  std::vector<int> pa, pb;
  int64_t *d_prows = nullptr, *d_pwoff = nullptr;
};

struct vk_level {
  bool set = false;
  vk_csr J{}, P{}, R{};
  bool has_transfer = false;
  std::vector<vk_group> groups;
  int64_t n_items = 0;              // sum over groups of n_cells * n_K
  std::vector<int64_t> cb_rows;     // directly solved diagonal blocks: row offsets (n_blocks + 1)
  int64_t cb_max = 0;               // largest block
  int64_t cb_sq = 0;                // sum of squared block sizes
  int lpr_J = 4, lpr_P = 4, lpr_R = 4;
  vk_gcsr gJ;           // grouped CSR of J, used by the J products while gJ.active and use_gJ
  bool use_gJ = false;
  int lpr_gJ = 16;      // lanes per group in use
  int lpr_gJ_lib = 16;  // the library's own choice (planned, then autotuned)
  // carved from the workspace
  double* inv_p = nullptr;      // 1 / multiplicity
  int32_t* dof_off = nullptr;   // DoF -> (cell, local) lists: offsets (n + 1)
  int32_t* dof_list = nullptr;  // flat indices, ascending per DoF
  int32_t* dof_ell = nullptr;   // the same lists at a fixed width ell_w (-1 padded), n x ell_w
  int32_t ell_w = 0;            // 4 or 8 (largest multiplicity rounded up), 0: use the offset lists
  double* b = nullptr;          // V-cycle right-hand side
  double* d = nullptr;          // V-cycle iterate
  double* r = nullptr;          // defect scratch
  double* cb_a = nullptr;       // the blocks, eliminated in place by Gauss-Jordan
  double* cb_gi = nullptr;      // pivot rows' old values, inner panels (per block VK_GJ_NBI_MAX x VK_GJ_NBO)
  double* cb_go = nullptr;      // pivot rows' old values, outer blocks (per block VK_GJ_NBO x n_b)
  double* cb_W = nullptr;       // the eliminated blocks (= cb_a)
  int64_t* d_cb_rows = nullptr; // device copies of the block offsets
  int64_t* d_cb_woff = nullptr; // offset of each block's dense matrix
  int32_t* cb_q = nullptr;      // pivot rows (block-local), per block
  int32_t* cb_used = nullptr;   // per row: 0, or 1 + the column it is the pivot of
  // tournament pivoting of wide blocks: leaves' proposals (cb_cand_stride per block), the
  // panel's scaled pivot rows (per block VK_GJ_NBI_MAX^2) and pivot rows (per block
  // VK_GJ_NBI_MAX, -1 for a failed step)
  int32_t* cb_cand = nullptr;
  int64_t cb_cand_stride = 0;
  double* cb_prs = nullptr;
  int32_t* cb_pq = nullptr;
  vk_bt bt;
};

// A second stream for the look-ahead of the blocked inversion: after each outer block of columns
// the next block's columns are updated on the inversion's stream and all other columns on `aux`,
// overlapping the next block's panels (events: `gathered` orders aux after the pivot rows'
// gather, `bulk_done` the next gather after aux).
struct vk_lookahead {
  hipStream_t aux;
  hipEvent_t gathered, bulk_done;
};

struct vk_timing_rec {
  int32_t kind, level, slot;
};

struct vk_ctx {
  // per-launch event timing
  bool timing = false;
  int32_t timing_level = -1;
  uint32_t timing_kinds = ~0u;  // bit k: record launches of vk_kernel_kind k
  int32_t timing_every = 1;      // record one of every timing_every eligible launches
  int64_t timing_seen = 0;       // eligible launches since timing was enabled
  std::vector<hipEvent_t> ev;           // 2 * pool size, created on first enable
  std::vector<vk_timing_rec> recs;
  int32_t n_levels = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;       // internal stream: coarse inversion during patch setup
  vk_lookahead la{};                // second stream and events of the first block level's inversion
  // internal stream for the patch inversions, masked to 3/4 of the CUs (when the runtime allows
  // it), so they do not hold back the side stream's short block-inversion launches
  hipStream_t setup = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // further side streams: the block inversions of different levels are independent chains, one
  // stream each (created when a setup first needs them); n_xside of them belong to the last setup
  std::vector<hipStream_t> xside;
  std::vector<hipEvent_t> xjoin;
  int n_xside = 0;
  std::vector<vk_level> lv;
  std::string err;
  int32_t* status = nullptr;   // device status block (4 KiB)
  // pinned host staging for small device-to-host reads: a read into pageable memory can wait
  // for every stream of the device, which would serialise the side stream's block inversions
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_ready = false;
  vk_prec prec = VK_F64;
  int32_t restart = 0;
  bool setup_done = false;
  double omega = 0.7;
  vk_mode mode = VK_ADDITIVE;
  int32_t sweep_variant = 0;  // additive sweep: 0 DoF gather, 1 coloured scatter
  bool fast_setup = true;     // register-resident patch inversion where compiled
  bool mfma_setup = true;     // the matrix-core kernel where one is compiled for the patch width
  bool patch_map = true;      // ... gathering its patches through the patch entry map
  int64_t coarse_min_tourney = VK_TOURNEY_MIN_N;  // blocks wider than this choose pivots by tournament
  int32_t coarse_solver = 0;  // 0: block-tridiagonal factorisation where it applies, 1: dense inverse
  bool spmv_grouped = true;   // J products through the grouped CSR where a plan exists
  int spmv_lanes = 0;         // lanes per group of the grouped products (0: chosen per level)
  bool maps_ready = false;    // multiplicities and DoF lists (depend on the mesh only)
  // the block inversions of the last setup run on `side`; the first call that applies a
  // block makes `stream` wait for them, and the first synchronisation after that checks
  // their status words
  bool coarse_pending = false;
  bool coarse_check_due = false;
  // patch inversions of the levels below the finest, still running on the setup stream after
  // vanka_setup: the context stream waits for level l's event before it first smooths on l
  std::vector<hipEvent_t> patch_ev;  // per level, recorded on the setup stream
  uint64_t patch_pending = 0;         // bit l: not yet waited for
  bool patch_check_due = false;       // their status words not yet read

  void* Y = nullptr;          // per-cell products y_K of the additive sweep
  // batched GMRES: segments of the finest level solved as independent systems
  std::vector<int64_t> seg_rows;  // host, n_seg + 1
  int32_t n_seg = 1;
  int64_t* d_seg = nullptr;       // device copy
  double* seg_scal = nullptr;     // per-segment scalars (see api.hip)
  int32_t* seg_flags = nullptr;   // per-segment active flags and counters
  // setup scratch for patches too wide for LDS
  double* big_scratch = nullptr;
  int32_t big_chunk = 0;
  vk_blocked_ws blocked;  // patches wider than LDS through the blocked kernels (big_scratch holds the blocks)
  // multiplicative sweep: per-cell local defects of one colour
  double* rK = nullptr;
  // Krylov
  int64_t n_pad = 0;
  double* V = nullptr;   // (restart + 1) vectors
  double* Z = nullptr;   // restart vectors
  double* H = nullptr;   // (restart + 1) x restart, column-major
  double* h2 = nullptr;  // second CGS pass coefficients
  double* cs = nullptr;
  double* sn = nullptr;
  double* g = nullptr;
  double* y = nullptr;
  double* partial = nullptr;  // block partial sums
  double* scal = nullptr;     // device scalars
  double* ghist = nullptr;    // per Arnoldi step of a cycle: |g_{j+1}|, ||w|| (2 (restart + 1))
  void* noalloc = nullptr;    // device address of the fixed scratch on the context's device
  int32_t n_partial = 0;
  // hipGraph replay: one graph per Arnoldi step index (single and batched GMRES) and one
  // for the stand-alone V-cycle, captured on first use and replayed while nothing baked
  // into them (pointers, launch shapes, omega, sweep counts) has changed
  bool graphs = false;
  hipStream_t cap = nullptr;  // capture stream (the caller's stream may be the null stream)
  uint64_t gen = 1;           // bumped by every call that changes a baked parameter
  struct graph_slot {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;
    int64_t key[6] = {0, 0, 0, 0, 0, 0};
  };
  std::vector<graph_slot> gslots;
  int64_t graph_launches = 0, graph_captures = 0;
};

// ---- launchers (defined in the .hip files) --------------------------------
// sparse
int vk_pick_lpr(int64_t n_rows, int64_t nnz);
hipError_t launch_spmv(hipStream_t s, const vk_csr& A, int lpr, double alpha, const double* x,
                       double beta, const double* z, double* y);
hipError_t launch_validate_csr(hipStream_t s, const vk_csr& A, int32_t* flag);
hipError_t launch_spmv_g(hipStream_t s, const vk_csr& A, const vk_gcsr& g, int lpr, double alpha, const double* x,
                         double beta, const double* z, double* y);
// y = alpha J x + beta z with the level's chosen format (grouped CSR or CSR)
hipError_t launch_spmv_J(hipStream_t s, const vk_level& L, double alpha, const double* x, double beta,
                         const double* z, double* y);
// plan the grouped CSR of L.J in the space reserved for it (host, once per pattern and workspace)
bool vk_gcsr_plan(vk_level& L);
int vk_pick_lpr_g(int64_t nnz, int64_t n_rows);
hipError_t launch_validate_cells(hipStream_t s, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs,
                                 int64_t n, const int32_t* colour_cells, int32_t* flag);
hipError_t launch_fill(hipStream_t s, int64_t n, double v, double* x);
// sets *flag if two cells of one colour share a DoF (mask: one zeroed 64-bit word per DoF)
hipError_t launch_colour_check(hipStream_t s, int32_t n_K, const int32_t* cell_dofs, const int32_t* colour_cells,
                               const int32_t* colour_ptr, int32_t n_colours, unsigned long long* mask,
                               int32_t* flag);
hipError_t launch_fill_i32(hipStream_t s, int64_t n, int32_t v, int32_t* x);
// patches
hipError_t launch_count_add(hipStream_t s, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs, int32_t* count);
hipError_t launch_inv_count(hipStream_t s, int64_t n, const int32_t* count, double* inv_p);
hipError_t launch_dof_map(hipStream_t s, const vk_level& L, int32_t* count);
// largest multiplicity of the level into *max_count (atomic max; *max_count starts at 0)
hipError_t launch_dof_max_count(hipStream_t s, const vk_level& L, int32_t* max_count);
// the fixed-width copy of the DoF lists (L.ell_w set)
hipError_t launch_dof_ell(hipStream_t s, const vk_level& L);
hipError_t launch_patch_setup(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec, double* big_scratch,
                              int32_t big_chunk, int32_t* status);
// mfma: the matrix-core kernel where one is compiled for the patch width (else the VALU kernel)
// uint16 elements per cell of the patch entry map for patches n_K wide (0: no map for this width)
int64_t vk_patch_map_elems(int32_t n_K);
// plan G.pmap from J's pattern and G's cells; too_long (one int32) becomes nonzero when a row of a
// patch has more than 65535 entries (the map cannot hold its offsets)
hipError_t launch_patch_map(hipStream_t s, const vk_csr& J, const vk_group& G, int32_t* too_long);
hipError_t launch_patch_setup_fast(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec, int32_t* status,
                                   bool* handled, bool mfma = true, bool map = false);
// Patches of more than VK_LDS_SETUP_MAX_NK (at most 512) rows through the blocked Gauss-Jordan
// kernels of the directly solved blocks, in chunks of the workspace's blocked-setup buffers.
hipError_t launch_patch_setup_blocked(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec,
                                      const vk_blocked_ws& ws, int32_t* status);
hipError_t launch_patch_apply(hipStream_t s, const vk_group& G, vk_prec prec, int32_t colour, const double* r,
                              const double* rK, double* d, const double* inv_p, double omega);
hipError_t launch_patch_residual(hipStream_t s, const vk_csr& J, int lpr, const vk_group& G, int32_t colour,
                                 const double* b, const double* d, double* rK);
hipError_t launch_patch_export(hipStream_t s, const vk_group& G, vk_prec prec, int32_t cell0, int32_t n, double* out);
// ev0 / ev1 (may be null): events that take the kernel's start and end times
hipError_t launch_patch_gemv(hipStream_t s, const vk_group& G, vk_prec prec, const double* r, void* Y, int cpb = 0,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// d += omega / p * (sum of the cell products); overwrite: d = that term
hipError_t launch_dof_gather(hipStream_t s, const vk_level& L, vk_prec prec, const void* Y, double omega, double* d,
                             bool overwrite = false, bool fixed_width = true);
int vk_default_cpb(int32_t n_K, int32_t ld, vk_prec prec);
int vk_prec_vw(vk_prec prec);
int vk_prec_bytes(vk_prec prec);
// directly solved blocks (the coarsest level, and in batches every system's coarsest level)
int64_t vk_coarse_max_n();
// tourney: blocks wider than min_tourney rows choose their pivots by tournament
hipError_t launch_block_invert(hipStream_t s, const vk_level& L, int32_t* status, double** result,
                               const vk_lookahead* la = nullptr, int64_t min_tourney = VK_TOURNEY_MIN_N);
// Blocked Gauss-Jordan inversion of L's blocks (cb_rows, cb_max <= 512), whose dense column-major
// matrices are already in L.cb_a; a failing pivot sets status[0] to min(bad_base + block).
hipError_t launch_blocks_invert_dense(hipStream_t s, const vk_level& L, int32_t* status, int32_t bad_base);
hipError_t launch_block_apply(hipStream_t s, const vk_level& L, const double* x, double* y);
// Gauss-Jordan inversion of L's blocks whose dense column-major matrices are already in L.cb_a
// (any width up to vk_coarse_max_n(), partial pivoting over all rows); status[0] = -1 on failure.
hipError_t launch_block_invert_dense_any(hipStream_t s, const vk_level& L, int32_t* status);
// block-tridiagonal factorisation of a single wide block (coarse_bt.hip): plan (host, once per
// pattern and workspace; false: the block is not suited and stays with the dense inverse),
// factorisation (every setup) and solve x = J^{-1} b on the block's rows
bool vk_bt_plan(vk_level& L);
hipError_t launch_bt_factor(hipStream_t s, const vk_level& L, int32_t* status);
hipError_t launch_bt_solve(hipStream_t s, const vk_level& L, const double* b, double* x);
hipError_t launch_block_export(hipStream_t s, const vk_level& L, int32_t block, double* out);
// Krylov
hipError_t launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial,
                      int32_t n_partial, double* out, bool sqrt_out);
hipError_t launch_mdot(hipStream_t s, int64_t n, const double* V, int64_t ldv, int32_t m, const double* w,
                       double* partial, int32_t n_partial, double* out);
hipError_t launch_maxpy(hipStream_t s, int64_t n, const double* V, int64_t ldv, int32_t m, const double* h,
                        double sign, double* w);
hipError_t launch_scale_by_inv(hipStream_t s, int64_t n, const double* x, const double* den, double* y);
hipError_t launch_givens(hipStream_t s, int32_t j, int32_t ldh, double* H, const double* h2, double* cs,
                         double* sn, double* g, double* out);
hipError_t launch_gmres_init(hipStream_t s, int32_t m, double* H, double* g, const double* beta);
hipError_t launch_trisolve(hipStream_t s, int32_t jn, int32_t ldh, const double* H, const double* g, double* y);
// segmented Krylov kernels (one independent system per segment)
hipError_t launch_seg_dot(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* x,
                          const double* y, double* partial, int32_t n_partial, double* out, bool sqrt_out);
hipError_t launch_seg_mdot(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* V,
                           int64_t ldv, int32_t m, const double* w, double* partial, int32_t n_partial, double* out,
                           int32_t ldo);
hipError_t launch_seg_maxpy(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* V,
                            int64_t ldv, int32_t m, const double* h, int32_t ldh, const int32_t* mcount,
                            double sign, double* w);
hipError_t launch_seg_scale(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* x,
                            const double* den, const int32_t* active, double* y);
hipError_t launch_seg_init(hipStream_t s, int32_t n_seg, int32_t m, double* H, double* g, const double* beta,
                           const double* tol, const int32_t* its, int32_t max_iter, int32_t* active, int32_t* jn);
hipError_t launch_seg_givens(hipStream_t s, int32_t n_seg, int32_t j, int32_t m, double* H, const double* h2,
                             double* cs, double* sn, double* g, const double* tol, int32_t* its, int32_t max_iter,
                             int32_t* active, int32_t* jn, double* resid);
hipError_t launch_seg_trisolve(hipStream_t s, int32_t n_seg, int32_t m, const double* H, const double* g,
                               const int32_t* jn, double* y);
