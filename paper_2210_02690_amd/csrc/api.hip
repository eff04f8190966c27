// C ABI of libvk: context and level description, workspace planning, Vanka
// setup, smoothing, V-cycle and GMRES driver loops.  Every numerical step runs
// in the kernels of sparse.hip, patch.hip, coarse.hip and krylov.hip; this file
// only sequences launches on the context's stream.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>

#include "vk_internal.h"

#include <mutex>

// Fixed device scratch of vanka_smooth_noalloc: one copy per GPU, held until the process ends.  Host
// code never passes `scratch` itself to a kernel (on the host it names a stand-in, not device
// memory): vk_create looks up each device's address once with hipGetSymbolAddress.
#define VK_NOALLOC_SCRATCH_BYTES (64ull << 20)
static __device__ __align__(256) char scratch[VK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

vk_status fail(vk_ctx* ctx, vk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

vk_status fail_hip(vk_ctx* ctx, hipError_t e, const char* what) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  return fail(ctx, VK_ERR_HIP, buf);
}

#define VK_TRY(expr)                                       \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return fail_hip(ctx, _e, #expr); \
  } while (0)

#define VK_CHECK(st)                 \
  do {                               \
    vk_status _s = (st);             \
    if (_s != VK_OK) return _s;      \
  } while (0)

bool csr_ok(const vk_csr* A) {
  if (!A) return false;
  if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) return false;
  if (!A->row_ptr) return false;
  if (A->nnz > 0 && (!A->col || !A->val)) return false;
  if (A->n_cols > INT32_MAX) return false;
  return true;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Sequential carving of the workspace (256-byte aligned pieces).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  template <typename T>
  T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)count * sizeof(T);
    return p;
  }
};

bool levels_consistent(const vk_ctx* ctx, std::string* why) {
  for (int l = 0; l < ctx->n_levels; ++l) {
    const vk_level& L = ctx->lv[l];
    if (!L.set) {
      if (why) *why = "level " + std::to_string(l) + " not set";
      return false;
    }
    if (l > 0) {
      const int64_t nc = ctx->lv[l - 1].J.n_rows, nf = L.J.n_rows;
      if (L.P.n_rows != nf || L.P.n_cols != nc || L.R.n_rows != nc || L.R.n_cols != nf) {
        if (why) *why = "transfer sizes of level " + std::to_string(l) + " do not match J_l / J_{l-1}";
        return false;
      }
    }
  }
  return true;
}

// Lays out the workspace; with base == nullptr only the size is computed.
size_t plan_workspace(vk_ctx* ctx, vk_prec prec, int32_t restart, char* base) {
  Carver cv(base);
  const int nl = ctx->n_levels;
  const int vw = vk_prec_vw(prec), sb = vk_prec_bytes(prec);
  int32_t big_nk = 0, big_cells = 0;
  int64_t rk = 0, ycount = 0;
  for (int l = 0; l < nl; ++l) {
    vk_level& L = ctx->lv[l];
    const int64_t n = L.J.n_rows;
    L.b = cv.take<double>(n);
    L.d = cv.take<double>(n);
    L.r = cv.take<double>(n);
    L.gJ = vk_gcsr();  // a grouped-CSR plan lives in this workspace: made again for the new one
    L.use_gJ = false;
    if (L.J.nnz >= VK_GCSR_MIN_NNZ) {
      L.gJ.cap_words = L.J.nnz / VK_GCSR_MAX_FRAC;
      L.gJ.cap_groups = n;
      L.gJ.gcol = cv.take<uint32_t>(L.gJ.cap_words);
      L.gJ.g_row = cv.take<int32_t>(n + 1);
      L.gJ.g_coff = cv.take<int64_t>(n + 1);
      L.gJ.g_v0 = cv.take<int64_t>(n + 1);
    }
    if (!L.groups.empty()) {
      L.inv_p = cv.take<double>(n);
      L.dof_off = cv.take<int32_t>(n + 1);
      L.dof_list = cv.take<int32_t>(L.n_items > 0 ? L.n_items : 1);
      L.dof_ell = cv.take<int32_t>(8 * n);
      if (L.n_items > ycount) ycount = L.n_items;
    }
    for (vk_group& G : L.groups) {
      G.ld = (int32_t)round_up(G.n_K, vw);
      G.cell_stride = (int64_t)G.n_K * G.ld;
      G.inv = cv.take<char>((int64_t)G.n_cells * G.cell_stride * sb);
      // the patch entry map lives in this workspace: planned again for the new one
      const int64_t me = vk_patch_map_elems(G.n_K);
      G.pmap = me > 0 ? cv.take<uint16_t>((int64_t)G.n_cells * me) : nullptr;
      G.pmap_ok = false;
      if (G.n_K > VK_LDS_SETUP_MAX_NK) {
        if (G.n_K > big_nk) big_nk = G.n_K;
        if (G.n_cells > big_cells) big_cells = G.n_cells;
      }
      const int64_t r = (int64_t)G.max_colour_cells * G.n_K;
      if (r > rk) rk = r;
    }
    const int nbk = (int)L.cb_rows.size() - 1;
    if (nbk > 0) {
      L.cb_a = cv.take<double>(L.cb_sq);
      L.bt = vk_bt();  // a block-tridiagonal plan lives in cb_a: made again for the new buffer
      L.cb_gi = cv.take<double>((int64_t)nbk * VK_GJ_NBI_MAX * VK_GJ_NBO);
      L.cb_go = cv.take<double>((int64_t)VK_GJ_NBO * (L.cb_rows[nbk] - L.cb_rows[0]));
      L.d_cb_rows = cv.take<int64_t>(nbk + 1);
      L.d_cb_woff = cv.take<int64_t>(nbk);
      L.cb_q = cv.take<int32_t>(n);
      L.cb_used = cv.take<int32_t>(n);
      L.cb_cand_stride = (L.cb_max + 511) / 512 * VK_GJ_NBI_MAX;
      L.cb_cand = cv.take<int32_t>(nbk * L.cb_cand_stride);
      L.cb_prs = cv.take<double>((int64_t)nbk * VK_GJ_NBI_MAX * VK_GJ_NBI_MAX);
      L.cb_pq = cv.take<int32_t>((int64_t)nbk * VK_GJ_NBI_MAX);
    }
  }
  ctx->blocked = vk_blocked_ws();
  if (big_nk > 0) {
    const int64_t per = (int64_t)big_nk * big_nk;
    int64_t chunk = (int64_t)(512ll << 20) / (per * 8);
    if (chunk < 1) chunk = 1;
    if (chunk > big_cells) chunk = big_cells;
    ctx->big_chunk = (int32_t)chunk;
    ctx->big_scratch = cv.take<double>(chunk * per);
    // the blocked inversion of the wide patches: the scratch holds a chunk of dense blocks,
    // at most cap / n_K^2 cells of a group at a time
    vk_blocked_ws& bw = ctx->blocked;
    bw.a = ctx->big_scratch;
    bw.cap = chunk * per;
    for (int l = 0; l < nl; ++l)
      for (const vk_group& G : ctx->lv[l].groups) {
        if (G.n_K <= VK_LDS_SETUP_MAX_NK) continue;
        int64_t cg = bw.cap / ((int64_t)G.n_K * G.n_K);
        if (cg > G.n_cells) cg = G.n_cells;
        if (cg * G.n_K > bw.rows_cap) bw.rows_cap = cg * G.n_K;
        if (cg > bw.blocks_cap) bw.blocks_cap = cg;
      }
    bw.q = cv.take<int32_t>(bw.rows_cap);
    bw.used = cv.take<int32_t>(bw.rows_cap);
    bw.gi = cv.take<double>(bw.blocks_cap * VK_GJ_NBI_MAX * 64);
    bw.go = cv.take<double>(64 * bw.rows_cap);
    bw.rows = cv.take<int64_t>(bw.blocks_cap + 1);
    bw.woff = cv.take<int64_t>(bw.blocks_cap);
  } else {
    ctx->big_chunk = 0;
    ctx->big_scratch = nullptr;
  }
  ctx->rK = cv.take<double>(rk > 0 ? rk : 1);
  ctx->Y = cv.take<double>(ycount > 0 ? ycount : 1);
  const int64_t nL = ctx->lv[nl - 1].J.n_rows;
  ctx->n_pad = round_up(nL, 32);
  const int32_t m = restart;
  const int32_t ns = ctx->n_seg;
  ctx->V = cv.take<double>((int64_t)(m + 1) * ctx->n_pad);
  ctx->Z = cv.take<double>((int64_t)m * ctx->n_pad);
  ctx->H = cv.take<double>((int64_t)ns * (m + 1) * m);
  ctx->h2 = cv.take<double>((int64_t)ns * (m + 1));
  ctx->cs = cv.take<double>((int64_t)ns * m);
  ctx->sn = cv.take<double>((int64_t)ns * m);
  ctx->g = cv.take<double>((int64_t)ns * (m + 1));
  ctx->y = cv.take<double>((int64_t)ns * m);
  ctx->n_partial = (ns * 64 > 1024 ? ns * 64 : 1024) * (m + 1);
  ctx->partial = cv.take<double>(ctx->n_partial);
  ctx->scal = cv.take<double>(16);
  ctx->ghist = cv.take<double>(2 * (int64_t)(m + 1));
  ctx->d_seg = cv.take<int64_t>(ns + 1);
  ctx->seg_scal = cv.take<double>(5 * (int64_t)ns);
  ctx->seg_flags = cv.take<int32_t>(3 * (int64_t)ns);
  return cv.off;
}

// host tables that kernels read: block offsets, block storage offsets, segments
vk_status upload_tables(vk_ctx* ctx) {
  for (int l = 0; l < ctx->n_levels; ++l) {
    vk_level& L = ctx->lv[l];
    const int nbk = (int)L.cb_rows.size() - 1;
    if (nbk <= 0) continue;
    std::vector<int64_t> woff(nbk);
    int64_t acc = 0;
    for (int b = 0; b < nbk; ++b) {
      woff[b] = acc;
      const int64_t nb = L.cb_rows[b + 1] - L.cb_rows[b];
      acc += nb * nb;
    }
    VK_TRY(hipMemcpy(L.d_cb_rows, L.cb_rows.data(), sizeof(int64_t) * (nbk + 1), hipMemcpyHostToDevice));
    VK_TRY(hipMemcpy(L.d_cb_woff, woff.data(), sizeof(int64_t) * nbk, hipMemcpyHostToDevice));
  }
  VK_TRY(hipMemcpy(ctx->d_seg, ctx->seg_rows.data(), sizeof(int64_t) * (ctx->n_seg + 1), hipMemcpyHostToDevice));
  return VK_OK;
}

constexpr int32_t kTimingPool = 16384;

// Brackets one launch with a pair of events when timing is on.
// Brackets one launch with a pair of timing events.  With `in_launch`, the launch itself takes the
// events (start() / stop() to hipExtLaunchKernel), which times the kernel alone and adds no
// packets to the stream.
struct Timed {
  vk_ctx* ctx;
  hipStream_t stream;
  bool in_launch;
  int32_t slot = -1;
  Timed(vk_ctx* c, int32_t kind, int32_t level, hipStream_t s = nullptr, bool launch_events = false)
      : ctx(c), stream(s ? s : c->stream), in_launch(launch_events) {
    if (!ctx->timing || (int32_t)ctx->recs.size() >= kTimingPool || level < -1) return;
    if (ctx->timing_level >= 0 && level != ctx->timing_level) return;
    if (!((ctx->timing_kinds >> kind) & 1u)) return;
    if (ctx->timing_seen++ % ctx->timing_every != 0) return;
    slot = (int32_t)ctx->recs.size();
    ctx->recs.push_back({kind, level, slot});
    if (!in_launch) (void)hipEventRecord(ctx->ev[2 * slot], stream);
  }
  hipEvent_t start() const { return slot >= 0 ? ctx->ev[2 * slot] : nullptr; }
  hipEvent_t stop() const { return slot >= 0 ? ctx->ev[2 * slot + 1] : nullptr; }
  ~Timed() {
    if (slot >= 0 && !in_launch) (void)hipEventRecord(ctx->ev[2 * slot + 1], stream);
  }
};

// Scratch of one smoothing call: the defect r (n_l doubles), the per-cell products y_K (one entry
// per (cell, local DoF) of the level, FP64 or FP32) and the multiplicative mode's local defects.
struct sweep_bufs {
  double* r;
  void* Y;
  double* rK;
};

vk_status smooth_with(vk_ctx* ctx, int l, const double* b, double* d, int32_t sweeps, bool zero,
                      const sweep_bufs& buf);

sweep_bufs workspace_bufs(vk_ctx* ctx, int l) { return {ctx->lv[l].r, ctx->Y, ctx->rK}; }

vk_status smooth(vk_ctx* ctx, int l, const double* b, double* d, int32_t sweeps, bool zero) {
  return smooth_with(ctx, l, b, d, sweeps, zero, workspace_bufs(ctx, l));
}

// Orders the context stream after level l's patch inversions of the last setup (no host wait);
// l < 0: after every level's.  Their status words are read by the next patch_check.
vk_status patch_wait(vk_ctx* ctx, int l) {
  for (int k = 1; k < ctx->n_levels && ctx->patch_pending; ++k) {
    if ((l >= 0 && k != l) || !((ctx->patch_pending >> k) & 1)) continue;
    VK_TRY(hipStreamWaitEvent(ctx->stream, ctx->patch_ev[k], 0));
    ctx->patch_pending &= ~(1ull << k);
  }
  return VK_OK;
}

// For the direct entry points (which may run under a caller's graph capture): the host waits for
// the setup stream itself and reads the status words through it, leaving the context stream
// untouched; afterwards nothing is pending.  report = false discards what it finds.
vk_status patch_settle(vk_ctx* ctx, bool report) {
  if (!ctx->patch_pending && !ctx->patch_check_due) return VK_OK;
  const bool due = ctx->patch_check_due;
  ctx->patch_pending = 0;
  ctx->patch_check_due = false;
  VK_TRY(hipMemcpyAsync(ctx->pinned, ctx->status + 64, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->setup));
  VK_TRY(hipStreamSynchronize(ctx->setup));
  if (!report || !due) return VK_OK;
  const int32_t* st = reinterpret_cast<const int32_t*>(ctx->pinned);
  for (int l = 1; l < ctx->n_levels; ++l)
    if (st[l] != INT_MAX) {
      ctx->setup_done = false;
      char buf[128];
      snprintf(buf, sizeof(buf), "patch matrix of cell %d on level %d is singular (zero pivot)", st[l], l);
      return fail(ctx, VK_ERR_SINGULAR, buf);
    }
  return VK_OK;
}

vk_status to_host(vk_ctx* ctx, void* dst, const void* src, size_t bytes);

// Singular patches of the levels whose inversions vanka_setup left running: read once every such
// level has been waited for (synchronises the context stream then).
vk_status patch_check(vk_ctx* ctx) {
  if (!ctx->patch_check_due || ctx->patch_pending) return VK_OK;
  int32_t st[64];
  VK_CHECK(to_host(ctx, st, ctx->status + 64, sizeof(st)));
  ctx->patch_check_due = false;
  for (int l = 1; l < ctx->n_levels; ++l)
    if (st[l] != INT_MAX) {
      ctx->setup_done = false;
      char buf[128];
      snprintf(buf, sizeof(buf), "patch matrix of cell %d on level %d is singular (zero pivot)", st[l], l);
      return fail(ctx, VK_ERR_SINGULAR, buf);
    }
  return VK_OK;
}

vk_status smooth_with(vk_ctx* ctx, int l, const double* b, double* d, int32_t sweeps, bool zero,
                      const sweep_bufs& buf) {
  vk_level& L = ctx->lv[l];
  hipStream_t s = ctx->stream;
  if ((ctx->patch_pending >> l) & 1) VK_CHECK(patch_wait(ctx, l));
  // from d = 0 the first additive DoF-gather sweep writes d instead of adding to a zeroed d
  const bool gather = ctx->sweep_variant != VK_SWEEP_COLOURED_SCATTER;
  const bool write_first = zero && sweeps > 0 && ctx->mode == VK_ADDITIVE && gather;
  if (zero && !write_first) VK_TRY(launch_fill(s, L.J.n_rows, 0.0, d));
  for (int it = 0; it < sweeps; ++it) {
    if (ctx->mode == VK_ADDITIVE) {
      const double* r = b;
      // a whole sweep that forms its defect, bracketed as one unit (every kernel of Eq. 3.5)
      Timed tsw(ctx, VK_KERNEL_SWEEP, (it == 0 && zero) ? -2 : l);
      if (!(it == 0 && zero)) {
        Timed t(ctx, VK_KERNEL_SPMV, l);
        VK_TRY(launch_spmv_J(s, L, -1.0, d, 1.0, b, buf.r));
        r = buf.r;
      }
      if (gather) {
        for (const vk_group& G : L.groups) {
          Timed t(ctx, VK_KERNEL_PATCH_GEMV, l, s, true);
          VK_TRY(launch_patch_gemv(s, G, ctx->prec, r, buf.Y, 0, t.start(), t.stop()));
        }
        Timed t(ctx, VK_KERNEL_DOF_GATHER, l);
        VK_TRY(launch_dof_gather(s, L, ctx->prec, buf.Y, ctx->omega, d, write_first && it == 0,
                                 ctx->sweep_variant == VK_SWEEP_DOF_GATHER));
      } else {
        for (const vk_group& G : L.groups)
          for (int c = 0; c < G.n_colours; ++c) {
            Timed t(ctx, VK_KERNEL_PATCH_APPLY, l);
            VK_TRY(launch_patch_apply(s, G, ctx->prec, c, r, nullptr, d, L.inv_p, ctx->omega));
          }
      }
    } else {
      // groups are independent systems: colour c of every group, then colour c + 1
      int max_c = 0;
      for (const vk_group& G : L.groups) max_c = G.n_colours > max_c ? G.n_colours : max_c;
      for (int c = 0; c < max_c; ++c) {
        for (const vk_group& G : L.groups) {
          if (c >= G.n_colours) continue;
          {
            Timed t(ctx, VK_KERNEL_PATCH_RESIDUAL, l);
            VK_TRY(launch_patch_residual(s, L.J, L.lpr_J, G, c, b, d, buf.rK));
          }
          Timed t(ctx, VK_KERNEL_PATCH_APPLY, l);
          VK_TRY(launch_patch_apply(s, G, ctx->prec, c, nullptr, buf.rK, d, nullptr, ctx->omega));
        }
      }
    }
  }
  return VK_OK;
}

vk_status coarse_wait(vk_ctx* ctx, bool check_now);

vk_status vcycle_level(vk_ctx* ctx, int l, const double* b, double* x, int32_t nu1, int32_t nu2) {
  hipStream_t s = ctx->stream;
  vk_level& L = ctx->lv[l];
  if (l == 0) {
    if (ctx->coarse_pending) VK_CHECK(coarse_wait(ctx, false));  // only now wait for the inversion
    if (L.bt.active) VK_TRY(launch_bt_solve(s, L, b, x));
    else VK_TRY(launch_block_apply(s, L, b, x));
    return VK_OK;
  }
  vk_level& C = ctx->lv[l - 1];
  if (nu1 > 0) VK_CHECK(smooth(ctx, l, b, x, nu1, true));
  else VK_TRY(launch_fill(s, L.J.n_rows, 0.0, x));
  // systems whose coarsest level is this one are solved directly (their rows carry no cells)
  if (ctx->coarse_pending && L.cb_rows.size() > 1) VK_CHECK(coarse_wait(ctx, false));
  if (L.bt.active) VK_TRY(launch_bt_solve(s, L, b, x));
  else VK_TRY(launch_block_apply(s, L, b, x));
  VK_TRY(launch_spmv_J(s, L, -1.0, x, 1.0, b, L.r));
  VK_TRY(launch_spmv(s, L.R, L.lpr_R, 1.0, L.r, 0.0, nullptr, C.b));
  VK_CHECK(vcycle_level(ctx, l - 1, C.b, C.d, nu1, nu2));
  VK_TRY(launch_spmv(s, L.P, L.lpr_P, 1.0, C.d, 1.0, x, x));
  if (nu2 > 0) VK_CHECK(smooth(ctx, l, b, x, nu2, false));
  return VK_OK;
}

// Device-to-host copy on the context stream through the pinned staging buffer; synchronises
// the context stream only.
vk_status to_host(vk_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) {
    VK_TRY(hipMemcpyAsync(ctx->pinned, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    VK_TRY(hipStreamSynchronize(ctx->stream));
    std::memcpy(dst, ctx->pinned, bytes);
  } else {
    VK_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    VK_TRY(hipStreamSynchronize(ctx->stream));
  }
  return VK_OK;
}

// Host-to-device copy on the context stream; synchronises the context stream.
vk_status to_dev(vk_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) {
    std::memcpy(ctx->pinned, src, bytes);
    VK_TRY(hipMemcpyAsync(dst, ctx->pinned, bytes, hipMemcpyHostToDevice, ctx->stream));
  } else {
    VK_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  }
  VK_TRY(hipStreamSynchronize(ctx->stream));
  return VK_OK;
}

vk_status read_scalars(vk_ctx* ctx, const double* dev, int count, double* out) {
  return to_host(ctx, out, dev, sizeof(double) * count);
}

// Two device-to-host copies behind one synchronisation (both fit the pinned staging buffer).
vk_status to_host2(vk_ctx* ctx, void* dst0, const void* src0, size_t b0, void* dst1, const void* src1, size_t b1) {
  if (b0 + b1 > ctx->pinned_bytes) {
    VK_CHECK(to_host(ctx, dst0, src0, b0));
    return to_host(ctx, dst1, src1, b1);
  }
  VK_TRY(hipMemcpyAsync(ctx->pinned, src0, b0, hipMemcpyDeviceToHost, ctx->stream));
  VK_TRY(hipMemcpyAsync(ctx->pinned + b0, src1, b1, hipMemcpyDeviceToHost, ctx->stream));
  VK_TRY(hipStreamSynchronize(ctx->stream));
  std::memcpy(dst0, ctx->pinned, b0);
  std::memcpy(dst1, ctx->pinned + b0, b1);
  return VK_OK;
}

// How many Arnoldi steps to enqueue before the host next looks at the residual estimates.  The
// convergence test runs on the host from values the device wrote, so every look is one round trip
// in which the GPU idles; steps enqueued past convergence are discarded, each a V-cycle of wasted
// work.  From the mean reduction factor per step so far, rho = (r_now / r_start)^(1/steps), the
// steps still needed are log(tol / r_now) / log(rho); one fewer than that is enqueued (at most 8),
// so a steady rate costs two looks and no wasted step.  Without a rate yet: one step.
int32_t steps_ahead(double r_start, double r_now, int32_t steps, double tol) {
  if (steps < 1 || !(r_now > tol) || !(r_start > 0.0) || !(r_now > 0.0)) return 1;
  const double rho = std::pow(r_now / r_start, 1.0 / steps);
  if (!(rho < 0.999)) return 1;
  const double need = std::log(tol / r_now) / std::log(rho);
  if (!(need > 2.0)) return 1;
  const double c = std::floor(need) - 1.0;
  return c >= 8.0 ? 8 : (int32_t)c;
}

// Runs enqueue() on ctx->stream, or, with graphs on, replays the graph held in `slot` when it was
// captured under the same key and parameter generation (capturing it first otherwise).  enqueue
// must take its stream from ctx->stream, which points at the capture stream while recording.
// Event timing needs eager launches, so it turns replay off.
template <class F>
vk_status replay(vk_ctx* ctx, size_t slot, const int64_t (&key)[6], F&& enqueue) {
  if (!ctx->graphs || ctx->timing) return enqueue();
  // While the last setup's block inversion is still running, the step runs eagerly: its work up to
  // the coarse solve then overlaps the inversion (a replay would have to wait for it first).
  if (ctx->coarse_pending || ctx->patch_pending) return enqueue();
  if (ctx->gslots.size() <= slot) ctx->gslots.resize(slot + 1);
  vk_ctx::graph_slot& g = ctx->gslots[slot];
  const bool hit = g.exec && g.gen == ctx->gen && std::equal(key, key + 6, g.key);
  if (!hit) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    hipStream_t user = ctx->stream;
    VK_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed));
    ctx->stream = ctx->cap;
    const vk_status st = enqueue();
    ctx->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
    if (st != VK_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return st;
    }
    if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamEndCapture");
    const hipError_t e2 = hipGraphInstantiateWithFlags(&g.exec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      g.exec = nullptr;
      return fail_hip(ctx, e2, "hipGraphInstantiateWithFlags");
    }
    g.gen = ctx->gen;
    std::copy(key, key + 6, g.key);
    ++ctx->graph_captures;
  }
  VK_TRY(hipGraphLaunch(g.exec, ctx->stream));
  ++ctx->graph_launches;
  return VK_OK;
}

// Make the context stream wait for the block inversions of the last setup (no host wait).
// With check_now the stream is synchronised and their status words are checked at once.
vk_status coarse_check(vk_ctx* ctx);
vk_status coarse_wait(vk_ctx* ctx, bool check_now) {
  if (ctx->coarse_pending) {
    VK_TRY(hipStreamWaitEvent(ctx->stream, ctx->join_ev, 0));
    for (int i = 0; i < ctx->n_xside; ++i) VK_TRY(hipStreamWaitEvent(ctx->stream, ctx->xjoin[i], 0));
    ctx->coarse_pending = false;
    ctx->coarse_check_due = true;
  }
  if (check_now) return coarse_check(ctx);
  return VK_OK;
}

// Status of the block inversions: [0] pivot failure, [1] coupling outside a block.  Call
// after coarse_wait; synchronises the stream.
vk_status patch_check(vk_ctx* ctx);
vk_status coarse_check(vk_ctx* ctx) {
  VK_CHECK(patch_check(ctx));
  if (!ctx->coarse_check_due) return VK_OK;
  int32_t st[2];
  VK_CHECK(to_host(ctx, st, ctx->status, sizeof(st)));
  ctx->coarse_check_due = false;
  if (st[1] != 0) {
    ctx->setup_done = false;
    return fail(ctx, VK_ERR_ARG, "a directly solved block is coupled to rows outside it");
  }
  if (st[0] != INT_MAX) {
    ctx->setup_done = false;
    return fail(ctx, VK_ERR_SINGULAR, "a directly solved (coarsest-level) block is singular (zero pivot)");
  }
  return VK_OK;
}

char g_create_err[256] = "";

vk_status create_fail(vk_status st, const char* msg) {
  snprintf(g_create_err, sizeof(g_create_err), "%s", msg);
  return st;
}

vk_status ready(vk_ctx* ctx) {
  if (!ctx) return VK_ERR_ARG;
  if (!ctx->ws_ready) return fail(ctx, VK_ERR_WORKSPACE, "workspace not set");
  if (!ctx->setup_done) return fail(ctx, VK_ERR_STATE, "vanka_setup has not run since the workspace was set");
  return VK_OK;
}

}  // namespace

// The patch inversions fill every CU they may use, and the block inversions, one workgroup per
// block and a long chain of short launches, are slowed down by them.  Their stream therefore
// leaves 1/8 of the CUs (32 of 256) out of its mask: with the 3D coarse block factorised block by
// block, the 3D setup measured 55.7 ms with 1/4 left out, 47.6 with 1/8 and with 1/16, and 56 ms
// with all CUs (the chain then waits behind the patch inversions).  Without CU masking the patch
// inversions stay on the caller's stream.
// A stream restricted to the first n_cu - n_cu / leave_out CUs; null if CU masking is unavailable.
// (One such stream per context: with a second one, measured here, the side stream's launches waited
// for the whole patch inversion.)
hipStream_t create_masked_stream(int leave_out) {
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 32) {
    (void)hipGetLastError();
    return nullptr;
  }
  const int keep = n_cu - n_cu / leave_out;
  std::vector<uint32_t> mask((n_cu + 31) / 32, 0u);
  for (int c = 0; c < keep; ++c) mask[c / 32] |= 1u << (c % 32);
  hipStream_t st = nullptr;
  if (hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return st;
}

void create_setup_stream(vk_ctx* ctx) { ctx->setup = create_masked_stream(8); }

extern "C" {

vk_status vk_create(vk_ctx** out, int32_t n_levels, void* hip_stream) {
  if (!out) return create_fail(VK_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (n_levels < 1 || n_levels > 32) return create_fail(VK_ERR_ARG, "n_levels must be in [1, 32]");
  vk_ctx* ctx = new (std::nothrow) vk_ctx;
  if (!ctx) return create_fail(VK_ERR_ARG, "host allocation failed");
  ctx->n_levels = n_levels;
  ctx->lv.resize(n_levels);
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipMalloc(&ctx->status, 4096);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), 65536, hipHostMallocDefault);
  if (e == hipSuccess) ctx->pinned_bytes = 65536;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->la.aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->la.gathered, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->la.bulk_done, hipEventDisableTiming);
  if (e == hipSuccess) e = noalloc_scratch(&ctx->noalloc);
  if (e == hipSuccess) create_setup_stream(ctx);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the error for the caller's next check
    if (ctx->setup) (void)hipStreamDestroy(ctx->setup);
    if (ctx->la.bulk_done) (void)hipEventDestroy(ctx->la.bulk_done);
    if (ctx->la.gathered) (void)hipEventDestroy(ctx->la.gathered);
    if (ctx->la.aux) (void)hipStreamDestroy(ctx->la.aux);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->status) (void)hipFree(ctx->status);
    delete ctx;
    char buf[256];
    snprintf(buf, sizeof(buf), "vk_create: HIP resource allocation failed: %s", hipGetErrorString(e));
    return create_fail(VK_ERR_HIP, buf);
  }
  *out = ctx;
  return VK_OK;
}

void vk_destroy(vk_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  for (vk_ctx::graph_slot& g : ctx->gslots)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);

  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  if (ctx->setup) {
    (void)hipStreamSynchronize(ctx->setup);
    (void)hipStreamDestroy(ctx->setup);
  }
  for (hipEvent_t e : ctx->patch_ev) (void)hipEventDestroy(e);
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);
  if (ctx->la.aux) {
    (void)hipStreamSynchronize(ctx->la.aux);
    (void)hipStreamDestroy(ctx->la.aux);
  }
  if (ctx->la.gathered) (void)hipEventDestroy(ctx->la.gathered);
  if (ctx->la.bulk_done) (void)hipEventDestroy(ctx->la.bulk_done);
  for (size_t i = 0; i < ctx->xside.size(); ++i) {
    (void)hipStreamSynchronize(ctx->xside[i]);
    (void)hipStreamDestroy(ctx->xside[i]);
    (void)hipEventDestroy(ctx->xjoin[i]);
  }
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->status) (void)hipFree(ctx->status);
  delete ctx;
}

const char* vk_last_error(const vk_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err; }

vk_status vk_set_level_groups(vk_ctx* ctx, int32_t l, const vk_csr* J, const vk_csr* P, const vk_csr* R,
                              int32_t n_groups, const vk_cell_group* groups, int32_t n_blocks,
                              const int64_t* block_rows) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);  // block inversions still reading the old setup
  for (hipStream_t x : ctx->xside) (void)hipStreamSynchronize(x);
  if (ctx->setup) (void)hipStreamSynchronize(ctx->setup);  // and patch inversions after a failed setup
  ctx->coarse_pending = false;
  ctx->coarse_check_due = false;
  ctx->patch_pending = 0;
  ctx->patch_check_due = false;
  if (l < 0 || l >= ctx->n_levels) return fail(ctx, VK_ERR_ARG, "level index out of range");
  if (!csr_ok(J) || J->n_rows != J->n_cols || J->n_rows == 0)
    return fail(ctx, VK_ERR_ARG, "J must be a non-empty square CSR matrix with valid pointers");
  if (J->n_rows > INT32_MAX) return fail(ctx, VK_ERR_ARG, "J too large for int32 columns");
  if (n_groups < 0 || n_groups > 64 || (n_groups > 0 && !groups))
    return fail(ctx, VK_ERR_ARG, "0 <= n_groups <= 64 cell groups required");
  if (n_blocks < 0 || (n_blocks > 0 && !block_rows)) return fail(ctx, VK_ERR_ARG, "invalid block table");
  if (l == 0 && (n_groups != 0 || n_blocks < 1))
    return fail(ctx, VK_ERR_ARG, "level 0 is solved directly: no cell groups, at least one block");
  if (l > 0 && n_groups < 1) return fail(ctx, VK_ERR_ARG, "levels >= 1 need at least one cell group");
  vk_level L;
  L.J = *J;
  // directly solved diagonal blocks
  if (n_blocks > 0) {
    L.cb_rows.assign(block_rows, block_rows + n_blocks + 1);
    for (int b = 0; b < n_blocks; ++b) {
      const int64_t nb = L.cb_rows[b + 1] - L.cb_rows[b];
      if (nb <= 0 || L.cb_rows[b] < 0 || L.cb_rows[b + 1] > J->n_rows)
        return fail(ctx, VK_ERR_ARG, "blocks must be non-empty, increasing and inside the level");
      if (nb > vk_coarse_max_n())
        return fail(ctx, VK_ERR_ARG, "a directly solved block exceeds the dense solver limit of 4096 unknowns");
      if (nb > L.cb_max) L.cb_max = nb;
      L.cb_sq += nb * nb;
    }
  }
  if (l > 0) {
    if (!csr_ok(P) || !csr_ok(R)) return fail(ctx, VK_ERR_ARG, "levels >= 1 need prolongation P and restriction R");
    if (P->n_rows != J->n_rows || R->n_cols != J->n_rows || P->n_cols != R->n_rows)
      return fail(ctx, VK_ERR_ARG, "P must be n_l x n_{l-1} and R n_{l-1} x n_l");
    L.P = *P;
    L.R = *R;
    L.has_transfer = true;
    int64_t items = 0;
    for (int gi = 0; gi < n_groups; ++gi) {
      const vk_cell_group& in = groups[gi];
      if (in.n_cells <= 0 || in.n_K <= 0 || in.n_K > VK_MAX_NK)
        return fail(ctx, VK_ERR_ARG, "n_cells must be positive and 1 <= n_K <= 512");
      if (in.n_K > J->n_rows) return fail(ctx, VK_ERR_ARG, "n_K exceeds the number of unknowns");
      if (!in.cell_dofs || !in.colour_cells || !in.colour_ptr || in.n_colours <= 0 || in.n_colours > 64)
        return fail(ctx, VK_ERR_ARG, "cell_dofs, colour_cells, colour_ptr and 1 <= n_colours <= 64 required");
      if (in.colour_ptr[0] != 0 || in.colour_ptr[in.n_colours] != in.n_cells)
        return fail(ctx, VK_ERR_ARG, "colour_ptr must start at 0 and end at n_cells");
      vk_group G;
      for (int c = 0; c < in.n_colours; ++c) {
        const int32_t cnt = in.colour_ptr[c + 1] - in.colour_ptr[c];
        if (cnt < 0) return fail(ctx, VK_ERR_ARG, "colour_ptr must be non-decreasing");
        if (cnt > G.max_colour_cells) G.max_colour_cells = cnt;
      }
      G.n_cells = in.n_cells;
      G.n_K = in.n_K;
      G.cell_dofs = in.cell_dofs;
      G.colour_cells = in.colour_cells;
      G.colour_ptr.assign(in.colour_ptr, in.colour_ptr + in.n_colours + 1);
      G.n_colours = in.n_colours;
      G.y_off = items;
      items += (int64_t)in.n_cells * in.n_K;
      L.groups.push_back(G);
    }
    if (items > INT32_MAX) return fail(ctx, VK_ERR_ARG, "too many (cell, DoF) pairs on one level");
    L.n_items = items;
  }
  // structural validation on the device
  hipStream_t s = ctx->stream;
  VK_TRY(launch_fill_i32(s, 1, 0, ctx->status + 1000));
  VK_TRY(launch_validate_csr(s, L.J, ctx->status + 1000));
  if (l > 0) {
    VK_TRY(launch_validate_csr(s, L.P, ctx->status + 1000));
    VK_TRY(launch_validate_csr(s, L.R, ctx->status + 1000));
    for (const vk_group& G : L.groups)
      VK_TRY(launch_validate_cells(s, G.n_cells, G.n_K, G.cell_dofs, L.J.n_rows, G.colour_cells,
                                   ctx->status + 1000));
  }
  int32_t flag = 0;
  VK_CHECK(to_host(ctx, &flag, ctx->status + 1000, sizeof(int32_t)));
  if (flag != 0) {
    char buf[256];
    snprintf(buf, sizeof(buf),
             "level %d failed validation (flags 0x%x: 1/2 row pointers, 4 column range, 8 unsorted or duplicate "
             "columns, 16 cell DoF range, 32 colour cell range)",
             l, flag);
    return fail(ctx, VK_ERR_ARG, buf);
  }
  L.lpr_J = vk_pick_lpr(L.J.n_rows, L.J.nnz);
  if (l > 0) {
    L.lpr_P = vk_pick_lpr(L.P.n_rows, L.P.nnz);
    L.lpr_R = vk_pick_lpr(L.R.n_rows, L.R.nnz);
  }
  L.set = true;
  ctx->lv[l] = L;
  if (l == ctx->n_levels - 1) {
    ctx->seg_rows = {0, L.J.n_rows};
    ctx->n_seg = 1;
  }
  ctx->ws_ready = false;
  ctx->setup_done = false;
  return VK_OK;
}

vk_status vk_set_level(vk_ctx* ctx, int32_t l, const vk_csr* J, const vk_csr* P, const vk_csr* R, int32_t n_cells,
                       int32_t n_K, const int32_t* cell_dofs, const int32_t* colour_cells,
                       const int32_t* colour_ptr, int32_t n_colours) {
  if (!ctx) return VK_ERR_ARG;
  if (l == 0) {
    if (!J) return fail(ctx, VK_ERR_ARG, "J must be a non-empty square CSR matrix with valid pointers");
    const int64_t rows[2] = {0, J->n_rows};
    return vk_set_level_groups(ctx, 0, J, nullptr, nullptr, 0, nullptr, 1, rows);
  }
  vk_cell_group g{n_cells, n_K, cell_dofs, colour_cells, colour_ptr, n_colours};
  return vk_set_level_groups(ctx, l, J, P, R, 1, &g, 0, nullptr);
}

vk_status vk_set_segments(vk_ctx* ctx, int32_t n_seg, const int64_t* seg_rows) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  const vk_level& F = ctx->lv[ctx->n_levels - 1];
  if (!F.set) return fail(ctx, VK_ERR_STATE, "set the finest level before its segments");
  if (n_seg < 1 || n_seg > 4096 || !seg_rows) return fail(ctx, VK_ERR_ARG, "1 <= n_seg <= 4096 segments required");
  if (seg_rows[0] != 0 || seg_rows[n_seg] != F.J.n_rows)
    return fail(ctx, VK_ERR_ARG, "segments must start at 0 and end at the finest level's size");
  for (int i = 0; i < n_seg; ++i)
    if (seg_rows[i + 1] <= seg_rows[i]) return fail(ctx, VK_ERR_ARG, "segments must be non-empty and increasing");
  ctx->seg_rows.assign(seg_rows, seg_rows + n_seg + 1);
  ctx->n_seg = n_seg;
  ctx->ws_ready = false;
  ctx->setup_done = false;
  return VK_OK;
}

size_t vk_workspace_bytes(const vk_ctx* cctx, vk_prec prec, int32_t restart) {
  if (!cctx || restart < 1 || restart > VK_MAX_RESTART) return 0;
  if (prec != VK_F64 && prec != VK_F32 && prec != VK_BF16) return 0;
  if (!levels_consistent(cctx, nullptr)) return 0;
  vk_ctx tmp = *cctx;  // plan on a copy: the query does not touch the context
  tmp.ev.clear();
  return plan_workspace(&tmp, prec, restart, nullptr);
}

vk_status vk_set_workspace(vk_ctx* ctx, void* dev, size_t bytes, vk_prec prec, int32_t restart) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);  // block inversions still reading the old setup
  for (hipStream_t x : ctx->xside) (void)hipStreamSynchronize(x);
  if (ctx->setup) (void)hipStreamSynchronize(ctx->setup);  // and patch inversions after a failed setup
  ctx->coarse_pending = false;
  ctx->coarse_check_due = false;
  ctx->patch_pending = 0;
  ctx->patch_check_due = false;
  if (prec != VK_F64 && prec != VK_F32 && prec != VK_BF16) return fail(ctx, VK_ERR_ARG, "unknown precision");
  if (restart < 1 || restart > VK_MAX_RESTART) return fail(ctx, VK_ERR_ARG, "restart must be in [1, 64]");
  std::string why;
  if (!levels_consistent(ctx, &why)) return fail(ctx, VK_ERR_STATE, why);
  if (!dev || (reinterpret_cast<uintptr_t>(dev) & 255u)) return fail(ctx, VK_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  vk_ctx probe = *ctx;
  probe.ev.clear();
  const size_t need = plan_workspace(&probe, prec, restart, nullptr);
  if (bytes < need) {
    char buf[160];
    snprintf(buf, sizeof(buf), "workspace of %zu bytes is smaller than the %zu required", bytes, need);
    return fail(ctx, VK_ERR_WORKSPACE, buf);
  }
  for (int l = 1; l < ctx->n_levels; ++l) {
    for (const vk_group& G : ctx->lv[l].groups) {
      const int ld = (int)round_up(G.n_K, vk_prec_vw(prec));
      const int cpb = G.cpb_override > 0 ? G.cpb_override : vk_default_cpb(G.n_K, ld, prec);
      if (cpb <= 0 || VK_NT / cpb < ld / vk_prec_vw(prec))
        return fail(ctx, VK_ERR_ARG, "patch too wide for the apply kernel at this precision / tile");
    }
  }
  ctx->ws = reinterpret_cast<char*>(dev);
  ctx->ws_bytes = bytes;
  ctx->prec = prec;
  ctx->restart = restart;
  plan_workspace(ctx, prec, restart, ctx->ws);
  VK_CHECK(upload_tables(ctx));
  ctx->ws_ready = true;
  ctx->setup_done = false;
  ctx->maps_ready = false;
  for (int l = 0; l < ctx->n_levels; ++l)
    for (vk_group& G : ctx->lv[l].groups) G.cpb_tuned = 0;
  return VK_OK;
}

vk_status vanka_setup(vk_ctx* ctx, double omega, vk_mode mode, int32_t* bad_level, int32_t* bad_cell) {
  if (!ctx) return VK_ERR_ARG;
  if (bad_level) *bad_level = -1;
  if (bad_cell) *bad_cell = -1;
  if (!ctx->ws_ready) return fail(ctx, VK_ERR_WORKSPACE, "workspace not set");
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(ctx, VK_ERR_ARG, "omega must be positive");
  if (mode != VK_ADDITIVE && mode != VK_MULT_COLOURED) return fail(ctx, VK_ERR_ARG, "unknown smoother mode");
  ctx->setup_done = false;
  // the previous setup's block inversions (and their status words) come before this one's
  VK_CHECK(coarse_wait(ctx, false));
  VK_CHECK(patch_settle(ctx, false));  // the last setup's coarser levels still write their status words
  ctx->coarse_check_due = false;
  // recorded graphs stay valid across setups unless omega, the mode or where an inverse lives changes
  if (omega != ctx->omega || mode != ctx->mode) ++ctx->gen;
  ctx->omega = omega;
  ctx->mode = mode;
  std::vector<double*> old_W;
  for (const vk_level& L : ctx->lv) old_W.push_back(L.cb_W);
  hipStream_t s = ctx->stream;
  // status words: [0] directly solved blocks (pivot), [1] block coupling, [64 + l] first singular cell of level l
  // ([600 + l] the largest DoF multiplicity of level l, [1000] the input validation flag)
  VK_TRY(launch_fill_i32(s, 2, INT_MAX, ctx->status));
  VK_TRY(launch_fill_i32(s, 1, 0, ctx->status + 1));
  VK_TRY(launch_fill_i32(s, 64, INT_MAX, ctx->status + 64));
  // the block inversions occupy one workgroup per block: run them on the side
  // stream while the patch inversions fill the rest of the GPU
  VK_TRY(hipEventRecord(ctx->fork_ev, s));
  VK_TRY(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
  // the patch inversions on the CU-masked setup stream
  const hipStream_t ps = ctx->setup ? ctx->setup : s;
  if (ps != s) VK_TRY(hipStreamWaitEvent(ps, ctx->fork_ev, 0));
  if (!ctx->maps_ready) {
    // multiplicities and DoF -> (cell, local) lists depend on the mesh only
    for (int l = 1; l < ctx->n_levels; ++l) {
      vk_level& L = ctx->lv[l];
      int32_t* count = reinterpret_cast<int32_t*>(L.r);
      VK_TRY(launch_fill_i32(ps, L.J.n_rows, 0, count));
      for (const vk_group& G : L.groups) VK_TRY(launch_count_add(ps, G.n_cells, G.n_K, G.cell_dofs, count));
      VK_TRY(launch_inv_count(ps, L.J.n_rows, count, L.inv_p));
      VK_TRY(launch_dof_map(ps, L, count));
    }
    // the colouring: cells of one colour must share no DoF (status words [700 + l]), checked
    // once per mesh with one 64-bit colour mask per DoF in the level's iterate vector
    VK_TRY(launch_fill_i32(ps, 64, 0, ctx->status + 700));
    for (int l = 1; l < ctx->n_levels; ++l) {
      vk_level& L = ctx->lv[l];
      unsigned long long* mask = reinterpret_cast<unsigned long long*>(L.d);
      VK_TRY(launch_fill(ps, L.J.n_rows, 0.0, L.d));
      for (const vk_group& G : L.groups)
        VK_TRY(launch_colour_check(ps, G.n_K, G.cell_dofs, G.colour_cells, G.colour_ptr.data(), G.n_colours, mask,
                                   ctx->status + 700 + l));
    }
    // fixed-width lists when every DoF lies in at most 8 cells (status words [600 + l]: the
    // largest multiplicity of level l); read once per mesh
    VK_TRY(launch_fill_i32(ps, 64, 0, ctx->status + 600));
    for (int l = 1; l < ctx->n_levels; ++l)
      if (!ctx->lv[l].groups.empty()) VK_TRY(launch_dof_max_count(ps, ctx->lv[l], ctx->status + 600 + l));
    // the patch entry maps of the matrix-core inversion (status words [800 + l]: a patch row of
    // level l too long for 16-bit offsets)
    VK_TRY(launch_fill_i32(ps, 64, 0, ctx->status + 800));
    for (int l = 1; l < ctx->n_levels; ++l)
      for (const vk_group& G : ctx->lv[l].groups) VK_TRY(launch_patch_map(ps, ctx->lv[l].J, G, ctx->status + 800 + l));
    VK_TRY(hipStreamSynchronize(ps));
    int32_t mc[64], cc[64], tl[64];
    VK_CHECK(to_host(ctx, mc, ctx->status + 600, sizeof(mc)));
    VK_CHECK(to_host(ctx, cc, ctx->status + 700, sizeof(cc)));
    VK_CHECK(to_host(ctx, tl, ctx->status + 800, sizeof(tl)));
    for (int l = 1; l < ctx->n_levels; ++l)
      for (vk_group& G : ctx->lv[l].groups) G.pmap_ok = G.pmap != nullptr && tl[l] == 0;
    for (int l = 1; l < ctx->n_levels; ++l)
      if (cc[l] != 0)
        return fail(ctx, VK_ERR_ARG, "level " + std::to_string(l) +
                                         ": two cells of one colour share a DoF (the colouring must be DoF-disjoint)");
    for (int l = 1; l < ctx->n_levels; ++l) {
      vk_level& L = ctx->lv[l];
      L.ell_w = L.groups.empty() ? 0 : (mc[l] <= 4 ? 4 : (mc[l] <= 8 ? 8 : 0));
      if (L.ell_w > 0) VK_TRY(launch_dof_ell(ps, L));
    }
  }
  // The finest level first: the context stream waits for its inversions alone, while the coarser
  // levels' run on beside the first V-cycle's finest-level sweeps (each level's event is waited
  // for where that level is first smoothed).
  if (ps != s && ctx->patch_ev.size() < (size_t)ctx->n_levels) {
    for (size_t l = ctx->patch_ev.size(); l < (size_t)ctx->n_levels; ++l) {
      hipEvent_t e = nullptr;
      VK_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ctx->patch_ev.push_back(e);
    }
  }
  for (int l = ctx->n_levels - 1; l >= 1; --l) {
    vk_level& L = ctx->lv[l];
    Timed t(ctx, VK_KERNEL_PATCH_SETUP, l, ps);
    for (const vk_group& G : L.groups) {
      bool handled = false;
      if (ctx->fast_setup)
        VK_TRY(launch_patch_setup_fast(ps, L.J, G, ctx->prec, ctx->status + 64 + l, &handled, ctx->mfma_setup,
                                       ctx->patch_map));
      // wider than LDS and no register-resident kernel: the blocked kernels of the directly
      // solved blocks, one block per cell
      if (!handled && ctx->fast_setup && G.n_K > VK_LDS_SETUP_MAX_NK && G.n_K <= 512 && ctx->blocked.cap > 0) {
        VK_TRY(launch_patch_setup_blocked(ps, L.J, G, ctx->prec, ctx->blocked, ctx->status + 64 + l));
        handled = true;
      }
      if (!handled)
        VK_TRY(launch_patch_setup(ps, L.J, G, ctx->prec, ctx->big_scratch, ctx->big_chunk, ctx->status + 64 + l));
    }
    if (ps != s) VK_TRY(hipEventRecord(ctx->patch_ev[l], ps));
  }
  ctx->patch_pending = 0;
  ctx->patch_check_due = false;
  if (ps != s) {
    const int lf = ctx->n_levels - 1;
    VK_TRY(hipStreamWaitEvent(s, ctx->patch_ev[lf], 0));
    for (int l = 1; l < lf; ++l)
      if (!ctx->lv[l].groups.empty()) ctx->patch_pending |= 1ull << l;
    ctx->patch_check_due = ctx->patch_pending != 0;
  }
  // Block inversions on the side streams, concurrent with the patch inversions (enqueued after
  // them, so the host's launch work does not hold the patch kernels back).  The levels' chains are
  // independent: one stream each, the level with the largest blocks (the longest chain) first.
  std::vector<int> blevels;
  for (int l = 0; l < ctx->n_levels; ++l)
    if (ctx->lv[l].cb_rows.size() > 1) blevels.push_back(l);
  // grouped CSR for the large levels' J (planned once per pattern and workspace, on the host)
  for (int l = 0; l < ctx->n_levels; ++l) {
    vk_level& L = ctx->lv[l];
    if (!L.gJ.planned && L.gJ.gcol) {
      VK_TRY(hipStreamSynchronize(s));  // the last solve may still read the old plan
      if (vk_gcsr_plan(L)) {
        L.use_gJ = ctx->spmv_grouped;
        L.lpr_gJ_lib = vk_pick_lpr_g(L.J.nnz, L.J.n_rows);
        L.lpr_gJ = ctx->spmv_lanes ? ctx->spmv_lanes : L.lpr_gJ_lib;
      } else {
        L.use_gJ = false;
      }
      ++ctx->gen;
    }
  }
  // a single wide block goes through its block-tridiagonal structure where it has one (planned
  // once per pattern and workspace, on the host: the pattern's level sets)
  for (int l : blevels) {
    vk_level& L = ctx->lv[l];
    if (!L.bt.planned) {
      const bool was = L.bt.active;
      if (ctx->coarse_solver == 0) {
        VK_TRY(hipStreamSynchronize(ctx->side));  // the last setup's factorisation still reads the buffers
        (void)vk_bt_plan(L);
      } else {
        L.bt = vk_bt();
        L.bt.planned = true;
      }
      if (L.bt.active || was) ++ctx->gen;
    }
  }
  std::stable_sort(blevels.begin(), blevels.end(),
                   [&](int a, int b) { return ctx->lv[a].cb_max > ctx->lv[b].cb_max; });
  ctx->n_xside = 0;
  for (size_t k = 0; k < blevels.size(); ++k) {
    hipStream_t st = ctx->side;
    if (k > 0) {
      const size_t i = k - 1;
      if (ctx->xside.size() <= i) {
        hipStream_t ns = nullptr;
        hipEvent_t ne = nullptr;
        VK_TRY(hipStreamCreateWithFlags(&ns, hipStreamNonBlocking));
        const hipError_t e = hipEventCreateWithFlags(&ne, hipEventDisableTiming);
        if (e != hipSuccess) {
          (void)hipStreamDestroy(ns);
          return fail_hip(ctx, e, "hipEventCreateWithFlags");
        }
        ctx->xside.push_back(ns);
        ctx->xjoin.push_back(ne);
      }
      st = ctx->xside[i];
      VK_TRY(hipStreamWaitEvent(st, ctx->fork_ev, 0));
    }
    vk_level& L = ctx->lv[blevels[k]];
    {
      Timed t(ctx, VK_KERNEL_BLOCK_INVERT, blevels[k], st);
      // the level with the largest blocks (the longest chain) gets the look-ahead stream
      if (L.bt.active) VK_TRY(launch_bt_factor(st, L, ctx->status));
      else VK_TRY(launch_block_invert(st, L, ctx->status, &L.cb_W, k == 0 ? &ctx->la : nullptr, ctx->coarse_min_tourney));
    }
    if (k > 0) {
      VK_TRY(hipEventRecord(ctx->xjoin[k - 1], st));
      ctx->n_xside = (int)k;
    }
  }
  VK_TRY(hipEventRecord(ctx->join_ev, ctx->side));
  for (int l = 0; l < ctx->n_levels; ++l)
    if (ctx->lv[l].cb_W != old_W[l]) ++ctx->gen;
  // the block inversions keep running on the side stream: the first solve waits for them
  ctx->coarse_pending = true;
  ctx->coarse_check_due = false;
  int32_t st[64];
  VK_CHECK(to_host(ctx, st, ctx->status + 64, sizeof(st)));
  for (int l = 1; l < ctx->n_levels; ++l) {
    if ((ctx->patch_pending >> l) & 1) continue;  // still running: read by the first solve
    if (st[l] != INT_MAX) {
      if (bad_level) *bad_level = l;
      if (bad_cell) *bad_cell = st[l];
      char buf[128];
      snprintf(buf, sizeof(buf), "patch matrix of cell %d on level %d is singular (zero pivot)", st[l], l);
      return fail(ctx, VK_ERR_SINGULAR, buf);
    }
  }
  ctx->setup_done = true;
  ctx->maps_ready = true;
  return VK_OK;
}

vk_status vanka_smooth(vk_ctx* ctx, int32_t l, const double* b, double* d, int32_t sweeps, int32_t d_is_zero) {
  VK_CHECK(ready(ctx));
  VK_CHECK(patch_settle(ctx, true));
  if (l < 1 || l >= ctx->n_levels) return fail(ctx, VK_ERR_ARG, "smoothing needs a level >= 1");
  if (!b || !d || sweeps < 0) return fail(ctx, VK_ERR_ARG, "null vector or negative sweep count");
  if (d_is_zero) {
    if (sweeps == 0) {
      VK_TRY(launch_fill(ctx->stream, ctx->lv[l].J.n_rows, 0.0, d));
      return VK_OK;
    }
    return smooth(ctx, l, b, d, sweeps, true);
  }
  return smooth(ctx, l, b, d, sweeps, false);
}

vk_status vanka_smooth_noalloc(vk_ctx* ctx, int32_t l, const double* b, double* d, int32_t sweeps,
                               int32_t d_is_zero) {
  VK_CHECK(ready(ctx));
  VK_CHECK(patch_settle(ctx, true));
  if (l < 1 || l >= ctx->n_levels) return fail(ctx, VK_ERR_ARG, "smoothing needs a level >= 1");
  if (!b || !d || sweeps < 0) return fail(ctx, VK_ERR_ARG, "null vector or negative sweep count");
  if (!ctx->noalloc) return fail(ctx, VK_ERR_STATE, "no fixed scratch on this device");
  const vk_level& L = ctx->lv[l];
  // the scratch: r, then y_K, then the multiplicative mode's local defects (256-byte aligned parts)
  const int64_t sy = ctx->prec == VK_F64 ? 8 : 4;
  int64_t rk = 0;
  for (const vk_group& G : L.groups) rk = std::max(rk, (int64_t)G.max_colour_cells * G.n_K);
  const int64_t off_y = round_up(8 * L.J.n_rows, 256);
  const int64_t off_rk = off_y + round_up(sy * L.n_items, 256);
  const int64_t need = off_rk + 8 * rk;
  if (need > (int64_t)VK_NOALLOC_SCRATCH_BYTES) {
    char buf[200];
    snprintf(buf, sizeof(buf), "level %d needs %lld bytes of scratch; the fixed scratch holds %llu", l,
             (long long)need, (unsigned long long)VK_NOALLOC_SCRATCH_BYTES);
    return fail(ctx, VK_ERR_ARG, buf);
  }
  char* base = reinterpret_cast<char*>(ctx->noalloc);
  const sweep_bufs bufs{reinterpret_cast<double*>(base), base + off_y, reinterpret_cast<double*>(base + off_rk)};
  if (d_is_zero && sweeps == 0) {
    VK_TRY(launch_fill(ctx->stream, L.J.n_rows, 0.0, d));
    return VK_OK;
  }
  return smooth_with(ctx, l, b, d, sweeps, d_is_zero != 0, bufs);
}

vk_status vcycle(vk_ctx* ctx, const double* b, double* x, int32_t nu_pre, int32_t nu_post) {
  VK_CHECK(ready(ctx));
  if (!b || !x || b == x) return fail(ctx, VK_ERR_ARG, "b and x must be distinct non-null vectors");
  if (nu_pre < 0 || nu_post < 0) return fail(ctx, VK_ERR_ARG, "negative sweep count");
  VK_CHECK(patch_settle(ctx, true));
  VK_CHECK(coarse_wait(ctx, true));
  const int64_t key[6] = {(int64_t)(uintptr_t)b, (int64_t)(uintptr_t)x, nu_pre, nu_post, 0, 0};
  return replay(ctx, 0, key, [&]() { return vcycle_level(ctx, ctx->n_levels - 1, b, x, nu_pre, nu_post); });
}

vk_status gmres_solve(vk_ctx* ctx, const double* b, double* x, int32_t restart, int32_t max_iter, double rtol,
                      double atol, int32_t nu_pre, int32_t nu_post, int32_t* iters, double* true_rel_res,
                      double* history) {
  VK_CHECK(ready(ctx));
  if (!b || !x || b == x) return fail(ctx, VK_ERR_ARG, "b and x must be distinct non-null vectors");
  if (restart < 1 || restart > ctx->restart) return fail(ctx, VK_ERR_ARG, "restart exceeds the workspace's value");
  if (max_iter < 0 || nu_pre < 0 || nu_post < 0 || !(rtol >= 0.0) || !(atol >= 0.0))
    return fail(ctx, VK_ERR_ARG, "negative iteration count, sweep count or tolerance");
  if (iters) *iters = 0;
  if (true_rel_res) *true_rel_res = 0.0;
  hipStream_t s = ctx->stream;
  const int L = ctx->n_levels - 1;
  vk_level& F = ctx->lv[L];
  const int64_t n = F.J.n_rows, ldv = ctx->n_pad;
  const int32_t ldh = restart + 1;
  double* sc = ctx->scal;
  double hb[2];
  VK_TRY(launch_dot(s, n, b, b, ctx->partial, ctx->n_partial, sc + 0, true));
  VK_CHECK(read_scalars(ctx, sc + 0, 1, hb));
  const double bnorm = hb[0];
  if (!std::isfinite(bnorm)) return fail(ctx, VK_ERR_ARG, "right-hand side is not finite");
  if (bnorm == 0.0) {
    VK_TRY(launch_fill(s, n, 0.0, x));
    VK_TRY(hipStreamSynchronize(s));
    if (history) history[0] = 0.0;
    return VK_OK;
  }
  const double tol = std::fmax(rtol * bnorm, atol);
  int32_t its = 0;
  bool first = true;
  bool converged = false;
  double beta = 0.0;
  double r_start = 0.0, r_last = 0.0;  // residual estimates: at the first restart's start, latest
  for (;;) {
    double* V0 = ctx->V;
    VK_TRY(launch_spmv_J(s, F, -1.0, x, 1.0, b, V0));
    VK_TRY(launch_dot(s, n, V0, V0, ctx->partial, ctx->n_partial, sc + 1, true));
    VK_CHECK(read_scalars(ctx, sc + 1, 1, hb));
    beta = hb[0];
    if (!std::isfinite(beta)) return fail(ctx, VK_ERR_BREAKDOWN, "residual is not finite");
    if (first) {
      if (history) history[0] = beta;
      first = false;
      r_start = beta;
    }
    r_last = beta;
    if (beta <= tol) {
      converged = true;
      break;
    }
    if (its >= max_iter) break;
    VK_TRY(launch_scale_by_inv(s, n, V0, sc + 1, V0));
    VK_TRY(launch_gmres_init(s, restart, ctx->H, ctx->g, sc + 1));
    // Step j writes |g_{j+1}| and ||w|| to ghist[2j], ghist[2j + 1] and nothing the earlier steps'
    // results depend on (column j of H, rotation j, g[j], g[j + 1], v_{j+1}, z_j), so steps enqueued
    // past the stopping step leave the iterate unchanged: the host enqueues several steps, reads
    // their estimates in one round trip and takes the first that stops.
    int32_t jn = 0, j = 0;
    bool stop = false;
    while (!stop && j < restart && its < max_iter) {
      int32_t ahead = steps_ahead(r_start, r_last, its, tol);
      ahead = std::min(ahead, std::min(restart - j, max_iter - its));
      const int32_t j0 = j;
      for (int32_t q = 0; q < ahead; ++q, ++j) {
        double* Vj = ctx->V + (int64_t)j * ldv;
        double* Vn = ctx->V + (int64_t)(j + 1) * ldv;
        double* Zj = ctx->Z + (int64_t)j * ldv;
        double* Hc = ctx->H + (int64_t)j * ldh;
        double* out = ctx->ghist + 2 * (int64_t)j;
        const int32_t jj = j;
        auto step = [&]() -> vk_status {
          hipStream_t qs = ctx->stream;
          VK_CHECK(vcycle_level(ctx, L, Vj, Zj, nu_pre, nu_post));
          VK_TRY(launch_spmv_J(qs, F, 1.0, Zj, 0.0, nullptr, Vn));
          // classical Gram-Schmidt, applied twice
          VK_TRY(launch_mdot(qs, n, ctx->V, ldv, jj + 1, Vn, ctx->partial, ctx->n_partial, Hc));
          VK_TRY(launch_maxpy(qs, n, ctx->V, ldv, jj + 1, Hc, -1.0, Vn));
          VK_TRY(launch_mdot(qs, n, ctx->V, ldv, jj + 1, Vn, ctx->partial, ctx->n_partial, ctx->h2));
          VK_TRY(launch_maxpy(qs, n, ctx->V, ldv, jj + 1, ctx->h2, -1.0, Vn));
          VK_TRY(launch_dot(qs, n, Vn, Vn, ctx->partial, ctx->n_partial, Hc + jj + 1, true));
          VK_TRY(launch_givens(qs, jj, ldh, ctx->H, ctx->h2, ctx->cs, ctx->sn, ctx->g, out));
          VK_TRY(launch_scale_by_inv(qs, n, Vn, out + 1, Vn));
          return VK_OK;
        };
        const int64_t key[6] = {jj, ldh, nu_pre, nu_post, 0, 0};
        VK_CHECK(replay(ctx, 1 + (size_t)jj, key, step));
      }
      double gh[2 * VK_MAX_RESTART];
      VK_CHECK(read_scalars(ctx, ctx->ghist + 2 * (int64_t)j0, 2 * (j - j0), gh));
      VK_CHECK(coarse_check(ctx));
      for (int32_t t = 0; t < j - j0; ++t) {
        const double est = gh[2 * t], hn = gh[2 * t + 1];
        ++its;
        jn = j0 + t + 1;
        if (history) history[its] = est;
        if (!std::isfinite(est) || !std::isfinite(hn))
          return fail(ctx, VK_ERR_BREAKDOWN, "non-finite value in the Arnoldi process");
        r_last = est;
        if (est <= tol || hn == 0.0 || its >= max_iter) {
          stop = true;
          break;
        }
      }
    }
    VK_TRY(launch_trisolve(s, jn, ldh, ctx->H, ctx->g, ctx->y));
    VK_TRY(launch_maxpy(s, n, ctx->Z, ldv, jn, ctx->y, 1.0, x));
  }
  if (iters) *iters = its;
  if (true_rel_res) *true_rel_res = beta / bnorm;
  if (!converged) {
    char buf[160];
    snprintf(buf, sizeof(buf), "GMRES reached %d iterations with relative residual %.3e", its, beta / bnorm);
    return fail(ctx, VK_ERR_NOCONV, buf);
  }
  return VK_OK;
}

vk_status gmres_solve_batched(vk_ctx* ctx, const double* b, double* x, int32_t restart, int32_t max_iter,
                              double rtol, double atol, int32_t nu_pre, int32_t nu_post, int32_t* iters,
                              double* true_rel_res, int32_t* all_converged) {
  VK_CHECK(ready(ctx));
  if (!b || !x || b == x) return fail(ctx, VK_ERR_ARG, "b and x must be distinct non-null vectors");
  if (restart < 1 || restart > ctx->restart) return fail(ctx, VK_ERR_ARG, "restart exceeds the workspace's value");
  if (max_iter < 0 || nu_pre < 0 || nu_post < 0 || !(rtol >= 0.0) || !(atol >= 0.0))
    return fail(ctx, VK_ERR_ARG, "negative iteration count, sweep count or tolerance");
  if (!iters || !true_rel_res) return fail(ctx, VK_ERR_ARG, "per-segment outputs required");
  hipStream_t s = ctx->stream;
  const int L = ctx->n_levels - 1;
  vk_level& F = ctx->lv[L];
  const int32_t ns = ctx->n_seg;
  const int64_t ldv = ctx->n_pad;
  const int32_t m = restart;
  int64_t max_len = 0;
  for (int i = 0; i < ns; ++i) max_len = std::max(max_len, ctx->seg_rows[i + 1] - ctx->seg_rows[i]);
  const int64_t* seg = ctx->d_seg;
  double* bnorm = ctx->seg_scal;
  double* tol = bnorm + ns;
  double* beta = tol + ns;
  double* resid = beta + ns;  // resid[ns .. 2 ns) = norms of the new Arnoldi vectors
  int32_t* active = ctx->seg_flags;
  int32_t* its = active + ns;
  int32_t* jn = its + ns;
  const int64_t hs = (int64_t)(m + 1) * m;
  std::vector<double> hb(ns);
  std::vector<int32_t> hi(ns);
  VK_TRY(launch_seg_dot(s, ns, seg, max_len, b, b, ctx->partial, ctx->n_partial, bnorm, true));
  VK_CHECK(to_host(ctx, hb.data(), bnorm, sizeof(double) * ns));
  std::vector<double> tl(ns), bn(hb);
  for (int i = 0; i < ns; ++i) {
    if (!std::isfinite(bn[i])) return fail(ctx, VK_ERR_ARG, "right-hand side is not finite");
    // b_i = 0: x_i = 0 is exact; an infinite tolerance keeps the segment inactive
    tl[i] = bn[i] == 0.0 ? __builtin_inf() : std::fmax(rtol * bn[i], atol);
  }
  VK_CHECK(to_dev(ctx, tol, tl.data(), sizeof(double) * ns));
  VK_TRY(launch_fill_i32(s, ns, 0, its));
  int32_t done_steps = 0;  // Arnoldi steps over all cycles (every system starts at step 0)
  for (;;) {
    double* V0 = ctx->V;
    VK_TRY(launch_spmv_J(s, F, -1.0, x, 1.0, b, V0));
    VK_TRY(launch_seg_dot(s, ns, seg, max_len, V0, V0, ctx->partial, ctx->n_partial, beta, true));
    VK_TRY(launch_seg_init(s, ns, m, ctx->H, ctx->g, beta, tol, its, max_iter, active, jn));
    VK_CHECK(to_host(ctx, hi.data(), active, sizeof(int32_t) * ns));
    int n_active = 0;
    for (int i = 0; i < ns; ++i) n_active += hi[i];
    if (n_active == 0) break;
    VK_TRY(launch_seg_scale(s, ns, seg, max_len, V0, beta, active, V0));
    // The stopping test runs on the device (seg_givens clears a system's active flag); the host
    // enqueues several steps between looks at the flags.  Steps past the point where every system
    // stopped change nothing (each kernel skips inactive systems, and their jn is frozen), so
    // speculative steps only cost their V-cycle.  The look-ahead uses the slowest active system's
    // mean reduction per step.
    int32_t j_end = 0, j = 0;
    std::vector<double> res_now(ns);
    double worst_start = 0.0, worst_now = 0.0, worst_tol = 0.0;
    while (j < m) {
      const int32_t ahead = std::min(steps_ahead(worst_start, worst_now, done_steps, worst_tol), m - j);
      for (int32_t q0 = 0; q0 < ahead; ++q0, ++j) {
        double* Vj = ctx->V + (int64_t)j * ldv;
        double* Vn = ctx->V + (int64_t)(j + 1) * ldv;
        double* Zj = ctx->Z + (int64_t)j * ldv;
        // classical Gram-Schmidt twice, per segment; the first pass goes into column j of H
        double* Hc = ctx->H + (int64_t)j * (m + 1);
        const int32_t jj = j;
        auto step = [&]() -> vk_status {
          hipStream_t q = ctx->stream;
          VK_CHECK(vcycle_level(ctx, L, Vj, Zj, nu_pre, nu_post));
          VK_TRY(launch_spmv_J(q, F, 1.0, Zj, 0.0, nullptr, Vn));
          VK_TRY(launch_seg_mdot(q, ns, seg, max_len, ctx->V, ldv, jj + 1, Vn, ctx->partial, ctx->n_partial, Hc,
                                 (int32_t)hs));
          VK_TRY(launch_seg_maxpy(q, ns, seg, max_len, ctx->V, ldv, jj + 1, Hc, (int32_t)hs, nullptr, -1.0, Vn));
          VK_TRY(launch_seg_mdot(q, ns, seg, max_len, ctx->V, ldv, jj + 1, Vn, ctx->partial, ctx->n_partial,
                                 ctx->h2, m + 1));
          VK_TRY(launch_seg_maxpy(q, ns, seg, max_len, ctx->V, ldv, jj + 1, ctx->h2, m + 1, nullptr, -1.0, Vn));
          VK_TRY(launch_seg_dot(q, ns, seg, max_len, Vn, Vn, ctx->partial, ctx->n_partial, resid + ns, true));
          VK_TRY(launch_seg_givens(q, ns, jj, m, ctx->H, ctx->h2, ctx->cs, ctx->sn, ctx->g, tol, its, max_iter,
                                   active, jn, resid));
          VK_TRY(launch_seg_scale(q, ns, seg, max_len, Vn, resid + ns, active, Vn));
          return VK_OK;
        };
        const int64_t key[6] = {jj, m, nu_pre, nu_post, max_iter, 0};
        VK_CHECK(replay(ctx, 1 + (size_t)ctx->restart + (size_t)jj, key, step));
      }
      j_end = j;
      done_steps += ahead;
      VK_CHECK(to_host2(ctx, hi.data(), active, sizeof(int32_t) * ns, res_now.data(), resid, sizeof(double) * ns));
      VK_CHECK(coarse_check(ctx));
      n_active = 0;
      // the active system furthest from its tolerance (in reduction factors) sets the look-ahead
      double worst = -1.0;
      for (int i = 0; i < ns; ++i) {
        n_active += hi[i];
        if (!hi[i]) continue;
        const double need = std::log(res_now[i] / tl[i]);
        if (need > worst) {
          worst = need;
          worst_start = bn[i];
          worst_now = res_now[i];
          worst_tol = tl[i];
        }
      }
      if (n_active == 0) break;
    }
    VK_TRY(launch_seg_trisolve(s, ns, m, ctx->H, ctx->g, jn, ctx->y));
    VK_TRY(launch_seg_maxpy(s, ns, seg, max_len, ctx->Z, ldv, j_end, ctx->y, m, nullptr, 1.0, x));
  }
  // final true residuals
  VK_TRY(launch_spmv_J(s, F, -1.0, x, 1.0, b, ctx->V));
  VK_TRY(launch_seg_dot(s, ns, seg, max_len, ctx->V, ctx->V, ctx->partial, ctx->n_partial, beta, true));
  VK_CHECK(to_host(ctx, hb.data(), beta, sizeof(double) * ns));
  VK_CHECK(to_host(ctx, iters, its, sizeof(int32_t) * ns));
  int conv = 1;
  for (int i = 0; i < ns; ++i) {
    true_rel_res[i] = bn[i] > 0.0 ? hb[i] / bn[i] : 0.0;
    if (!(bn[i] == 0.0 || hb[i] <= tl[i])) conv = 0;
  }
  if (all_converged) *all_converged = conv;
  if (!conv) return fail(ctx, VK_ERR_NOCONV, "at least one system did not reach the tolerance");
  return VK_OK;
}

vk_status vk_spmv(vk_ctx* ctx, int32_t l, double alpha, const double* x, double beta, const double* z, double* y) {
  if (!ctx) return VK_ERR_ARG;
  if (l < 0 || l >= ctx->n_levels || !ctx->lv[l].set) return fail(ctx, VK_ERR_ARG, "level not set");
  if (!x || !y || (beta != 0.0 && !z)) return fail(ctx, VK_ERR_ARG, "null vector");
  if (x == y) return fail(ctx, VK_ERR_ARG, "x must not alias y");
  const vk_level& L = ctx->lv[l];
  VK_TRY(launch_spmv_J(ctx->stream, L, alpha, x, beta, z, y));
  return VK_OK;
}

vk_status vk_get_patch_inverses(vk_ctx* ctx, int32_t l, int32_t cell0, int32_t n, double* out) {
  VK_CHECK(ready(ctx));
  if (l < 1 || l >= ctx->n_levels || ctx->lv[l].groups.empty())
    return fail(ctx, VK_ERR_ARG, "patch inverses exist on levels >= 1");
  const vk_group& G = ctx->lv[l].groups[0];
  if (cell0 < 0 || n < 0 || (int64_t)cell0 + n > G.n_cells || !out) return fail(ctx, VK_ERR_ARG, "cell range");
  VK_CHECK(patch_settle(ctx, true));
  VK_TRY(launch_patch_export(ctx->stream, G, ctx->prec, cell0, n, out));
  return VK_OK;
}

vk_status vk_get_coarse_inverse(vk_ctx* ctx, double* out) {
  VK_CHECK(ready(ctx));
  if (!out) return fail(ctx, VK_ERR_ARG, "null output");
  if (ctx->lv[0].bt.active)
    return fail(ctx, VK_ERR_STATE,
                "the coarsest level is factorised block by block, not inverted (vk_set_coarse_solver 1 keeps the "
                "dense inverse)");
  VK_CHECK(coarse_wait(ctx, true));
  VK_TRY(launch_block_export(ctx->stream, ctx->lv[0], 0, out));
  return VK_OK;
}

vk_status vk_set_patch_tile(vk_ctx* ctx, int32_t l, int32_t cells_per_block) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  if (l < 1 || l >= ctx->n_levels || !ctx->lv[l].set) return fail(ctx, VK_ERR_ARG, "level not set");
  if (!(cells_per_block == 0 || cells_per_block == 1 || cells_per_block == 2 || cells_per_block == 4 ||
        cells_per_block == 8))
    return fail(ctx, VK_ERR_ARG, "cells_per_block must be 0, 1, 2, 4 or 8");
  vk_level& L = ctx->lv[l];
  for (const vk_group& G : L.groups)
    if (ctx->ws_ready && cells_per_block > 0 && VK_NT / cells_per_block < G.ld / vk_prec_vw(ctx->prec))
      return fail(ctx, VK_ERR_ARG, "tile leaves fewer threads per cell than 16-byte vectors per column");
  for (vk_group& G : L.groups) G.cpb_override = cells_per_block;
  return VK_OK;
}

vk_status vk_patch_layout(const vk_ctx* ctx, int32_t l, int64_t* bytes_per_cell, int32_t* ld) {
  if (!ctx || l < 1 || l >= ctx->n_levels || !ctx->ws_ready || ctx->lv[l].groups.empty()) return VK_ERR_ARG;
  const vk_group& G = ctx->lv[l].groups[0];
  if (bytes_per_cell) *bytes_per_cell = G.cell_stride * vk_prec_bytes(ctx->prec);
  if (ld) *ld = G.ld;
  return VK_OK;
}

vk_status vk_autotune(vk_ctx* ctx, int32_t reps) {
  VK_CHECK(ready(ctx));
  VK_CHECK(patch_settle(ctx, true));
  ++ctx->gen;
  if (reps < 1) reps = 1;
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  VK_TRY(hipEventCreate(&e0));
  VK_TRY(hipEventCreate(&e1));
  auto time_ms = [&](auto&& launch) -> float {
    if (launch() != hipSuccess) return 1e30f;  // warm-up
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps; ++i)
      if (launch() != hipSuccess) return 1e30f;
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 1e30f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms;
  };
  const int lprs[7] = {1, 2, 4, 8, 16, 32, 64};
  for (int l = 0; l < ctx->n_levels; ++l) {
    vk_level& L = ctx->lv[l];
    VK_TRY(launch_fill(s, L.J.n_rows, 1.0, L.b));
    auto tune_csr = [&](const vk_csr& A, double* x, double* y) -> int {
      int best = 4;
      float tb = 1e30f;
      for (int lpr : lprs) {
        if (lpr < 4 && A.nnz >= 16 * A.n_rows) continue;  // one or two lanes only for short rows
        const float t = time_ms([&] { return launch_spmv(s, A, lpr, 1.0, x, 0.0, nullptr, y); });
        if (t < tb) { tb = t; best = lpr; }
      }
      return best;
    };
    L.lpr_J = tune_csr(L.J, L.b, L.r);
    if (L.gJ.active && ctx->spmv_grouped) {  // the grouped format against the best CSR launch
      float tb = time_ms([&] { return launch_spmv(s, L.J, L.lpr_J, 1.0, L.b, 0.0, nullptr, L.r); });
      L.use_gJ = false;
      for (int lpr : {4, 8, 16, 32, 64}) {
        if (ctx->spmv_lanes ? lpr != ctx->spmv_lanes : lpr == 4) continue;  // 4: only when asked for
        const float t = time_ms([&] { return launch_spmv_g(s, L.J, L.gJ, lpr, 1.0, L.b, 0.0, nullptr, L.r); });
        if (t < tb) {
          tb = t;
          L.use_gJ = true;
          L.lpr_gJ = lpr;
          if (!ctx->spmv_lanes) L.lpr_gJ_lib = lpr;
        }
      }
    }
    if (l == 0) continue;
    vk_level& C = ctx->lv[l - 1];
    VK_TRY(launch_fill(s, C.J.n_rows, 1.0, C.b));
    L.lpr_P = tune_csr(L.P, C.b, L.r);
    L.lpr_R = tune_csr(L.R, L.b, C.r);
    for (vk_group& G : L.groups) {
      int best = 0;
      float tb = 1e30f;
      for (int cpb : {1, 2, 4, 8}) {
        if (VK_NT / cpb < G.ld / vk_prec_vw(ctx->prec)) continue;
        const float t = time_ms([&] { return launch_patch_gemv(s, G, ctx->prec, L.b, ctx->Y, cpb); });
        if (t < tb) { tb = t; best = cpb; }
      }
      G.cpb_tuned = best;
    }
  }
  VK_TRY(hipEventDestroy(e0));
  VK_TRY(hipEventDestroy(e1));
  // The GEMV tiles once more, inside V-cycles from the finest level, which move every level's
  // data through the caches as the solve does: back-to-back launches of one tile reread inverses
  // the last-level cache still holds (176x32 dG(2): 4 and 8 cells per workgroup time alike back
  // to back, 16.8 and 18.5 us inside the solve).  Levels with one cell group; the candidates
  // alternate over three rounds of `reps` V-cycles, every GEMV launch timed by its own events.
  const int Lf = ctx->n_levels - 1;
  bool single = false;
  for (int l = 1; l <= Lf; ++l) single = single || ctx->lv[l].groups.size() == 1;
  if (single && ctx->n_levels <= 32 && ctx->sweep_variant != VK_SWEEP_COLOURED_SCATTER) {
    const bool t_on = ctx->timing;
    const int32_t t_level = ctx->timing_level, t_every = ctx->timing_every;
    const uint32_t t_kinds = ctx->timing_kinds;
    const int cands[4] = {1, 2, 4, 8};
    int32_t first[32] = {0};
    bool valid[32][4] = {};
    double tot[32][4] = {};
    int64_t cnt[32][4] = {};
    for (int l = 1; l <= Lf; ++l)
      if (ctx->lv[l].groups.size() == 1) {
        const vk_group& G = ctx->lv[l].groups[0];
        first[l] = G.cpb_tuned;
        for (int c = 0; c < 4; ++c) valid[l][c] = VK_NT / cands[c] >= G.ld / vk_prec_vw(ctx->prec);
      }
    vk_level& F = ctx->lv[Lf];
    VK_TRY(launch_fill(s, F.J.n_rows, 1.0, F.b));
    vk_status st = ctx->coarse_pending ? coarse_wait(ctx, true) : VK_OK;
    for (int round = 0; round < 3 && st == VK_OK; ++round)
      for (int c = 0; c < 4 && st == VK_OK; ++c) {
        for (int l = 1; l <= Lf; ++l)
          if (ctx->lv[l].groups.size() == 1)
            ctx->lv[l].groups[0].cpb_tuned = valid[l][c] ? cands[c] : first[l];
        if ((st = vk_timing_kinds(ctx, 1u << VK_KERNEL_PATCH_GEMV, 1)) != VK_OK) break;
        if ((st = vk_timing_enable(ctx, 1, -1)) != VK_OK) break;
        for (int r = 0; r < reps && st == VK_OK; ++r) st = vcycle_level(ctx, Lf, F.b, F.d, 2, 2);
        for (int l = 1; l <= Lf && st == VK_OK; ++l) {
          if (ctx->lv[l].groups.size() != 1 || !valid[l][c]) continue;
          int64_t n = 0;
          double ms = 0.0;
          st = vk_timing_read(ctx, VK_KERNEL_PATCH_GEMV, l, &n, &ms);
          tot[l][c] += ms;
          cnt[l][c] += n;
        }
      }
    for (int l = 1; l <= Lf; ++l) {
      if (ctx->lv[l].groups.size() != 1) continue;
      int best = -1;
      for (int c = 0; c < 4; ++c)
        if (valid[l][c] && cnt[l][c] > 0 && (best < 0 || tot[l][c] / cnt[l][c] < tot[l][best] / cnt[l][best]))
          best = c;
      ctx->lv[l].groups[0].cpb_tuned = (st == VK_OK && best >= 0) ? cands[best] : first[l];
    }
    ctx->timing = t_on;
    ctx->timing_level = t_level;
    ctx->timing_kinds = t_kinds;
    ctx->timing_every = t_every;
    ctx->recs.clear();
    ctx->timing_seen = 0;
    if (st != VK_OK) return st;
  }
  return VK_OK;
}

vk_status vk_set_sweep_variant(vk_ctx* ctx, int32_t variant) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  if (variant != VK_SWEEP_DOF_GATHER && variant != VK_SWEEP_COLOURED_SCATTER && variant != VK_SWEEP_DOF_GATHER_OFFSETS)
    return fail(ctx, VK_ERR_ARG, "unknown sweep variant");
  ctx->sweep_variant = variant;
  return VK_OK;
}

vk_status vk_set_setup_variant(vk_ctx* ctx, int32_t variant) {
  if (!ctx) return VK_ERR_ARG;
  if (variant < 0 || variant > 3) return fail(ctx, VK_ERR_ARG, "unknown setup variant");
  ctx->fast_setup = variant != 1;
  ctx->mfma_setup = variant == 0 || variant == 3;
  ctx->patch_map = variant == 0;
  ctx->setup_done = false;
  return VK_OK;
}

vk_status vk_set_spmv_format(vk_ctx* ctx, int32_t grouped) {
  if (!ctx) return VK_ERR_ARG;
  if (grouped != 0 && grouped != 1 && grouped != 4 && grouped != 8 && grouped != 16 && grouped != 32 && grouped != 64)
    return fail(ctx, VK_ERR_ARG, "grouped must be 0, 1, 4, 8, 16, 32 or 64");
  ++ctx->gen;
  ctx->spmv_grouped = grouped != 0;
  ctx->spmv_lanes = grouped > 1 ? grouped : 0;
  for (vk_level& L : ctx->lv) {
    L.use_gJ = ctx->spmv_grouped && L.gJ.active;
    if (L.gJ.active) L.lpr_gJ = ctx->spmv_lanes ? ctx->spmv_lanes : L.lpr_gJ_lib;
  }
  return VK_OK;
}

double vk_spmv_bytes(vk_ctx* ctx, int32_t level) {
  if (!ctx || level < 0 || level >= ctx->n_levels) return -1.0;
  const vk_level& L = ctx->lv[level];
  const double n = (double)L.J.n_rows, nnz = (double)L.J.nnz;
  if (L.use_gJ && L.gJ.active) {
    int64_t words = 0;
    if (hipMemcpy(&words, L.gJ.g_coff + L.gJ.n_groups, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      return -1.0;
    }
    const double ng = (double)L.gJ.n_groups;
    // values, column words, per group its first row, column offset and first value offset; x, z
    // read, y written
    return 8.0 * nnz + 4.0 * (double)words + ng * (4.0 + 8.0 + 8.0) + 24.0 * n;
  }
  return 12.0 * nnz + 8.0 * (n + 1.0) + 24.0 * n;
}

int32_t vk_spmv_format(vk_ctx* ctx, int32_t level) {
  if (!ctx || level < 0 || level >= ctx->n_levels) return -1;
  const vk_level& L = ctx->lv[level];
  return L.use_gJ && L.gJ.active ? L.lpr_gJ : 0;
}

vk_status vk_set_coarse_solver(vk_ctx* ctx, int32_t mode) {
  if (!ctx) return VK_ERR_ARG;
  if (mode != 0 && mode != 1) return fail(ctx, VK_ERR_ARG, "unknown coarse solver");
  if (mode != ctx->coarse_solver) {
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (vk_level& L : ctx->lv) L.bt.planned = false;
  }
  ctx->coarse_solver = mode;
  ctx->setup_done = false;
  return VK_OK;
}

int32_t vk_coarse_plan(vk_ctx* ctx, int32_t level, double* setup_flops) {
  if (!ctx || level < 0 || level >= ctx->n_levels) return -1;
  const vk_level& L = ctx->lv[level];
  if (L.bt.active) {
    if (setup_flops) *setup_flops = L.bt.flops;
    return L.bt.nb;
  }
  if (setup_flops) {
    double f = 0.0;
    for (size_t b = 0; b + 1 < L.cb_rows.size(); ++b) {
      const double m = (double)(L.cb_rows[b + 1] - L.cb_rows[b]);
      f += 2.0 * m * m * m;
    }
    *setup_flops = f;
  }
  return 0;
}

vk_status vk_set_coarse_pivoting(vk_ctx* ctx, int32_t mode) {
  if (!ctx) return VK_ERR_ARG;
  if (mode < 0 || mode > 2) return fail(ctx, VK_ERR_ARG, "unknown coarse pivoting mode");
  ctx->coarse_min_tourney = mode == 0 ? VK_TOURNEY_MIN_N : (mode == 1 ? INT64_MAX : 0);
  ctx->setup_done = false;
  return VK_OK;
}

vk_status vk_set_graphs(vk_ctx* ctx, int32_t enable) {
  if (!ctx) return VK_ERR_ARG;
  if (enable != 0 && enable != 1) return fail(ctx, VK_ERR_ARG, "enable must be 0 or 1");
  if (enable && !ctx->cap) VK_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
  ctx->graphs = enable != 0;
  return VK_OK;
}

vk_status vk_graph_stats(const vk_ctx* ctx, int64_t* captures, int64_t* launches) {
  if (!ctx) return VK_ERR_ARG;
  if (captures) *captures = ctx->graph_captures;
  if (launches) *launches = ctx->graph_launches;
  return VK_OK;
}

vk_status vk_timing_enable(vk_ctx* ctx, int32_t enable, int32_t level) {
  if (!ctx) return VK_ERR_ARG;
  ++ctx->gen;
  if (enable) {
    if (ctx->ev.empty()) {
      ctx->ev.resize(2 * kTimingPool);
      for (auto& e : ctx->ev) VK_TRY(hipEventCreate(&e));
    }
    VK_TRY(hipStreamSynchronize(ctx->stream));
    ctx->recs.clear();
    ctx->timing_seen = 0;
  }
  ctx->timing = enable != 0;
  ctx->timing_level = level;
  return VK_OK;
}

vk_status vk_timing_kinds(vk_ctx* ctx, uint32_t mask, int32_t every) {
  if (!ctx) return VK_ERR_ARG;
  if (every < 1) return fail(ctx, VK_ERR_ARG, "every must be >= 1");
  ctx->timing_kinds = mask;
  ctx->timing_every = every;
  return VK_OK;
}

vk_status vk_timing_read(vk_ctx* ctx, int32_t kind, int32_t l, int64_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return VK_ERR_ARG;
  VK_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->setup) VK_TRY(hipStreamSynchronize(ctx->setup));
  int64_t cnt = 0;
  double tot = 0.0;
  for (const vk_timing_rec& r : ctx->recs) {
    if (r.kind != kind || (l >= 0 && r.level != l)) continue;
    float ms = 0.f;
    VK_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * r.slot], ctx->ev[2 * r.slot + 1]));
    ++cnt;
    tot += ms;
  }
  *launches = cnt;
  *total_ms = tot;
  return VK_OK;
}

}  // extern "C"
