// Vanka patch kernels (Sec. 3, Eq. 3.4 and 3.5):
//   setup : gather J_K = J restricted to dof(K,.) x dof(K,.) and invert it in
//           FP64 (Gauss-Jordan, partial pivoting), store A_K = J_K^{-1};
//   apply : per colour, y_K = A_K r_K (r_K gathered from the defect, or a
//           per-cell defect buffer) and d[dof(K,i)] += omega * s_i * y_K[i]
//           with s = 1/p (averaged additive form) or 1 (multiplicative form);
//   residual : per colour, the local defects (b - J d)[dof(K,.)] of the
//           multiplicative form.
//
// Storage of A_K: column by column, leading dimension ld >= n_K padded so a
// column is a whole number of 16-byte vectors; element (i, j) at j*ld + i.
// A thread owns VW consecutive rows of a column (one 16-byte load) and walks
// the columns of its column group, so consecutive threads read consecutive
// addresses of the same column.
#include <hip/hip_ext.h>

#include "vk_internal.h"

namespace {

template <int P> struct PT;
template <> struct PT<VK_F64> { using S = double;   using A = double; static constexpr int VW = 2; };
template <> struct PT<VK_F32> { using S = float;    using A = float;  static constexpr int VW = 4; };
template <> struct PT<VK_BF16> { using S = uint16_t; using A = float;  static constexpr int VW = 8; };

__device__ inline float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ inline float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int P> __device__ inline void load_vec(const typename PT<P>::S* p, typename PT<P>::A* a);
template <> __device__ inline void load_vec<VK_F64>(const double* p, double* a) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  a[0] = v.x; a[1] = v.y;
}
template <> __device__ inline void load_vec<VK_F32>(const float* p, float* a) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
}
template <> __device__ inline void load_vec<VK_BF16>(const uint16_t* p, float* a) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  a[0] = bf16_lo(v.x); a[1] = bf16_hi(v.x); a[2] = bf16_lo(v.y); a[3] = bf16_hi(v.y);
  a[4] = bf16_lo(v.z); a[5] = bf16_hi(v.z); a[6] = bf16_lo(v.w); a[7] = bf16_hi(v.w);
}

// the same 16 bytes as load_vec, loaded raw (so the load can stay in flight across a barrier)
// and converted later
template <int P> __device__ inline void cvt_vec(uint4 v, typename PT<P>::A* a);
template <> __device__ inline void cvt_vec<VK_F64>(uint4 v, double* a) {
  const double2 d = __builtin_bit_cast(double2, v);
  a[0] = d.x; a[1] = d.y;
}
template <> __device__ inline void cvt_vec<VK_F32>(uint4 v, float* a) {
  const float4 f = __builtin_bit_cast(float4, v);
  a[0] = f.x; a[1] = f.y; a[2] = f.z; a[3] = f.w;
}
template <> __device__ inline void cvt_vec<VK_BF16>(uint4 v, float* a) {
  a[0] = bf16_lo(v.x); a[1] = bf16_hi(v.x); a[2] = bf16_lo(v.y); a[3] = bf16_hi(v.y);
  a[4] = bf16_lo(v.z); a[5] = bf16_hi(v.z); a[6] = bf16_lo(v.w); a[7] = bf16_hi(v.w);
}

template <int P> __device__ inline typename PT<P>::S store_cvt(double v);
template <> __device__ inline double store_cvt<VK_F64>(double v) { return v; }
template <> __device__ inline float store_cvt<VK_F32>(double v) { return (float)v; }
template <> __device__ inline uint16_t store_cvt<VK_BF16>(double v) { return f32_to_bf16_rne((float)v); }

template <int P> __device__ inline double load_cvt(const typename PT<P>::S* p);
template <> __device__ inline double load_cvt<VK_F64>(const double* p) { return *p; }
template <> __device__ inline double load_cvt<VK_F32>(const float* p) { return (double)*p; }
template <> __device__ inline double load_cvt<VK_BF16>(const uint16_t* p) { return (double)bf16_lo(*p); }

// Small per-block arrays of the setup kernels (in LDS).
struct SetupSmem {
  double* fcol;
  double* prow;
  double* pval;
  int* skey;
  int* sloc;
  int* sdof;
  int* perm;
  int* piv;
};

__device__ inline SetupSmem carve_setup_smem(char* base, int n) {
  SetupSmem s;
  s.fcol = reinterpret_cast<double*>(base);
  s.prow = s.fcol + n;
  s.pval = s.prow + n;
  s.skey = reinterpret_cast<int*>(s.pval + 2);
  s.sloc = s.skey + n;
  s.sdof = s.sloc + n;
  s.perm = s.sdof + n;
  s.piv = s.perm + n;
  return s;
}

__host__ __device__ inline size_t setup_small_bytes(int n) { return (size_t)n * (2 * 8 + 4 * 4) + 32; }

// J_K[i][j] = J[dof_i][dof_j] (0 where J stores nothing), row-major in M.
__device__ void gather_patch(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const int32_t* __restrict__ dofs, int n, double* M,
                             SetupSmem& s) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) {
    s.sdof[i] = dofs[i];
    s.skey[i] = 0x7fffffff;
    s.sloc[i] = 0;
  }
  for (int e = tid; e < n * n; e += blockDim.x) M[e] = 0.0;
  __syncthreads();
  // sorted copy of the cell's DoFs (they are distinct): rank sort
  for (int i = tid; i < n; i += blockDim.x) {
    const int v = s.sdof[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (s.sdof[j] < v) ? 1 : 0;
    s.skey[rank] = v;
    s.sloc[rank] = i;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  for (int i = wave; i < n; i += nwave) {
    const int64_t row = s.sdof[i];
    const int64_t e1 = row_ptr[row + 1];
    for (int64_t e = row_ptr[row] + lane; e < e1; e += 64) {
      const int c = col[e];
      int lo = 0, hi = n;  // first key >= c
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s.skey[mid] < c) lo = mid + 1; else hi = mid;
      }
      if (lo < n && s.skey[lo] == c) M[i * n + s.sloc[lo]] = val[e];
    }
  }
  __syncthreads();
}

// In-place Gauss-Jordan inversion with partial (row) pivoting of the n x n
// row-major M, by the whole workgroup.  Pivot = first row of maximal |value|
// in the current column (the pivot sequence of LU with partial pivoting).
// Returns false on a zero or non-finite pivot (M is then meaningless).
__device__ bool gauss_jordan_inverse(double* M, int n, SetupSmem& s) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        const double a = fabs(M[i * n + k]);
        if (a > best) { best = a; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        s.piv[0] = bi;
        s.perm[k] = bi;
        s.pval[0] = bi < n ? M[bi * n + k] : 0.0;
      }
    }
    __syncthreads();
    // pivot index and value come from LDS: the row swap below rewrites M[p][k]
    const int p = s.piv[0];
    const double pv = s.pval[0];
    if (p >= n || pv == 0.0 || !isfinite(pv)) return false;
    if (p != k) {
      for (int j = tid; j < n; j += nt) {
        const double t = M[k * n + j];
        M[k * n + j] = M[p * n + j];
        M[p * n + j] = t;
      }
    }
    __syncthreads();
    const double inv = 1.0 / pv;
    for (int i = tid; i < n; i += nt) s.fcol[i] = M[i * n + k];
    for (int j = tid; j < n; j += nt) s.prow[j] = (j == k ? 1.0 : M[k * n + j]) * inv;
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) {
      const int i = e / n, j = e - i * n;
      M[e] = (i == k) ? s.prow[j] : ((j == k ? 0.0 : M[e]) - s.fcol[i] * s.prow[j]);
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = s.perm[k];
    if (p != k) {
      for (int i = tid; i < n; i += nt) {
        const double t = M[i * n + k];
        M[i * n + k] = M[i * n + p];
        M[i * n + p] = t;
      }
    }
    __syncthreads();
  }
  return true;
}

template <int P>
__device__ void write_inverse(const double* M, int n, typename PT<P>::S* out, int ld) {
  for (int o = threadIdx.x; o < n * ld; o += blockDim.x) {
    const int j = o / ld, i = o - j * ld;
    out[o] = store_cvt<P>(i < n ? M[i * n + j] : 0.0);
  }
}

// One workgroup per cell; M in LDS (n_K <= VK_LDS_SETUP_MAX_NK) or in global
// scratch (one n_K x n_K slab per workgroup of the current chunk).
template <int P, bool GLOBAL>
__global__ __launch_bounds__(VK_NT) void patch_setup_kernel(const int64_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            const int32_t* __restrict__ cell_dofs, int32_t cell0,
                                                            int32_t n, void* inv_out, int32_t ld,
                                                            int64_t cell_stride, double* scratch, int32_t* status) {
  extern __shared__ __align__(16) char smem[];
  const int K = cell0 + blockIdx.x;
  double* M;
  SetupSmem s;
  if (GLOBAL) {
    M = scratch + (int64_t)blockIdx.x * n * n;
    s = carve_setup_smem(smem, n);
  } else {
    M = reinterpret_cast<double*>(smem);
    s = carve_setup_smem(smem + (size_t)n * n * 8, n);
  }
  gather_patch(row_ptr, col, val, cell_dofs + (int64_t)K * n, n, M, s);
  const bool ok = gauss_jordan_inverse(M, n, s);
  if (!ok && threadIdx.x == 0) atomicMin(&status[0], K);
  using S = typename PT<P>::S;
  write_inverse<P>(M, n, reinterpret_cast<S*>(inv_out) + (int64_t)K * cell_stride, ld);
}

template <int P, bool FROM_BUF>
__global__ __launch_bounds__(VK_NT) void patch_apply_kernel(const void* __restrict__ inv_, int32_t ld,
                                                            int64_t cell_stride, int32_t n_K,
                                                            const int32_t* __restrict__ cells, int32_t n_launch,
                                                            const int32_t* __restrict__ cell_dofs,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ rK, double* d,
                                                            const double* __restrict__ inv_p, double omega,
                                                            int32_t cpb) {
  using S = typename PT<P>::S;
  using A = typename PT<P>::A;
  constexpr int VW = PT<P>::VW;
  extern __shared__ __align__(16) char smem[];
  int* sdof = reinterpret_cast<int*>(smem);
  A* srk = reinterpret_cast<A*>(smem + (((size_t)cpb * n_K * 4 + 15) & ~(size_t)15));
  A* part = srk + cpb * n_K;
  const int tpc = VK_NT / cpb;
  const int slot = threadIdx.x / tpc, t = threadIdx.x - slot * tpc;
  const int64_t idx = (int64_t)blockIdx.x * cpb + slot;
  const bool valid = idx < n_launch;
  const int K = valid ? cells[idx] : 0;
  for (int j = t; j < n_K; j += tpc) {
    const int dof = valid ? cell_dofs[(int64_t)K * n_K + j] : 0;
    sdof[slot * n_K + j] = dof;
    double rv = 0.0;
    if (valid) rv = FROM_BUF ? rK[idx * n_K + j] : r[dof];
    srk[slot * n_K + j] = (A)rv;
  }
  __syncthreads();
  const int vpc = ld / VW;
  const int G = tpc / vpc;
  const int g = t / vpc, v = t - g * vpc;
  A acc[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) acc[e] = (A)0;
  if (valid && g < G) {
    const S* base = reinterpret_cast<const S*>(inv_) + (int64_t)K * cell_stride + v * VW;
    const A* rk = srk + slot * n_K;
#pragma unroll 4
    for (int j = g; j < n_K; j += G) {
      A a[VW];
      load_vec<P>(base + (int64_t)j * ld, a);
      const A rj = rk[j];
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[e] = fma(a[e], rj, acc[e]);
    }
  }
  A* mypart = part + slot * tpc * VW;
  if (g < G) {
#pragma unroll
    for (int e = 0; e < VW; ++e) mypart[g * ld + v * VW + e] = acc[e];
  }
  __syncthreads();
  if (valid) {
    for (int i = t; i < n_K; i += tpc) {
      A y = (A)0;
      for (int gg = 0; gg < G; ++gg) y += mypart[gg * ld + i];
      const int dof = sdof[slot * n_K + i];
      const double sc = inv_p ? inv_p[dof] : 1.0;
      d[dof] += omega * sc * (double)y;
    }
  }
}

template <int LPR>
__global__ __launch_bounds__(256) void patch_residual_kernel(const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val,
                                                             const int32_t* __restrict__ cells, int32_t n_launch,
                                                             const int32_t* __restrict__ cell_dofs, int32_t n_K,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ d, double* rK) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t item = gid / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  const bool ok = item < (int64_t)n_launch * n_K;
  double sum = 0.0;
  int dof = 0;
  if (ok) {
    const int64_t idx = item / n_K;
    const int i = (int)(item - idx * n_K);
    dof = cell_dofs[(int64_t)cells[idx] * n_K + i];
    const int64_t e1 = row_ptr[dof + 1];
    for (int64_t e = row_ptr[dof] + lane; e < e1; e += LPR) sum += val[e] * d[col[e]];
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LPR);
  if (ok && lane == 0) rK[item] = b[dof] - sum;
}

__global__ void count_kernel(int64_t total, const int32_t* __restrict__ cell_dofs, int32_t* count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&count[cell_dofs[e]], 1);
}

__global__ void inv_count_kernel(int64_t n, const int32_t* __restrict__ count, double* inv_p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    inv_p[i] = count[i] > 0 ? 1.0 / (double)count[i] : 0.0;
}

template <int P>
__global__ void export_kernel(const void* __restrict__ inv_, int32_t ld, int64_t cell_stride, int32_t n_K,
                              int32_t cell0, int32_t n, double* out) {
  using S = typename PT<P>::S;
  const int64_t total = (int64_t)n * n_K * n_K;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = o / ((int64_t)n_K * n_K);
    const int rem = (int)(o - c * n_K * n_K);
    const int i = rem / n_K, j = rem - i * n_K;
    out[o] = load_cvt<P>(reinterpret_cast<const S*>(inv_) + (cell0 + c) * cell_stride + (int64_t)j * ld + i);
  }
}

inline unsigned capped_grid(int64_t work, int per_block, unsigned cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Patches too wide for LDS and for the register-resident kernels go through the
// blocked Gauss-Jordan kernels of the directly solved blocks (coarse.hip), a
// chunk of cells at a time: each cell's patch matrix is one block.
// ---------------------------------------------------------------------------

// Column-major dense patch matrices of cells [cell0, cell0 + gridDim.x) (zeroed beforehand):
// W_b[c n + i] = J[dof_i][dof_c].  One workgroup per cell, a wavefront per row.
__global__ __launch_bounds__(256) void patch_dense_cm_kernel(int32_t n, int32_t cell0,
                                                             const int32_t* __restrict__ cell_dofs,
                                                             const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val, double* W_all) {
  extern __shared__ int dsm[];
  int* sdof = dsm;
  int* skey = dsm + n;
  int* sloc = dsm + 2 * n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t* dofs = cell_dofs + (int64_t)(cell0 + (int64_t)blockIdx.x) * n;
  for (int i = tid; i < n; i += 256) sdof[i] = dofs[i];
  __syncthreads();
  for (int i = tid; i < n; i += 256) {
    const int v = sdof[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (sdof[j] < v) ? 1 : 0;
    skey[rank] = v;
    sloc[rank] = i;
  }
  __syncthreads();
  double* W = W_all + (int64_t)blockIdx.x * n * n;
  for (int i = wave; i < n; i += 4) {
    const int64_t row = sdof[i];
    const int64_t e1 = row_ptr[row + 1];
    for (int64_t e = row_ptr[row] + lane; e < e1; e += 64) {
      const int c = col[e];
      int lo = 0, hi = n;  // first key >= c
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (skey[mid] < c) lo = mid + 1; else hi = mid;
      }
      if (lo < n && skey[lo] == c) W[(int64_t)sloc[lo] * n + i] = val[e];
    }
  }
}

// rows[b] = b n, woff[b] = b n^2 (b < nb; rows also at nb)
__global__ void block_offsets_kernel(int32_t nb, int64_t n, int64_t* rows, int64_t* woff) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= nb) rows[b] = b * n;
  if (b < nb) woff[b] = b * n * n;
}

// The inverses of the eliminated blocks (row-major W_b, pivot rows q_b) into the patch store:
// J_K^{-1}[k][q_j] = W_b[q_k][j], column-major with leading dimension ld, rows n..ld-1 zero.
template <int P>
__global__ void patch_export_blocked_kernel(int32_t n, int32_t cell0, int32_t nc, const double* __restrict__ W_all,
                                            const int32_t* __restrict__ q_all, void* inv_out, int32_t ld,
                                            int64_t cell_stride) {
  using S = typename PT<P>::S;
  const int64_t per = (int64_t)n * ld, total = (int64_t)nc * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, rem = e - b * per;
    const int j = (int)(rem / ld), k = (int)(rem - (int64_t)j * ld);
    const int32_t* q = q_all + b * n;
    S* out = reinterpret_cast<S*>(inv_out) + (cell0 + b) * cell_stride;
    out[(int64_t)q[j] * ld + k] = store_cvt<P>(k < n ? W_all[b * n * n + (int64_t)q[k] * n + j] : 0.0);
  }
}

template <int P>
hipError_t setup_blocked(hipStream_t s, const vk_csr& J, const vk_group& G, const vk_blocked_ws& ws,
                         int32_t* status) {
  const int64_t n = G.n_K;
  int64_t chunk = ws.cap / (n * n);
  if (ws.rows_cap / n < chunk) chunk = ws.rows_cap / n;
  if (ws.blocks_cap < chunk) chunk = ws.blocks_cap;
  if (chunk < 1 || n > 512) return hipErrorInvalidValue;
  vk_level B;  // the chunk's cells as the blocks of a level
  B.cb_max = n;
  B.cb_a = ws.a;
  B.cb_q = ws.q;
  B.cb_used = ws.used;
  B.cb_gi = ws.gi;
  B.cb_go = ws.go;
  B.d_cb_rows = ws.rows;
  B.d_cb_woff = ws.woff;
  const int32_t nb_max = (int32_t)(G.n_cells < chunk ? G.n_cells : chunk);
  block_offsets_kernel<<<(unsigned)((nb_max + 256) / 256), 256, 0, s>>>(nb_max, n, ws.rows, ws.woff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int32_t c0 = 0; c0 < G.n_cells; c0 += (int32_t)chunk) {
    const int32_t nc = (int32_t)((G.n_cells - c0) < chunk ? (G.n_cells - c0) : chunk);
    B.cb_rows.assign((size_t)nc + 1, 0);
    for (int32_t b = 0; b <= nc; ++b) B.cb_rows[b] = (int64_t)b * n;
    if ((e = launch_fill(s, (int64_t)nc * n * n, 0.0, ws.a)) != hipSuccess) return e;
    patch_dense_cm_kernel<<<(unsigned)nc, 256, (size_t)3 * n * sizeof(int), s>>>((int32_t)n, c0, G.cell_dofs,
                                                                                 J.row_ptr, J.col, J.val, ws.a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_blocks_invert_dense(s, B, status, c0)) != hipSuccess) return e;
    const int64_t total = (int64_t)nc * n * G.ld;
    patch_export_blocked_kernel<P><<<capped_grid(total, 256, 16384), 256, 0, s>>>(
        (int32_t)n, c0, nc, ws.a, ws.q, G.inv, G.ld, G.cell_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t setup_prec(hipStream_t s, const vk_csr& J, const vk_group& L, double* big, int32_t chunk, int32_t* status) {
  const int n = L.n_K;
  if (n <= VK_LDS_SETUP_MAX_NK) {
    const size_t lds = (size_t)n * n * 8 + setup_small_bytes(n);
    patch_setup_kernel<P, false><<<L.n_cells, VK_NT, lds, s>>>(J.row_ptr, J.col, J.val, L.cell_dofs, 0, n,
                                                               L.inv, L.ld, L.cell_stride, nullptr, status);
    return hipGetLastError();
  }
  const size_t lds = setup_small_bytes(n);
  for (int32_t c0 = 0; c0 < L.n_cells; c0 += chunk) {
    const int32_t cnt = (L.n_cells - c0) < chunk ? (L.n_cells - c0) : chunk;
    patch_setup_kernel<P, true><<<cnt, VK_NT, lds, s>>>(J.row_ptr, J.col, J.val, L.cell_dofs, c0, n, L.inv,
                                                        L.ld, L.cell_stride, big, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t apply_prec(hipStream_t s, const vk_group& L, int cpb, int32_t colour, const double* r,
                      const double* rK, double* d, const double* ip, double omega) {
  const int32_t c0 = L.colour_ptr[colour], c1 = L.colour_ptr[colour + 1];
  const int32_t n_launch = c1 - c0;
  if (n_launch <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n_launch + cpb - 1) / cpb);
  constexpr int VW = PT<P>::VW;
  using A = typename PT<P>::A;
  const size_t lds = (((size_t)cpb * L.n_K * 4 + 15) & ~(size_t)15) + (size_t)cpb * L.n_K * sizeof(A) +
                     (size_t)VK_NT * VW * sizeof(A);
  if (rK)
    patch_apply_kernel<P, true><<<grid, VK_NT, lds, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, L.colour_cells + c0,
                                                         n_launch, L.cell_dofs, r, rK, d, ip, omega, cpb);
  else
    patch_apply_kernel<P, false><<<grid, VK_NT, lds, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, L.colour_cells + c0,
                                                          n_launch, L.cell_dofs, r, rK, d, ip, omega, cpb);
  return hipGetLastError();
}

}  // namespace

int vk_prec_vw(vk_prec p) { return p == VK_F64 ? 2 : (p == VK_F32 ? 4 : 8); }
int vk_prec_bytes(vk_prec p) { return p == VK_F64 ? 8 : (p == VK_F32 ? 4 : 2); }

// Cells per 256-thread workgroup: the largest of 8, 4, 2, 1 whose per-cell
// thread count covers a column (tpc >= ld / VW) with at most 1/8 of the
// threads idle; otherwise the one with the fewest idle threads.
int vk_default_cpb(int32_t n_K, int32_t ld, vk_prec prec) {
  (void)n_K;
  const int vpc = ld / vk_prec_vw(prec);
  int best = 0;
  double best_idle = 2.0;
  for (int cpb : {8, 4, 2, 1}) {
    const int tpc = VK_NT / cpb;
    if (tpc < vpc) continue;
    const int G = tpc / vpc;
    const double idle = 1.0 - (double)(G * vpc) / tpc;
    if (idle <= 0.125) return cpb;
    if (idle < best_idle) { best_idle = idle; best = cpb; }
  }
  return best;
}

hipError_t launch_count_add(hipStream_t s, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs, int32_t* count) {
  const int64_t total = (int64_t)n_cells * n_K;
  if (total == 0) return hipSuccess;
  count_kernel<<<capped_grid(total, 256, 4096), 256, 0, s>>>(total, cell_dofs, count);
  return hipGetLastError();
}

hipError_t launch_inv_count(hipStream_t s, int64_t n, const int32_t* count, double* inv_p) {
  inv_count_kernel<<<capped_grid(n, 256, 4096), 256, 0, s>>>(n, count, inv_p);
  return hipGetLastError();
}

hipError_t launch_patch_setup(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec, double* big,
                              int32_t chunk, int32_t* status) {
  if (G.n_cells == 0) return hipSuccess;
  switch (prec) {
    case VK_F64: return setup_prec<VK_F64>(s, J, G, big, chunk, status);
    case VK_F32: return setup_prec<VK_F32>(s, J, G, big, chunk, status);
    default: return setup_prec<VK_BF16>(s, J, G, big, chunk, status);
  }
}

hipError_t launch_patch_apply(hipStream_t s, const vk_group& G, vk_prec prec, int32_t colour, const double* r,
                              const double* rK, double* d, const double* inv_p, double omega) {
  const int cpb = G.cpb_override > 0 ? G.cpb_override : vk_default_cpb(G.n_K, G.ld, prec);
  switch (prec) {
    case VK_F64: return apply_prec<VK_F64>(s, G, cpb, colour, r, rK, d, inv_p, omega);
    case VK_F32: return apply_prec<VK_F32>(s, G, cpb, colour, r, rK, d, inv_p, omega);
    default: return apply_prec<VK_BF16>(s, G, cpb, colour, r, rK, d, inv_p, omega);
  }
}

hipError_t launch_patch_residual(hipStream_t s, const vk_csr& J, int lpr, const vk_group& L, int32_t colour,
                                 const double* b, const double* d, double* rK) {
  const int32_t c0 = L.colour_ptr[colour], c1 = L.colour_ptr[colour + 1];
  const int32_t n_launch = c1 - c0;
  if (n_launch <= 0) return hipSuccess;
  const int64_t items = (int64_t)n_launch * L.n_K;
  const unsigned grid = capped_grid(items * lpr, 256, 0x7fffffff);
  switch (lpr) {
    case 4: patch_residual_kernel<4><<<grid, 256, 0, s>>>(J.row_ptr, J.col, J.val, L.colour_cells + c0, n_launch, L.cell_dofs, L.n_K, b, d, rK); break;
    case 8: patch_residual_kernel<8><<<grid, 256, 0, s>>>(J.row_ptr, J.col, J.val, L.colour_cells + c0, n_launch, L.cell_dofs, L.n_K, b, d, rK); break;
    case 16: patch_residual_kernel<16><<<grid, 256, 0, s>>>(J.row_ptr, J.col, J.val, L.colour_cells + c0, n_launch, L.cell_dofs, L.n_K, b, d, rK); break;
    case 32: patch_residual_kernel<32><<<grid, 256, 0, s>>>(J.row_ptr, J.col, J.val, L.colour_cells + c0, n_launch, L.cell_dofs, L.n_K, b, d, rK); break;
    default: patch_residual_kernel<64><<<grid, 256, 0, s>>>(J.row_ptr, J.col, J.val, L.colour_cells + c0, n_launch, L.cell_dofs, L.n_K, b, d, rK); break;
  }
  return hipGetLastError();
}

hipError_t launch_patch_export(hipStream_t s, const vk_group& L, vk_prec prec, int32_t cell0, int32_t n,
                               double* out) {
  const int64_t total = (int64_t)n * L.n_K * L.n_K;
  if (total == 0) return hipSuccess;
  const unsigned g = capped_grid(total, 256, 8192);
  switch (prec) {
    case VK_F64: export_kernel<VK_F64><<<g, 256, 0, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, cell0, n, out); break;
    case VK_F32: export_kernel<VK_F32><<<g, 256, 0, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, cell0, n, out); break;
    default: export_kernel<VK_BF16><<<g, 256, 0, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, cell0, n, out); break;
  }
  return hipGetLastError();
}

// ===========================================================================
// Setup with one lane per patch row, rows held in registers (n_K = N known at
// compile time).  Gauss-Jordan elimination with implicit partial pivoting: at
// step k the pivot is the not-yet-used row with the largest |value| in column
// k (first such row on ties); rows never move.  With q_k the pivot row of
// step k, the stored rows W satisfy J_K^{-1}[k][q_j] = W[q_k][j].
// The patch rows are staged through LDS in chunks of CH rows (the gather
// scatters CSR entries by column, which registers cannot be indexed by).
// ===========================================================================
namespace {

template <int N> struct RowCfg {
  static constexpr int W = (N + 63) / 64;          // wavefronts per cell
  static constexpr int CH = 16;                    // staged rows per chunk (<= 11 KiB of LDS)
  static constexpr int U = 7;                      // elimination steps per register rotation
};

template <int P, int N>
__global__ __launch_bounds__(64 * RowCfg<N>::W) void patch_setup_rows_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const int32_t* __restrict__ cell_dofs, void* inv_out, int32_t ld, int64_t cell_stride, int32_t* status) {
  constexpr int W = RowCfg<N>::W, CH = RowCfg<N>::CH, NT = 64 * W;
  __shared__ int sdof[N], skey[N], sloc[N], qs[N];
  __shared__ double stage[CH * N];
  __shared__ double prow_s[N];
  __shared__ double red_abs[W];
  __shared__ int red_idx[W];
  const int K = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < N; i += NT) {
    sdof[i] = cell_dofs[(int64_t)K * N + i];
    skey[i] = 0x7fffffff;
    sloc[i] = 0;
  }
  __syncthreads();
  for (int i = tid; i < N; i += NT) {
    const int v = sdof[i];
    int rank = 0;
    for (int j = 0; j < N; ++j) rank += (sdof[j] < v) ? 1 : 0;
    skey[rank] = v;
    sloc[rank] = i;
  }
  double row[N];
#pragma unroll
  for (int c = 0; c < N; ++c) row[c] = 0.0;
#pragma unroll
  for (int r0 = 0; r0 < N; r0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * N; e += NT) stage[e] = 0.0;
    __syncthreads();
    {
      // NT / CH lanes per staged row, several independent loads per lane
      constexpr int LPR = NT / CH;
      const int rr = tid / LPR, sub = tid - rr * LPR;
      if (r0 + rr < N) {
        const int64_t grow = sdof[r0 + rr];
        const int64_t e0 = row_ptr[grow], e1 = row_ptr[grow + 1];
#pragma unroll 4
        for (int64_t e = e0 + sub; e < e1; e += LPR) {
          const int c = col[e];
          const double v = val[e];
          int lo = 0, hi = N;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (skey[mid] < c) lo = mid + 1; else hi = mid;
          }
          if (lo < N && skey[lo] == c) stage[rr * N + sloc[lo]] = v;
        }
      }
    }
    __syncthreads();
    if (tid >= r0 && tid < r0 + CH && tid < N) {
#pragma unroll
      for (int c = 0; c < N; ++c) row[c] = stage[(tid - r0) * N + c];
    }
  }
  const bool mine = tid < N;
  bool used = !mine;
  bool singular = false;
  int my_step = 0;
  for (int i = tid; i < N; i += NT) qs[i] = 0;
  // Column k of step k sits in register row[k mod U]: the loop runs U steps
  // with constant register indices, then rotates every row left by U.  After
  // N steps (N is a multiple of U) the rotation has come full circle.
  static_assert(N % RowCfg<N>::U == 0, "patch width must be a multiple of the unroll factor");
  constexpr int U = RowCfg<N>::U;
#pragma unroll 1
  for (int k0 = 0; k0 < N; k0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      const double my = used ? -1.0 : fabs(row[u]);
      double a = wave_max(my);
      int ai = wave_min((!used && my == a) ? tid : 0x7fffffff);
      if (W > 1) {
        if (lane == 0) { red_abs[wave] = a; red_idx[wave] = ai; }
        __syncthreads();
        a = red_abs[0];
        ai = red_idx[0];
#pragma unroll
        for (int w = 1; w < W; ++w) {
          const double oa = red_abs[w];
          const int oi = red_idx[w];
          if (oa > a || (oa == a && oi < ai)) { a = oa; ai = oi; }
        }
      }
      const int p = ai;  // uniform across the workgroup
      const bool piv = (tid == p);
      const bool bad = !(a > 0.0) || !isfinite(a) || p >= N;
      if (piv) {
        // the pivot row, scaled: (c == k ? 1 : row[c]) / pivot
        const double inv = 1.0 / row[u];
#pragma unroll
        for (int c = 0; c < N; ++c) prow_s[c] = (c == u ? 1.0 : row[c]) * inv;
        qs[k] = p;
        used = true;
        my_step = k;
      }
      __syncthreads();
      if (bad) {
        singular = true;
      } else if (mine) {
        // other rows: row - f * prow (column k: -f * prow[k]); the pivot row
        // becomes prow itself (keep = 0, f = -1)
        const double f = piv ? -1.0 : row[u];
        const double keep = piv ? 0.0 : 1.0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const double pc = prow_s[c];
          row[c] = (c == u) ? -f * pc : fma(-f, pc, keep * row[c]);
        }
      }
      __syncthreads();
    }
    double tmp[U];
#pragma unroll
    for (int c = 0; c < U; ++c) tmp[c] = row[c];
#pragma unroll
    for (int c = 0; c < N - U; ++c) row[c] = row[c + U];
#pragma unroll
    for (int c = 0; c < U; ++c) row[N - U + c] = tmp[c];
  }
  if (singular && tid == 0) atomicMin(status, K);
  using S = typename PT<P>::S;
  S* out = reinterpret_cast<S*>(inv_out) + (int64_t)K * cell_stride;
  if (mine) {
    // J_K^{-1}[my_step][q_j] = row[j]
#pragma unroll
    for (int j = 0; j < N; ++j) out[(int64_t)qs[j] * ld + my_step] = store_cvt<P>(row[j]);
  }
  for (int e = tid; e < N * (ld - N); e += NT) {
    const int c = e / (ld - N), i = N + (e - c * (ld - N));
    out[(int64_t)c * ld + i] = store_cvt<P>(0.0);
  }
}

// ---------------------------------------------------------------------------
// Wide patches (compiled for n_K = 84, 85, 105, 120, 170, 180: 2D Q2/P1disc
// dG(3), dG(4), the 3D Q2/P1disc dG(0), dG(1) patches and (Q4)^2/P3disc dG(1),
// dG(2)): beyond 64 rows one row per lane takes several wavefronts per cell that
// each hold whole rows, so the FP64 matrix is instead spread over a 512-thread
// workgroup in registers: wavefront w holds the columns [w CW, (w + 1) CW),
// lane l the rows l, l + 64, l + 128 (up to 3 x 64 rows).  Step k of the same
// implicit-pivoting Gauss-Jordan elimination: the wavefront owning column k
// finds the pivot (DPP reductions) and publishes the column through LDS (two
// buffers, so one barrier per step suffices); every wavefront reads the pivot
// row's values of its own columns from the owning lane (readlane) and updates.
// ---------------------------------------------------------------------------
template <int N> struct WideCfg {
  static constexpr int NW = 8;                     // wavefronts per cell
  static constexpr int CW = (N + NW - 1) / NW;     // columns per wavefront
  static constexpr int R = (N + 63) / 64;          // rows per lane
};

__device__ inline double readlane_f64(double v, int lane) {
  const int2 a = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(a.x, lane);
  r.y = __builtin_amdgcn_readlane(a.y, lane);
  return __builtin_bit_cast(double, r);
}

template <int P, int N>
__global__ __launch_bounds__(64 * WideCfg<N>::NW) void patch_setup_wide_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const int32_t* __restrict__ cell_dofs, void* inv_out, int32_t ld, int64_t cell_stride, int32_t* status) {
  constexpr int NW = WideCfg<N>::NW, CW = WideCfg<N>::CW, R = WideCfg<N>::R, NT = 64 * NW;
  static_assert(NW * CW >= N && R * 64 >= N && R <= 4, "wide patch layout");
  __shared__ int sdof[N], skey[N], sloc[N], qs[N], kinv[N];
  __shared__ double stage[64 * N];
  __shared__ double fcol[2][64 * R];
  __shared__ int piv_s[2];
  __shared__ double pabs_s[2];
  const int K = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < N; i += NT) {
    sdof[i] = cell_dofs[(int64_t)K * N + i];
    skey[i] = 0x7fffffff;
    sloc[i] = 0;
    qs[i] = i;      // overwritten by every successful step; keeps the output in range otherwise
    kinv[i] = i;
  }
  __syncthreads();
  for (int i = tid; i < N; i += NT) {
    const int v = sdof[i];
    int rank = 0;
    for (int j = 0; j < N; ++j) rank += (sdof[j] < v) ? 1 : 0;
    skey[rank] = v;
    sloc[rank] = i;
  }
  // gather: rows in chunks of 64 through LDS, then each lane keeps its row's columns
  double Pm[R][CW];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    __syncthreads();
    for (int e = tid; e < 64 * N; e += NT) stage[e] = 0.0;
    __syncthreads();
    {
      constexpr int LPR = NT / 64;
      const int rr = tid / LPR, sub = tid - rr * LPR;
      const int i = r * 64 + rr;
      if (i < N) {
        const int64_t grow = sdof[i];
        const int64_t e0 = row_ptr[grow], e1 = row_ptr[grow + 1];
#pragma unroll 4
        for (int64_t e = e0 + sub; e < e1; e += LPR) {
          const int c = col[e];
          const double v = val[e];
          int lo = 0, hi = N;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (skey[mid] < c) lo = mid + 1; else hi = mid;
          }
          if (lo < N && skey[lo] == c) stage[rr * N + sloc[lo]] = v;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int j = wave * CW + c;
      Pm[r][c] = (r * 64 + lane < N && j < N) ? stage[lane * N + j] : 0.0;
    }
  }
  uint32_t used = 0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r * 64 + lane >= N) used |= 1u << r;
  bool singular = false;
#pragma unroll 1
  for (int wk = 0; wk < NW; ++wk) {
#pragma unroll
    for (int ck = 0; ck < CW; ++ck) {
      const int k = wk * CW + ck;
      if (k < N) {  // uniform
        const int buf = k & 1;
        if (wave == wk) {
          double best = -1.0;
          int bi = 0x7fffffff;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const double av = fabs(Pm[r][ck]);
            if (!((used >> r) & 1u) && av > best) { best = av; bi = r * 64 + lane; }
          }
          const double m = wave_max(best);
          const int wi = wave_min((best == m && bi != 0x7fffffff) ? bi : 0x7fffffff);
#pragma unroll
          for (int r = 0; r < R; ++r) fcol[buf][r * 64 + lane] = Pm[r][ck];
          if (lane == 0) {
            piv_s[buf] = wi;
            pabs_s[buf] = m;
          }
        }
        __syncthreads();
        const int p = __builtin_amdgcn_readfirstlane(piv_s[buf]);
        const double pa = pabs_s[buf];
        const bool bad = p >= N || !(pa > 0.0) || !isfinite(pa);  // uniform
        if (bad) {
          singular = true;
        } else {
          const double inv = 1.0 / fcol[buf][p];
          const int pl = p & 63, ps = p >> 6;
          double f[R], keep[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const bool piv = (r * 64 + lane) == p;
            f[r] = piv ? -1.0 : fcol[buf][r * 64 + lane];
            keep[r] = piv ? 0.0 : 1.0;
          }
          const bool own = wave == wk;
#pragma unroll
          for (int c = 0; c < CW; ++c) {
            double pv = Pm[0][c];
#pragma unroll
            for (int r = 1; r < R; ++r) pv = (ps == r) ? Pm[r][c] : pv;
            pv = readlane_f64(pv, pl);
            const bool kc = own && (c == ck);
            const double pc = kc ? inv : pv * inv;
#pragma unroll
            for (int r = 0; r < R; ++r) Pm[r][c] = kc ? -f[r] * pc : fma(-f[r], pc, keep[r] * Pm[r][c]);
          }
          if (pl == lane) used |= 1u << ps;
          if (tid == 0) {
            qs[k] = p;
            kinv[p] = k;
          }
        }
      }
    }
  }
  if (singular && tid == 0) atomicMin(status, K);
  __syncthreads();
  using S = typename PT<P>::S;
  S* out = reinterpret_cast<S*>(inv_out) + (int64_t)K * cell_stride;
  // J_K^{-1}[kinv[i]][q_j] = W[i][j]; column-major with leading dimension ld
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r * 64 + lane;
    if (i < N) {
      const int ki = kinv[i];
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const int j = wave * CW + c;
        if (j < N) out[(int64_t)qs[j] * ld + ki] = store_cvt<P>(Pm[r][c]);
      }
    }
  }
  for (int e = tid; e < N * (ld - N); e += NT) {
    const int c = e / (ld - N), i = N + (e - c * (ld - N));
    out[(int64_t)c * ld + i] = store_cvt<P>(0.0);
  }
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// The cell's DoFs -> their local indices, an open-addressing hash table in LDS (linear probing,
// slots hold (DoF, local index), DoF -1 = empty).  1024 slots for at most 256 DoFs.
struct PatchHash {
  static constexpr int SLOTS = 1024;
  __device__ static int slot(int dof) { return (int)(((uint32_t)dof * 2654435761u) >> 22); }
  __device__ __attribute__((always_inline)) static void insert(int2* tab, int dof, int loc) {
    int h = slot(dof);
    for (;;) {  // the DoFs of a cell are distinct and fewer than the slots: ends
      if (atomicCAS(&tab[h].x, -1, dof) == -1) {
        tab[h].y = loc;
        return;
      }
      h = (h + 1) & (SLOTS - 1);
    }
  }
};

// Rows [row0, row0 + 16) of the patch into stage (row r - row0, local column).  pre[r] is the
// offset of row row0 + r among the 16 rows' CSR entries (pre[16] their number) and rbeg[i] row i's
// first CSR entry.  Each thread takes one contiguous range of the entries, issues every load of up
// to Q entries before using any, and looks the columns up in the hash table with two rounds of
// batched probes (a third, rare, probe sequence finishes the remaining lookups).
template <int NT>
__device__ __attribute__((always_inline)) inline void gather_rows(const int32_t* __restrict__ col, const double* __restrict__ val,
                                   const int64_t* rbeg, const int* pre, int row0, const int2* htab,
                                   double* stage, int ldst) {
  constexpr int Q = 6;
  int pr[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) pr[k] = __builtin_amdgcn_readfirstlane(pre[k]);  // uniform: scalar registers
  const int total = pr[16];
  const int per = (total + NT - 1) / NT;
  const int e0 = threadIdx.x * per;
  const int e1 = min(e0 + per, total);
  for (int eb = e0; eb < e1; eb += Q) {
    int cq[Q], rq[Q], hq[Q], lq[Q];
    double vq[Q];
    int64_t gq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = eb + q;
      int r = 0;
#pragma unroll
      for (int k = 1; k < 16; ++k) r += (e >= pr[k]) ? 1 : 0;
      rq[q] = r;
      gq[q] = rbeg[row0 + (e < e1 ? r : 0)] + (e - pr[r]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const bool ok = eb + q < e1;
      const int64_t g = ok ? gq[q] : 0;
      cq[q] = col[g];
      vq[q] = val[g];
      if (!ok) cq[q] = -1;
    }
    // probe rounds: lq = local index (>= 0), -1 not in the patch, -2 unresolved
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      hq[q] = PatchHash::slot(cq[q]);
      lq[q] = cq[q] < 0 ? -1 : -2;
    }
#pragma unroll
    for (int round = 0; round < 2; ++round) {
      int2 eq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) eq[q] = htab[hq[q]];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (lq[q] == -2) {
          if (eq[q].x == cq[q]) lq[q] = eq[q].y;
          else if (eq[q].x == -1) lq[q] = -1;
        }
        hq[q] = (hq[q] + 1) & (PatchHash::SLOTS - 1);
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      int h = hq[q];
      for (int probe = 0; lq[q] == -2 && probe < PatchHash::SLOTS; ++probe) {
        const int2 e = htab[h];
        if (e.x == cq[q]) lq[q] = e.y;
        else if (e.x == -1) lq[q] = -1;
        h = (h + 1) & (PatchHash::SLOTS - 1);
      }
      if (lq[q] >= 0) stage[rq[q] * ldst + lq[q]] = vq[q];
    }
  }
}

// 1 / a for the Gauss-Jordan pivots: the hardware reciprocal refined by two Newton steps
// (each doubles the correct bits), in place of the IEEE division sequence.
__device__ inline double recip_f64(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  r = fma(r, fma(-a, r, 1.0), r);
  return r;
}

// ---------------------------------------------------------------------------
// Wide patches on the FP64 matrix cores (compiled for n_K = 170, the 3D Q2/P1disc dG(1) patch):
// blocked Gauss-Jordan with implicit partial pivoting.  The patch, padded to NP = 16 T, lives in
// registers as T x T tiles of 16 x 16: tile-row wavefront w (of T) holds tile row w, and one more
// wavefront, which holds no tiles, eliminates the panels.  Columns are eliminated in panels of
// NB = 4; with panel j factored (its eliminated columns M and pivot rows q_t in LDS):
//   1. the owners of the pivot rows copy their old values, B[t][c] = W[q_t][c], to LDS and clear
//      those rows;
//   2. every tile applies the panel as one rank-NB update on the matrix cores,
//        W'[i][c] = (i pivotal in this panel ? 0 : W[i][c]) + sum_t M[i][t] B[t][c],
//      and the panel's own columns become M; the tiles then copy the columns of panel j + 2 to LDS.
// Meanwhile the panel wavefront applies the same update to panel j + 1's columns (copied to LDS
// one panel earlier, B's entries in those columns read from them) and runs panel j + 1's NB
// elimination steps on them in registers, so the tile updates never wait for a panel.
// This composes the NB single-column Gauss-Jordan steps exactly (for one step it reads
// W'[i][c] = W[i][c] - W[i][k] W[p][c] / W[p][k], W'[p][c] = W[p][c] / W[p][k]).  After all steps
// J_K^{-1}[k][q_j] = W[q_k][j], written out through LDS one 16-column block at a time so the
// stores of a column are contiguous.
// Pivot choice: the largest |a| among the rows not yet pivotal, compared on a 32-bit key (|a|'s
// exponent and 13 leading mantissa bits, then 255 - row), so one integer wavefront maximum gives
// the row as well: candidates within a relative 2^-13 count as ties and the lowest row wins (the
// first maximal row of the LU pivot sequence whenever the maximum is unique to that precision;
// the multipliers stay below 1 + 2^-13 in magnitude).
// The FP64 MFMA (16 x 16 x 4) computes D(m, n) = sum_k A(m, k) B(k, n) + C: lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16), and accumulator element v holds D(4 v + l / 16, l % 16),
// so a tile's lane l owns rows 4 v + l / 16 of column l % 16.  Tile indices are compile-time
// (the register arrays are never indexed at run time) and the branches depend on wave-uniform
// values only.
// ---------------------------------------------------------------------------
template <int N> struct MfCfg {
  static constexpr int NP = (N + 15) / 16 * 16;  // padded width
  static constexpr int T = NP / 16;              // tiles per dimension = wavefronts
  static constexpr int NT = 64 * (T + 1);       // T tile-row wavefronts and the panel wavefront
  static constexpr int NB = 4;                   // panel width (one MFMA depth)
  static constexpr int R = (NP + 63) / 64;       // panel rows per lane
  static constexpr int PW = T;                   // the wavefront that eliminates the panels
  static constexpr int PLD = NB + 1;             // LDS row length of a panel (doubles)
};

// The patch entry map of the matrix-core kernel, planned once per pattern: for every cell and every
// accumulator element of its T x T tiles (the layout above: tile (I, J), lane l, element v hold
// patch row 16 I + 4 v + l / 16, column 16 J + l % 16), the offset of that entry in the row's CSR
// entries, 0xFFFF where J stores none (and in the padding).  Stored as [cell][I][J][lane][v]
// uint16, so a lane reads its four elements of one tile as one 8-byte word and a wavefront one
// tile as 512 contiguous bytes.  One workgroup per cell builds the cell's map in LDS: the cell's
// DoFs go into the LDS hash, every wavefront walks whole CSR rows (four loads per lane in flight)
// and records the offsets of the columns it finds.
__device__ __forceinline__ int patch_map_pos(int i, int j, int T) {
  const int m = i & 15, n = j & 15;
  return (((i >> 4) * T + (j >> 4)) * 64 + n + 16 * (m & 3)) * 4 + (m >> 2);
}

template <int N>
__global__ __launch_bounds__(512) void patch_map_kernel(const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ cell_dofs, uint64_t* pmap,
                                                        int32_t* too_long) {
  constexpr int T = MfCfg<N>::T, NT = 512, ME = T * T * 256;
  __shared__ uint16_t sm[ME];
  __shared__ int2 htab[PatchHash::SLOTS];
  __shared__ int64_t rbeg[N];
  __shared__ int rlen[N];
  const int K = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int h = tid; h < PatchHash::SLOTS; h += NT) htab[h] = make_int2(-1, 0);
  for (int e = tid; e < ME / 2; e += NT) reinterpret_cast<uint32_t*>(sm)[e] = 0xFFFFFFFFu;
  __syncthreads();
  if (tid < N) {
    const int dof = cell_dofs[(int64_t)K * N + tid];
    const int64_t b0 = row_ptr[dof];
    const int64_t len = row_ptr[dof + 1] - b0;
    rbeg[tid] = b0;
    rlen[tid] = (int)(len < 65535 ? len : 65535);
    if (len > 65535) atomicOr(too_long, 1);
    PatchHash::insert(htab, dof, tid);
  }
  __syncthreads();
  for (int i = wv; i < N; i += NT / 64) {
    const int len = rlen[i];
    const int32_t* cr = col + rbeg[i];
    for (int e0 = 0; e0 < len; e0 += 256) {
      int c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + 64 * q + lane;
        c[q] = e < len ? cr[e] : -1;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (c[q] < 0) continue;
        int h = PatchHash::slot(c[q]);
        int loc = -1;
        for (int probe = 0; probe < PatchHash::SLOTS; ++probe) {  // the table has empty slots: ends
          const int2 t = htab[h];
          if (t.x == c[q]) {
            loc = t.y;
            break;
          }
          if (t.x == -1) break;
          h = (h + 1) & (PatchHash::SLOTS - 1);
        }
        if (loc >= 0) sm[patch_map_pos(i, loc, T)] = (uint16_t)(e0 + 64 * q + lane);
      }
    }
  }
  __syncthreads();
  uint64_t* out = pmap + (int64_t)K * (ME / 4);
  for (int e = tid; e < ME / 4; e += NT) out[e] = reinterpret_cast<const uint64_t*>(sm)[e];
}

template <int P, int N, bool MAP>
__global__ __launch_bounds__(MfCfg<N>::NT) void patch_setup_mfma_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const int32_t* __restrict__ cell_dofs, const uint64_t* __restrict__ pmap, void* inv_out, int32_t ld,
    int64_t cell_stride, int32_t* status) {
  using C = MfCfg<N>;
  constexpr int NP = C::NP, T = C::T, NT = C::NT, NB = C::NB, R = C::R, PW = C::PW, PLD = C::PLD;
  static_assert(R <= 4 && NP <= 256, "patch width");
  __shared__ int qs[NP], kinv[NP];
  __shared__ __align__(16) int pq[2][NB];  // the panel's pivot rows (-1: none), double-buffered
  __shared__ double stage[16 * NP];       // gather rows / output columns
  __shared__ double pan[2][NP * PLD];     // eliminated panel columns M (double-buffered)
  __shared__ double pc[2][NP * PLD];      // the next panel's columns before its last update
  __shared__ double bs[2][NB * NP];       // old pivot rows (double-buffered)
  __shared__ int2 htab[PatchHash::SLOTS]; // DoF -> local index
  __shared__ int64_t rbeg[N];             // first CSR entry of each patch row
  __shared__ int rlen[NP];                // CSR entries per patch row (0 beyond N)
  __shared__ int pre[17];
  __shared__ int bad_s;
  const int K = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // this wavefront's tile row
  const int l16 = lane & 15, l4 = lane >> 4;
  if (!MAP)
    for (int h = tid; h < PatchHash::SLOTS; h += NT) htab[h] = make_int2(-1, 0);
  for (int i = tid; i < NP; i += NT) {
    qs[i] = i < N ? i : 0;  // overwritten by every pivot; keeps the output in range otherwise
    kinv[i] = -1;
    rlen[i] = 0;
  }
  for (int e = tid; e < 2 * NB * NP; e += NT) (&bs[0][0])[e] = 0.0;
  if (tid == 0) bad_s = 0;
  f64x4_t acc[T];
#pragma unroll
  for (int J = 0; J < T; ++J) acc[J] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
  if constexpr (MAP) {
    // ---- gather through the patch entry map: every load of the tile row issued at once ----
    if (w < T) {  // the tile-row wavefronts
      int64_t rb[4];  // first CSR entry of this lane's rows 16 w + 4 v + l / 16
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + 4 * v + l4;
        rb[v] = i < N ? row_ptr[cell_dofs[(int64_t)K * N + i]] : 0;
      }
      const uint64_t* mp = pmap + ((int64_t)K * T + w) * T * 64 + lane;
      uint64_t mw[T];
#pragma unroll
      for (int J = 0; J < T; ++J) mw[J] = mp[J * 64];
#pragma unroll
      for (int J = 0; J < T; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t o = (uint32_t)(mw[J] >> (16 * v)) & 0xFFFFu;
          if (o != 0xFFFFu) acc[J][v] = val[rb[v] + o];
        }
    }
    __syncthreads();
  } else {
  __syncthreads();
  if (tid < N) {
    const int dof = cell_dofs[(int64_t)K * N + tid];
    const int64_t b0 = row_ptr[dof];
    rbeg[tid] = b0;
    rlen[tid] = (int)(row_ptr[dof + 1] - b0);
    PatchHash::insert(htab, dof, tid);
  }
  // ---- gather: 16 patch rows at a time through LDS, then into the tiles of that row block ----
  for (int I = 0; I < T; ++I) {
    __syncthreads();
    for (int e = tid; e < 16 * NP; e += NT) stage[e] = 0.0;
    if (tid < 64) {  // prefix offsets of the block's rows: one wavefront scan
      int v = lane < 16 ? rlen[16 * I + lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
      }
      if (lane < 16) pre[lane + 1] = v;
      if (lane == 0) pre[0] = 0;
    }
    __syncthreads();
    gather_rows<NT>(col, val, rbeg, pre, 16 * I, htab, stage, NP);
    __syncthreads();
    if (w == I) {
#pragma unroll
      for (int J = 0; J < T; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[J][v] = stage[(4 * v + l4) * NP + 16 * J + l16];
    }
  }
  }
  // ---- elimination, panel by panel; the panel wavefront factors panel j + 1 while the tile
  //      wavefronts finish panel j's update.  The two kinds of wavefront run separate loops with
  //      the same sequence of barriers (the panel wavefront holds no tiles, so none of its
  //      registers go to them) ----
  constexpr int NPAN = (N + NB - 1) / NB;
  using S = typename PT<P>::S;
  S* out = reinterpret_cast<S*>(inv_out) + (int64_t)K * cell_stride;
  // output: J_K^{-1}[kinv[i]][q_j] = W[i][j], one 16-column block at a time through LDS; every
  // thread copies its share of block J from stage to the output columns
  constexpr int OW = (16 * NP + NT - 1) / NT;  // output elements per thread and block
  auto copy_block = [&](int J) {
    int cq[OW];
    double xv[OW];
#pragma unroll
    for (int o = 0; o < OW; ++o) {
      const int e = tid + NT * o;
      const int jj = e / ld, r = e - jj * ld;
      const int c = 16 * J + jj;
      const bool ok = e < 16 * ld && c < N;
      cq[o] = ok ? qs[c] : -1;
      xv[o] = (ok && r < N) ? stage[jj * NP + r] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < OW; ++o) {
      const int e = tid + NT * o;
      const int jj = e / ld, r = e - jj * ld;
      if (cq[o] >= 0) out[(int64_t)cq[o] * ld + r] = store_cvt<P>(xv[o]);
    }
  };
  static_assert(NPAN >= 2 && 2 * NB <= 16, "two panels in the first tile column");
  // panels 0 and 1: their columns to LDS
  if (w < T) {
    if (l16 < 2 * NB) {
      double* dst = pc[l16 / NB];
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(16 * w + 4 * v + l4) * PLD + (l16 % NB)] = acc[0][v];
    }
  }
  __syncthreads();
  if (w == PW) {
    // ---- the panel wavefront ----
    // per row block: all ones while the lane's row may still become a pivot, and 255 - row
    uint32_t um[R], rid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      um[r] = r * 64 + lane < N ? 0xFFFFFFFFu : 0u;
      rid[r] = (uint32_t)(255 - 64 * r - lane);
    }
    bool singular = false;
    double pr[R][NB];  // the current panel's columns, the lane's rows r * 64 + lane
    bool zr[R];        // the lane's rows that became pivots in the current panel
    int pv[NB];        // the current panel's pivot rows (-1: none); uniform
    // the NB elimination steps of panel jj on pr; M and the pivot rows go to LDS
    auto factor = [&](int jj) {
      const int k0 = NB * jj;
#pragma unroll
      for (int r = 0; r < R; ++r) zr[r] = false;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const int k = k0 + t;
        // 32-bit pivot keys: |a|'s exponent and 13 leading mantissa bits, then 255 - row (0 for
        // rows already pivotal), so one integer wavefront maximum gives the row as well
        uint32_t key = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, pr[r][t]) >> 32);
          key = max(key, (((hi & 0x7FFFFF80u) << 1) | rid[r]) & um[r]);
        }
        const uint32_t mk = wave_max_u32(key);
        const int p = 255 - (int)(mk & 0xFFu);
        // uniform: a padding column of the last panel, no nonzero candidate, or a non-finite
        // largest one (the step is then a no-op on the other columns: its row of B stays zero)
        const bool skip = k >= N || (mk >> 8) == 0 || (mk >> 21) == 0x7FFu || p >= N;
        if (skip && k < N) singular = true;
        const int pl = p & 63, ps = p >> 6;
        // the pivot row's entries: every lane selects its row of block ps (uniform), lane pl's
        // are read out
        double prow[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          double x = pr[0][c];
#pragma unroll
          for (int r = 1; r < R; ++r) x = (ps == r) ? pr[r][c] : x;
          prow[c] = readlane_f64(x, pl);
        }
        const double inv = skip ? 0.0 : recip_f64(prow[t]);
#pragma unroll
        for (int c = 0; c < NB; ++c) prow[c] = (c == t) ? inv : prow[c] * inv;
        // straight-line update, the next panel column first (the next step's pivot search needs
        // only it); the pivot row becomes the scaled pivot row
        bool isp[R];
#pragma unroll
        for (int r = 0; r < R; ++r) isp[r] = !skip && r == ps && lane == pl;
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
          const int c = (t + 1 + cc) % NB;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const double u = (c == t) ? -pr[r][t] * inv : fma(-pr[r][t], prow[c], pr[r][c]);
            pr[r][c] = isp[r] ? prow[c] : u;
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          um[r] = isp[r] ? 0u : um[r];
          zr[r] = zr[r] || isp[r];
        }
        pv[t] = skip ? -1 : p;
      }
      double* pn = pan[jj & 1];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (r * 64 + lane < NP) pn[(r * 64 + lane) * PLD + c] = pr[r][c];
      if (lane == 0) {
        *reinterpret_cast<int4*>(pq[jj & 1]) = make_int4(pv[0], pv[1], pv[2], pv[3]);
#pragma unroll
        for (int t = 0; t < NB; ++t)
          if (pv[t] >= 0) {
            qs[k0 + t] = pv[t];
            kinv[pv[t]] = k0 + t;
          }
      }
    };
    // panel jj's columns from LDS buffer b (rows beyond NP read as zero)
    auto load_cols = [&](const double* b, double (&x)[R][NB]) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[r][c] = (r * 64 + lane < NP) ? b[(r * 64 + lane) * PLD + c] : 0.0;
    };
    load_cols(pc[0], pr);
    factor(0);
    for (int j = 0; j < NPAN; ++j) {
      __syncthreads();  // B: the tiles carry the updates of panels < j; panel j + 1's columns, with
                        // the updates of panels < j, are in pc
      if (j + 1 < NPAN) {
        // panel j's update applied here to panel j + 1's columns: x' = (x with the pivot rows of
        // panel j cleared) + M B, B[t][.] = the old pivot rows restricted to these columns
        const double* b = pc[(j + 1) & 1];
        double x[R][NB];
        load_cols(b, x);
        double bv[NB][NB];
#pragma unroll
        for (int t = 0; t < NB; ++t)
#pragma unroll
          for (int c = 0; c < NB; ++c) bv[t][c] = pv[t] >= 0 ? b[pv[t] * PLD + c] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            double y = zr[r] ? 0.0 : x[r][c];
#pragma unroll
            for (int t = 0; t < NB; ++t) y = fma(pr[r][t], bv[t][c], y);
            x[r][c] = y;
          }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < NB; ++c) pr[r][c] = x[r][c];
      }
      __syncthreads();  // C: the old pivot rows of panel j are in LDS
      if (j + 1 < NPAN) factor(j + 1);
    }
    if (singular && lane == 0) bad_s = 1;
    __syncthreads();
#pragma unroll 1
    for (int J = 0; J < T; ++J) {
      __syncthreads();
      __syncthreads();  // block J's columns in stage
      copy_block(J);
    }
  } else {
    // ---- the tile-row wavefronts ----
    for (int j = 0; j < NPAN; ++j) {
      __syncthreads();  // B: panel j factored; every tile carries the updates of panels < j
      const int Jp = NB * j / 16, h0 = NB * j % 16;  // panel j: columns [h0, h0 + NB) of tile column Jp
      const bool nxt2 = j + 2 < NPAN;
      const int J2 = nxt2 ? NB * (j + 2) / 16 : -1, h2 = NB * (j + 2) % 16;
      double* pn = pan[j & 1];
      double* bb = bs[j & 1];
      const int* pqj = pq[j & 1];
      // the owners of the panel's pivot rows copy their old values to LDS and clear the rows (rows
      // of steps without a pivot stay zero in B).  Each lane finds, for each of its four rows,
      // the step whose pivot it is (if any), so the accumulator element is fixed at compile time
      // and only the LDS row depends on the lane.
      {
        const int4 q4 = *reinterpret_cast<const int4*>(pqj);
        const int q0 = __builtin_amdgcn_readfirstlane(q4.x), q1 = __builtin_amdgcn_readfirstlane(q4.y);
        const int q2 = __builtin_amdgcn_readfirstlane(q4.z), q3 = __builtin_amdgcn_readfirstlane(q4.w);
        // uniform: does this wavefront hold a pivot row of the panel (-1 >> 4 is -1, never w)
        if ((q0 >> 4) == w || (q1 >> 4) == w || (q2 >> 4) == w || (q3 >> 4) == w) {
          int tv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * w + 4 * v + l4;
            tv[v] = row == q0 ? 0 : row == q1 ? 1 : row == q2 ? 2 : row == q3 ? 3 : -1;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (tv[v] >= 0) {
              double* dst = &bb[tv[v] * NP + l16];
#pragma unroll
              for (int J = 0; J < T; ++J) dst[16 * J] = acc[J][v];
            }
          // the rows are cleared by a multiplication, not under the lane branch (which would
          // make the compiler copy every accumulator)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double kv = tv[v] >= 0 ? 0.0 : 1.0;
#pragma unroll
            for (int J = 0; J < T; ++J) acc[J][v] *= kv;
          }
        }
      }
      __syncthreads();  // C
      // rank-NB update of every tile, W' = W + M B; the panel's own columns become M.  Then the
      // columns of panel j + 2 (now carrying the updates of panels <= j) go to LDS for the panel
      // wavefront, which applies panel j + 1's update to them itself.
      const bool in_pan = l16 >= h0 && l16 < h0 + NB;
      {
        const double a = pn[(16 * w + l16) * PLD + l4];
#pragma unroll
        for (int J = 0; J < T; ++J) {
          acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb[l4 * NP + 16 * J + l16], acc[J], 0, 0, 0);
          if (J == Jp && in_pan) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[J][v] = pn[(16 * w + 4 * v + l4) * PLD + (l16 - h0)];
          }
        }
        if (nxt2 && l16 >= h2 && l16 < h2 + NB) {
          double* dst = pc[(j + 2) & 1];
#pragma unroll
          for (int J = 0; J < T; ++J)
            if (J == J2) {
#pragma unroll
              for (int v = 0; v < 4; ++v) dst[(16 * w + 4 * v + l4) * PLD + (l16 - h2)] = acc[J][v];
            }
        }
        // the next panel's buffer of old pivot rows, cleared while nobody reads it
        double* bo = bs[(j + 1) & 1];
        for (int e = tid; e < NB * NP; e += 64 * T) bo[e] = 0.0;
      }
    }
    __syncthreads();  // the panel wavefront's singular flag
    // each of this lane's rows goes to stage row kinv[i] (i itself only after a failed pivot)
    int dr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + 4 * v + l4;
      const int ki = i < N ? kinv[i] : -1;
      dr[v] = i < N ? (ki >= 0 ? ki : i) : -1;
    }
#pragma unroll
    for (int J = 0; J < T; ++J) {
      __syncthreads();  // the previous block's copies are done with stage
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (dr[v] >= 0) stage[l16 * NP + dr[v]] = acc[J][v];
      __syncthreads();  // block J's columns in stage
      copy_block(J);
    }
  }
  if (tid == 0 && bad_s) atomicMin(status, K);
}

template <int P>
hipError_t setup_rows(hipStream_t s, const vk_csr& J, const vk_group& L, int32_t* status, bool* handled,
                      bool mfma, bool map) {
  *handled = true;
  switch (L.n_K) {
#define VK_ROWS_CASE(NN)                                                                                \
  case NN:                                                                                              \
    patch_setup_rows_kernel<P, NN><<<L.n_cells, 64 * RowCfg<NN>::W, 0, s>>>(                            \
        J.row_ptr, J.col, J.val, L.cell_dofs, L.inv, L.ld, L.cell_stride, status);                     \
    return hipGetLastError();
    VK_ROWS_CASE(42)
    VK_ROWS_CASE(63)
#undef VK_ROWS_CASE
#define VK_WIDE_CASE(NN)                                                                                \
  case NN:                                                                                              \
    patch_setup_wide_kernel<P, NN><<<L.n_cells, 64 * WideCfg<NN>::NW, 0, s>>>(                          \
        J.row_ptr, J.col, J.val, L.cell_dofs, L.inv, L.ld, L.cell_stride, status);                     \
    return hipGetLastError();
    VK_WIDE_CASE(84)   // measured faster than a row per lane on two wavefronts (batch setup 29.8 -> 27.7 ms)
    VK_WIDE_CASE(85)
    VK_WIDE_CASE(105)
    VK_WIDE_CASE(120)
    VK_WIDE_CASE(180)
#undef VK_WIDE_CASE
    case 170:
      if (mfma && map && L.pmap && L.pmap_ok) {
        patch_setup_mfma_kernel<P, 170, true><<<L.n_cells, MfCfg<170>::NT, 0, s>>>(
            J.row_ptr, J.col, J.val, L.cell_dofs, reinterpret_cast<const uint64_t*>(L.pmap), L.inv, L.ld,
            L.cell_stride, status);
      } else if (mfma) {
        patch_setup_mfma_kernel<P, 170, false><<<L.n_cells, MfCfg<170>::NT, 0, s>>>(
            J.row_ptr, J.col, J.val, L.cell_dofs, nullptr, L.inv, L.ld, L.cell_stride, status);
      } else {
        patch_setup_wide_kernel<P, 170><<<L.n_cells, 64 * WideCfg<170>::NW, 0, s>>>(
            J.row_ptr, J.col, J.val, L.cell_dofs, L.inv, L.ld, L.cell_stride, status);
      }
      return hipGetLastError();
    default:
      *handled = false;
      return hipSuccess;
  }
}

// ===========================================================================
// Averaged additive sweep in two passes (Eq. 3.5):
//   patch_gemv : y_K = A_K r_K for every cell (natural order), stored in Y;
//   dof_gather : z_mu = sum of the entries of Y that belong to DoF mu (the
//                E_K y_K accumulation of Eq. 3.5b, in ascending cell order),
//                d_mu += omega z_mu / p_mu.
// The DoF -> (cell, local index) lists are built at setup.
// ===========================================================================

// 16 bytes of a patch inverse, read once per sweep: loaded non-temporally, so the stream of
// inverses does not push the defect, the DoF lists and the iterate out of the caches (the 3D finest
// GEMV 0.519 -> 0.491 ms; the 176 x 32 channel's, whose inverses fit the last-level cache, gained too)
__device__ inline uint4 ld_stream(const void* p) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(uint4, __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p)));
}

template <int P>
__global__ __launch_bounds__(VK_NT) void patch_gemv_kernel(const void* __restrict__ inv_, int32_t ld,
                                                           int64_t cell_stride, int32_t n_K, int32_t n_cells,
                                                           const int32_t* __restrict__ cell_dofs,
                                                           const double* __restrict__ r,
                                                           typename PT<P>::A* __restrict__ Y, int32_t cpb) {
  using S = typename PT<P>::S;
  using A = typename PT<P>::A;
  constexpr int VW = PT<P>::VW;
  extern __shared__ __align__(16) char smem[];
  A* srk = reinterpret_cast<A*>(smem);
  A* part = srk + cpb * n_K;
  const int tpc = VK_NT / cpb;
  const int slot = threadIdx.x / tpc, t = threadIdx.x - slot * tpc;
  const int64_t K = (int64_t)xcd_block(blockIdx.x, gridDim.x) * cpb + slot;
  const bool valid = K < n_cells;
  const int vpc = ld / VW;
  const int G = tpc / vpc;
  const int g = t / vpc, v = t - g * vpc;
  const bool act = valid && g < G;
  const S* base = reinterpret_cast<const S*>(inv_) + K * cell_stride + v * VW;
  // The first PF columns of this thread's share of A_K are requested before the defect gather,
  // so the stream of inverses starts at once instead of after the gather's two dependent
  // round trips.  Columns past n_K re-read column n_K - 1 (inside the cell's inverse) and are
  // not used.
  constexpr int PF = 8;  // 16 measured slower (registers / occupancy)
  uint4 pre[PF];
  if (act) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int j = g + q * G < n_K ? g + q * G : n_K - 1;
      pre[q] = ld_stream(base + (int64_t)j * ld);
    }
  }
  for (int j = t; j < n_K; j += tpc) srk[slot * n_K + j] = valid ? (A)r[cell_dofs[K * n_K + j]] : (A)0;
  __syncthreads();
  A acc[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) acc[e] = (A)0;
  if (act) {
    const A* rk = srk + slot * n_K;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int j = g + q * G;
      if (j < n_K) {
        A a[VW];
        cvt_vec<P>(pre[q], a);
        const A rj = rk[j];
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = fma(a[e], rj, acc[e]);
      }
    }
#pragma unroll 4
    for (int j = g + PF * G; j < n_K; j += G) {
      A a[VW];
      cvt_vec<P>(ld_stream(base + (int64_t)j * ld), a);
      const A rj = rk[j];
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[e] = fma(a[e], rj, acc[e]);
    }
  }
  A* mypart = part + slot * tpc * VW;
  if (g < G) {
#pragma unroll
    for (int e = 0; e < VW; ++e) mypart[g * ld + v * VW + e] = acc[e];
  }
  __syncthreads();
  if (valid) {
    for (int i = t; i < n_K; i += tpc) {
      A y = (A)0;
      for (int gg = 0; gg < G; ++gg) y += mypart[gg * ld + i];
      Y[K * n_K + i] = y;
    }
  }
}

// d[mu] += omega / p_mu * sum of the cell products at mu; with `overwrite`, d[mu] = that term
// (the first sweep from d = 0, which then needs no zero fill; DoFs in no cell get 0)
template <typename TY>
__global__ __launch_bounds__(256) void dof_gather_kernel(int64_t n, const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ list,
                                                         const TY* __restrict__ Y, double omega, double* d,
                                                         int32_t overwrite) {
  const int64_t mu = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (mu >= n) return;
  const int32_t e0 = off[mu], e1 = off[mu + 1];
  double z = 0.0;
  for (int32_t e = e0; e < e1; ++e) z += (double)Y[list[e]];
  if (overwrite) d[mu] = e1 > e0 ? omega * z / (double)(e1 - e0) : 0.0;
  else if (e1 > e0) d[mu] += omega * z / (double)(e1 - e0);
}

// the same gather with each DoF's list at a fixed width W (entries -1 beyond its multiplicity):
// one dependent load fewer than through the offsets
template <typename TY, int W>
__global__ __launch_bounds__(256) void dof_gather_ell_kernel(int64_t n, const int32_t* __restrict__ ell,
                                                             const TY* __restrict__ Y, double omega, double* d,
                                                             int32_t overwrite) {
  const int64_t mu = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (mu >= n) return;
  int32_t e[W];
#pragma unroll
  for (int q = 0; q < W / 4; ++q) {
    const int4 v = reinterpret_cast<const int4*>(ell + mu * W)[q];
    e[4 * q] = v.x;
    e[4 * q + 1] = v.y;
    e[4 * q + 2] = v.z;
    e[4 * q + 3] = v.w;
  }
  double z = 0.0;
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (e[k] >= 0) {
      z += (double)Y[e[k]];
      ++cnt;
    }
  if (overwrite) d[mu] = cnt > 0 ? omega * z / (double)cnt : 0.0;
  else if (cnt > 0) d[mu] += omega * z / (double)cnt;
}

__global__ void dof_max_count_kernel(int64_t n, const int32_t* __restrict__ off, int32_t* max_count) {
  int32_t m = 0;
  for (int64_t mu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mu < n; mu += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = off[mu + 1] - off[mu];
    m = c > m ? c : m;
  }
  if (m > 0) atomicMax(max_count, m);
}

__global__ void dof_ell_kernel(int64_t n, int32_t w, const int32_t* __restrict__ off, const int32_t* __restrict__ list,
                               int32_t* ell) {
  for (int64_t mu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mu < n; mu += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e0 = off[mu], c = off[mu + 1] - e0;
    for (int k = 0; k < w; ++k) ell[mu * w + k] = k < c ? list[e0 + k] : -1;
  }
}

// exclusive prefix sum of count[0..n) into off[0..n] by one workgroup
__global__ __launch_bounds__(1024) void scan_kernel(int64_t n, const int32_t* __restrict__ count, int32_t* off) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b = tid * chunk, e = (b + chunk < n) ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += count[i];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int64_t v = part[i];
      part[i] = run;
      run += v;
    }
    off[n] = (int32_t)run;
  }
  __syncthreads();
  int64_t run = part[tid];
  for (int64_t i = b; i < e; ++i) {
    off[i] = (int32_t)run;
    run += count[i];
  }
}

__global__ void dof_fill_kernel(int64_t total, const int32_t* __restrict__ cell_dofs, int64_t base,
                                const int32_t* __restrict__ off, int32_t* cursor, int32_t* list) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t mu = cell_dofs[e];
    const int32_t pos = off[mu] + atomicAdd(&cursor[mu], 1);
    list[pos] = (int32_t)(base + e);
  }
}

// ascending order inside each DoF's list (deterministic accumulation order)
__global__ void dof_sort_kernel(int64_t n, const int32_t* __restrict__ off, int32_t* list) {
  for (int64_t mu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mu < n; mu += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e0 = off[mu], e1 = off[mu + 1];
    for (int32_t i = e0 + 1; i < e1; ++i) {
      const int32_t v = list[i];
      int32_t j = i - 1;
      while (j >= e0 && list[j] > v) {
        list[j + 1] = list[j];
        --j;
      }
      list[j + 1] = v;
    }
  }
}

template <int P>
hipError_t gemv_prec(hipStream_t s, const vk_group& L, int cpb, const double* r, void* Y, hipEvent_t ev0,
                     hipEvent_t ev1) {
  using A = typename PT<P>::A;
  constexpr int VW = PT<P>::VW;
  const unsigned grid = (unsigned)((L.n_cells + cpb - 1) / cpb);
  const size_t lds = (size_t)cpb * L.n_K * sizeof(A) + (size_t)VK_NT * VW * sizeof(A);
  A* y = reinterpret_cast<A*>(Y) + L.y_off;
  if (ev0 || ev1)  // the kernel's own start and end times go to the events (no extra packets)
    hipExtLaunchKernelGGL(patch_gemv_kernel<P>, dim3(grid), dim3(VK_NT), (uint32_t)lds, s, ev0, ev1, 0u,
                          (const void*)L.inv, (int32_t)L.ld, (int64_t)L.cell_stride, (int32_t)L.n_K,
                          (int32_t)L.n_cells, (const int32_t*)L.cell_dofs, r, y, (int32_t)cpb);
  else
    patch_gemv_kernel<P><<<grid, VK_NT, lds, s>>>(L.inv, L.ld, L.cell_stride, L.n_K, L.n_cells, L.cell_dofs, r, y,
                                                  cpb);
  return hipGetLastError();
}

}  // namespace

int64_t vk_patch_map_elems(int32_t n_K) { return n_K == 170 ? (int64_t)MfCfg<170>::T * MfCfg<170>::T * 256 : 0; }

hipError_t launch_patch_map(hipStream_t s, const vk_csr& J, const vk_group& G, int32_t* too_long) {
  if (!G.pmap || G.n_cells == 0 || vk_patch_map_elems(G.n_K) == 0) return hipSuccess;
  patch_map_kernel<170><<<G.n_cells, 512, 0, s>>>(J.row_ptr, J.col, G.cell_dofs,
                                                   reinterpret_cast<uint64_t*>(G.pmap), too_long);
  return hipGetLastError();
}

hipError_t launch_patch_setup_fast(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec, int32_t* status,
                                   bool* handled, bool mfma, bool map) {
  if (G.n_cells == 0) {
    *handled = true;
    return hipSuccess;
  }
  switch (prec) {
    case VK_F64: return setup_rows<VK_F64>(s, J, G, status, handled, mfma, map);
    case VK_F32: return setup_rows<VK_F32>(s, J, G, status, handled, mfma, map);
    default: return setup_rows<VK_BF16>(s, J, G, status, handled, mfma, map);
  }
}

hipError_t launch_patch_setup_blocked(hipStream_t s, const vk_csr& J, const vk_group& G, vk_prec prec,
                                      const vk_blocked_ws& ws, int32_t* status) {
  if (G.n_cells == 0) return hipSuccess;
  switch (prec) {
    case VK_F64: return setup_blocked<VK_F64>(s, J, G, ws, status);
    case VK_F32: return setup_blocked<VK_F32>(s, J, G, ws, status);
    default: return setup_blocked<VK_BF16>(s, J, G, ws, status);
  }
}

// DoF -> (cell, local) lists of a level over all its cell groups
hipError_t launch_dof_map(hipStream_t s, const vk_level& L, int32_t* count) {
  const int64_t n = L.J.n_rows;
  hipError_t e = launch_fill_i32(s, n, 0, count);
  if (e != hipSuccess) return e;
  for (const vk_group& G : L.groups)
    if ((e = launch_count_add(s, G.n_cells, G.n_K, G.cell_dofs, count)) != hipSuccess) return e;
  scan_kernel<<<1, 1024, 0, s>>>(n, count, L.dof_off);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(s, n, 0, count)) != hipSuccess) return e;
  for (const vk_group& G : L.groups) {
    const int64_t total = (int64_t)G.n_cells * G.n_K;
    if (total == 0) continue;
    dof_fill_kernel<<<capped_grid(total, 256, 4096), 256, 0, s>>>(total, G.cell_dofs, G.y_off, L.dof_off, count,
                                                                  L.dof_list);
  }
  dof_sort_kernel<<<capped_grid(n, 256, 4096), 256, 0, s>>>(n, L.dof_off, L.dof_list);
  return hipGetLastError();
}

hipError_t launch_patch_gemv(hipStream_t s, const vk_group& G, vk_prec prec, const double* r, void* Y, int cpb,
                             hipEvent_t ev0, hipEvent_t ev1) {
  if (G.n_cells == 0) return hipSuccess;
  if (cpb <= 0)
    cpb = G.cpb_override > 0 ? G.cpb_override : (G.cpb_tuned > 0 ? G.cpb_tuned : vk_default_cpb(G.n_K, G.ld, prec));
  switch (prec) {
    case VK_F64: return gemv_prec<VK_F64>(s, G, cpb, r, Y, ev0, ev1);
    case VK_F32: return gemv_prec<VK_F32>(s, G, cpb, r, Y, ev0, ev1);
    default: return gemv_prec<VK_BF16>(s, G, cpb, r, Y, ev0, ev1);
  }
}

hipError_t launch_dof_max_count(hipStream_t s, const vk_level& L, int32_t* max_count) {
  const int64_t n = L.J.n_rows;
  dof_max_count_kernel<<<capped_grid(n, 256, 1024), 256, 0, s>>>(n, L.dof_off, max_count);
  return hipGetLastError();
}

hipError_t launch_dof_ell(hipStream_t s, const vk_level& L) {
  const int64_t n = L.J.n_rows;
  dof_ell_kernel<<<capped_grid(n, 256, 4096), 256, 0, s>>>(n, L.ell_w, L.dof_off, L.dof_list, L.dof_ell);
  return hipGetLastError();
}

hipError_t launch_dof_gather(hipStream_t s, const vk_level& L, vk_prec prec, const void* Y, double omega,
                             double* d, bool overwrite, bool fixed_width) {
  const int64_t n = L.J.n_rows;
  const unsigned g = (unsigned)((n + 255) / 256);
  const int32_t ow = overwrite ? 1 : 0;
  if (fixed_width && (L.ell_w == 4 || L.ell_w == 8)) {
    const float* yf = reinterpret_cast<const float*>(Y);
    const double* yd = reinterpret_cast<const double*>(Y);
    if (prec == VK_F64) {
      if (L.ell_w == 4) dof_gather_ell_kernel<double, 4><<<g, 256, 0, s>>>(n, L.dof_ell, yd, omega, d, ow);
      else dof_gather_ell_kernel<double, 8><<<g, 256, 0, s>>>(n, L.dof_ell, yd, omega, d, ow);
    } else {
      if (L.ell_w == 4) dof_gather_ell_kernel<float, 4><<<g, 256, 0, s>>>(n, L.dof_ell, yf, omega, d, ow);
      else dof_gather_ell_kernel<float, 8><<<g, 256, 0, s>>>(n, L.dof_ell, yf, omega, d, ow);
    }
    return hipGetLastError();
  }
  if (prec == VK_F64)
    dof_gather_kernel<double><<<g, 256, 0, s>>>(n, L.dof_off, L.dof_list, reinterpret_cast<const double*>(Y), omega, d,
                                                 ow);
  else
    dof_gather_kernel<float><<<g, 256, 0, s>>>(n, L.dof_off, L.dof_list, reinterpret_cast<const float*>(Y), omega, d,
                                                ow);
  return hipGetLastError();
}
