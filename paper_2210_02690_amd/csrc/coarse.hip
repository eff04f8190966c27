// Directly solved diagonal blocks: the coarsest level (Sec. 3: a direct solver
// for J_0 d_0 = b_0 on T_0), and in a batch of independent systems every
// system's coarsest level.  All blocks of a level are processed together.
//
// Setup inverts the dense FP64 J_0 by blocked Gauss-Jordan elimination with
// implicit partial pivoting: the pivot of column k is the not-yet-used row
// q_k with the largest |value| (the first such row on ties); rows never move.
// For each panel of NB columns:
//   panel kernel  (one 256-thread workgroup, the panel rows in registers):
//                 the NB elimination steps restricted to the panel columns;
//   update kernel (whole GPU): the same transformation on every other
//                 column, as the rank-NB update
//                   out[i, c] = (i a pivot row of the panel ? 0 : in[i, c])
//                               + sum_j X[i, j] in[q_j, c],
//                 X the eliminated panel.
// Two buffers alternate so no workgroup reads what another writes.  The
// stored matrix W then satisfies J_0^{-1}[k][q_j] = W[q_k][j], so the coarse
// solve is y[k] = sum_j W[q_k][j] b[q_j].
#include <climits>

#include "vk_internal.h"

namespace {

constexpr int CT = 256;  // panel kernel threads

__device__ inline int block_of(const int64_t* __restrict__ rows, int nb, int64_t r) {
  int lo = 0, hi = nb;  // last block with rows[b] <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rows[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

// dense block b from the CSR rows of its rows; a coupling outside the block
// flags status[1] (the blocks must be diagonal blocks of J)
__global__ void block_to_dense_kernel(int n_blocks, const int64_t* __restrict__ rows,
                                      const int64_t* __restrict__ woff, const int64_t* __restrict__ row_ptr,
                                      const int32_t* __restrict__ col, const double* __restrict__ val, double* M,
                                      int32_t* status) {
  const int64_t total = rows[n_blocks];
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= total - rows[0]) return;
  const int64_t r = rows[0] + t;
  const int b = block_of(rows, n_blocks, r);
  const int64_t r0 = rows[b], nbk = rows[b + 1] - r0;
  double* W = M + woff[b];
  for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64) {
    const int64_t c = col[e];
    if (c < r0 || c >= r0 + nbk) {
      atomicOr(&status[1], 1);
      continue;
    }
    W[(r - r0) * nbk + (c - r0)] = val[e];
  }
}

template <int R, int NB>
__global__ __launch_bounds__(CT) void block_panel_kernel(const int64_t* __restrict__ rows,
                                                         const int64_t* __restrict__ woff, int64_t k0,
                                                         const double* __restrict__ Min_, double* __restrict__ Mout_,
                                                         int32_t* __restrict__ q_all, int32_t* __restrict__ used_all,
                                                         int32_t* status) {
  __shared__ double w_abs[CT / 64];
  __shared__ int w_idx[CT / 64];
  __shared__ double prow[NB];
  __shared__ int s_q[NB];
  const int bk = blockIdx.x;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < NB ? (int)left : NB);
  if (nb == 0) return;  // uniform for the workgroup
  const double* Min = Min_ + woff[bk];
  double* Mout = Mout_ + woff[bk];
  int32_t* q_g = q_all + r0;
  int32_t* used_g = used_all + r0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // P[r][.]: panel row tid + r * CT; the column loop is unrolled completely
  double P[R][NB];
  uint32_t used = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * CT;
    const bool ok = i < n;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[r][c] = (ok && c < nb) ? Min[i * n + k0 + c] : 0.0;
    if (!ok || used_g[i]) used |= 1u << r;
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {  // uniform
      double ba = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double av = fabs(P[r][j]);
        if (!((used >> r) & 1u) && av > ba) { ba = av; bi = tid + r * CT; }
      }
      const double m = wave_max(ba);
      const int wi = wave_min((ba == m && bi != INT_MAX) ? bi : INT_MAX);
      if (lane == 0) { w_abs[wave] = m; w_idx[wave] = wi; }
      __syncthreads();
      double pm = w_abs[0];
      int p = w_idx[0];
#pragma unroll
      for (int w = 1; w < CT / 64; ++w) {
        const double om = w_abs[w];
        const int oi = w_idx[w];
        if (om > pm || (om == pm && oi < p)) { pm = om; p = oi; }
      }
      const bool bad = p == INT_MAX || !(pm > 0.0) || !isfinite(pm);
      const int owner = bad ? -1 : p % CT, slot = bad ? -1 : p / CT;
      if (tid == owner) {
        double v[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          v[c] = P[0][c];
#pragma unroll
          for (int r = 1; r < R; ++r) v[c] = (slot == r) ? P[r][c] : v[c];
        }
        const double inv = 1.0 / v[j];
#pragma unroll
        for (int c = 0; c < NB; ++c) prow[c] = (c == j ? 1.0 : v[c]) * inv;
        used |= 1u << slot;
        s_q[j] = p;
      }
      if (bad && tid == 0) {
        atomicMin(&status[0], -1);  // failure path only
        s_q[j] = 0;
      }
      __syncthreads();
      if (!bad) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool piv = (tid == owner) && (r == slot);
          const double f = piv ? -1.0 : P[r][j];
          const double keep = piv ? 0.0 : 1.0;
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            const double pc = prow[c];
            P[r][c] = (c == j) ? -f * pc : fma(-f, pc, keep * P[r][c]);
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * CT;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) Mout[i * n + k0 + c] = P[r][c];
      used_g[i] = (used >> r) & 1u;
    }
  }
  if (tid < nb) q_g[k0 + tid] = s_q[tid];
}

// Rank-NB update of the columns outside the panel of every block (blockIdx.z);
// tiles of 32 rows x 64 columns.  A block whose elimination is complete is
// copied unchanged, so all blocks end in the same buffer.
template <int NB>
__global__ __launch_bounds__(256) void block_update_kernel(const int64_t* __restrict__ rows,
                                                           const int64_t* __restrict__ woff, int64_t k0,
                                                           const double* __restrict__ Min_, double* Mout_,
                                                           const int32_t* __restrict__ q_all) {
  __shared__ double Rt[NB][64];
  __shared__ double Xt[32][NB + 1];
  __shared__ int qs[NB];
  const int bk = blockIdx.z;
  const int64_t rb0 = rows[bk], n = rows[bk + 1] - rb0;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 64;
  if (r0 >= n || c0 >= n) return;  // uniform for the workgroup
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < NB ? (int)left : NB);
  const double* Min = Min_ + woff[bk];
  double* Mout = Mout_ + woff[bk];
  const int32_t* q_g = q_all + rb0;
  const int tid = threadIdx.x;
  if (tid < NB) qs[tid] = tid < nb ? q_g[k0 + tid] : -1;
  __syncthreads();
  for (int e = tid; e < NB * 64; e += 256) {
    const int j = e >> 6, cc = e & 63;
    const int64_t c = c0 + cc;
    Rt[j][cc] = (j < nb && c < n) ? Min[(int64_t)qs[j] * n + c] : 0.0;
  }
  for (int e = tid; e < 32 * NB; e += 256) {
    const int rr = e / NB, j = e - rr * NB;
    const int64_t i = r0 + rr;
    Xt[rr][j] = (i < n && j < nb) ? Mout[i * n + k0 + j] : 0.0;
  }
  const int tx = tid & 63, ty = tid >> 6;
  const int64_t c = c0 + tx;
  const bool col_ok = c < n && !(c >= k0 && c < k0 + nb);
  double base[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t i = r0 + ty + 4 * s;
    base[s] = (col_ok && i < n) ? Min[i * n + c] : 0.0;  // issued before the barrier
  }
  __syncthreads();
  if (!col_ok) return;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int rr = ty + 4 * s;
    const int64_t i = r0 + rr;
    if (i < n) {
      bool pivot_row = false;
#pragma unroll
      for (int j = 0; j < NB; ++j) pivot_row |= (qs[j] == i);
      double acc = pivot_row ? 0.0 : base[s];
#pragma unroll
      for (int j = 0; j < NB; ++j) acc = fma(Xt[rr][j], Rt[j][tx], acc);
      Mout[i * n + c] = acc;
    }
  }
}

// y[r0 + k] = sum_j W_b[q_k][j] x[r0 + q_j] for every row of every block,
// one wavefront per row
__global__ __launch_bounds__(256) void block_apply_kernel(int n_blocks, const int64_t* __restrict__ rows,
                                                          const int64_t* __restrict__ woff,
                                                          const double* __restrict__ W_,
                                                          const int32_t* __restrict__ q_all,
                                                          const double* __restrict__ x, double* __restrict__ y) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= rows[n_blocks] - rows[0]) return;
  const int64_t r = rows[0] + t;
  const int b = block_of(rows, n_blocks, r);
  const int64_t r0 = rows[b], n = rows[b + 1] - r0, k = r - r0;
  const int32_t* q = q_all + r0;
  const double* w = W_ + woff[b] + (int64_t)q[k] * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s = fma(w[j], x[r0 + q[j]], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[r] = s;
}

// out[k][q_j] = W_b[q_k][j]: block b's inverse in natural order
__global__ void block_export_kernel(int64_t n, const double* __restrict__ W, const int32_t* __restrict__ q,
                                    double* out) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, j = e - k * n;
    out[k * n + q[j]] = W[(int64_t)q[k] * n + j];
  }
}

template <int R, int NB>
hipError_t run_blocked(hipStream_t s, const vk_level& L, double** a, double** b, int32_t* status) {
  const int nbk = (int)L.cb_rows.size() - 1;
  const int64_t n = L.cb_max;
  const dim3 ugrid((unsigned)((n + 63) / 64), (unsigned)((n + 31) / 32), (unsigned)nbk);
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    block_panel_kernel<R, NB><<<nbk, CT, 0, s>>>(L.d_cb_rows, L.d_cb_woff, k0, *a, *b, L.cb_q, L.cb_used, status);
    block_update_kernel<NB><<<ugrid, 256, 0, s>>>(L.d_cb_rows, L.d_cb_woff, k0, *a, *b, L.cb_q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* t = *a;
    *a = *b;
    *b = t;
  }
  return hipSuccess;
}

}  // namespace

int64_t vk_coarse_max_n() { return 4096; }

hipError_t launch_block_invert(hipStream_t s, const vk_level& L, int32_t* status, double** result) {
  const int nbk = (int)L.cb_rows.size() - 1;
  *result = L.cb_a;
  if (nbk <= 0) return hipSuccess;
  const int64_t rows_total = L.cb_rows[nbk] - L.cb_rows[0];
  hipError_t e = launch_fill(s, L.cb_sq, 0.0, L.cb_a);
  if (e != hipSuccess) return e;
  block_to_dense_kernel<<<(unsigned)((rows_total * 64 + 255) / 256), 256, 0, s>>>(
      nbk, L.d_cb_rows, L.d_cb_woff, L.J.row_ptr, L.J.col, L.J.val, L.cb_a, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(s, L.J.n_rows, 0, L.cb_used)) != hipSuccess) return e;
  double* a = L.cb_a;
  double* b = L.cb_b;
  // R rows x NB panel columns per thread: R * NB <= 64 doubles
  const int64_t R = (L.cb_max + CT - 1) / CT;
  if (R <= 4) e = run_blocked<4, 16>(s, L, &a, &b, status);
  else if (R <= 8) e = run_blocked<8, 8>(s, L, &a, &b, status);
  else e = run_blocked<16, 4>(s, L, &a, &b, status);
  *result = a;
  return e;
}

hipError_t launch_block_apply(hipStream_t s, const vk_level& L, const double* x, double* y) {
  const int nbk = (int)L.cb_rows.size() - 1;
  if (nbk <= 0) return hipSuccess;
  const int64_t rows_total = L.cb_rows[nbk] - L.cb_rows[0];
  block_apply_kernel<<<(unsigned)((rows_total * 64 + 255) / 256), 256, 0, s>>>(nbk, L.d_cb_rows, L.d_cb_woff,
                                                                              L.cb_W, L.cb_q, x, y);
  return hipGetLastError();
}

hipError_t launch_block_export(hipStream_t s, const vk_level& L, int32_t block, double* out) {
  const int64_t n = L.cb_rows[block + 1] - L.cb_rows[block];
  int64_t woff = 0;
  for (int b = 0; b < block; ++b) {
    const int64_t nb = L.cb_rows[b + 1] - L.cb_rows[b];
    woff += nb * nb;
  }
  int64_t g = (n * n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  block_export_kernel<<<(unsigned)g, 256, 0, s>>>(n, L.cb_W + woff, L.cb_q + L.cb_rows[block], out);
  return hipGetLastError();
}
