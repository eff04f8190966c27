// Coarsest-level direct solve (Sec. 3: a direct solver for J_0 d_0 = b_0 on T_0).
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

// one wavefront per row
__global__ void csr_to_dense_kernel(int64_t n, const int64_t* __restrict__ row_ptr,
                                    const int32_t* __restrict__ col, const double* __restrict__ val, double* M) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  for (int64_t e = row_ptr[i] + lane; e < row_ptr[i + 1]; e += 64) M[i * n + col[e]] = val[e];
}

constexpr int CT = 256;  // panel kernel threads

template <int R, int NB>
__global__ __launch_bounds__(CT) void coarse_panel_kernel(int64_t n, int64_t k0, int nb,
                                                          const double* __restrict__ Min, double* __restrict__ Mout,
                                                          int32_t* __restrict__ q_g, int32_t* __restrict__ used_g,
                                                          int32_t* status) {
  __shared__ double w_abs[CT / 64];
  __shared__ int w_idx[CT / 64];
  __shared__ double prow[NB];
  __shared__ int s_q[NB];
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

// Rank-NB update of the columns outside the panel; tiles of 32 rows x 64 columns.
template <int NB>
__global__ __launch_bounds__(256) void coarse_update_kernel(int64_t n, int64_t k0, int nb,
                                                            const double* __restrict__ Min, double* Mout,
                                                            const int32_t* __restrict__ q_g) {
  __shared__ double Rt[NB][64];
  __shared__ double Xt[32][NB + 1];
  __shared__ int qs[NB];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 64;
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

// y[k] = sum_j W[q_k][j] x[q_j], one wavefront per output entry.
__global__ __launch_bounds__(256) void coarse_apply_kernel(int64_t n, const double* __restrict__ W,
                                                           const int32_t* __restrict__ q,
                                                           const double* __restrict__ x, double* __restrict__ y) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  const double* w = W + (int64_t)q[k] * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s = fma(w[j], x[q[j]], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[k] = s;
}

// out[k][q_j] = W[q_k][j]: the inverse in natural order
__global__ void coarse_export_kernel(int64_t n, const double* __restrict__ W, const int32_t* __restrict__ q,
                                     double* out) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, j = e - k * n;
    out[k * n + q[j]] = W[(int64_t)q[k] * n + j];
  }
}

template <int R, int NB>
hipError_t run_blocked(hipStream_t s, int64_t n, double** a, double** b, int32_t* q, int32_t* used,
                       int32_t* status) {
  const dim3 ugrid((unsigned)((n + 63) / 64), (unsigned)((n + 31) / 32));
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
    coarse_panel_kernel<R, NB><<<1, CT, 0, s>>>(n, k0, nb, *a, *b, q, used, status);
    coarse_update_kernel<NB><<<ugrid, 256, 0, s>>>(n, k0, nb, *a, *b, q);
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

hipError_t launch_coarse_invert(hipStream_t s, const vk_csr& J0, double* buf0, double* buf1, int32_t* perm,
                                int32_t* status, double** result) {
  const int64_t n = J0.n_rows;
  hipError_t e = launch_fill(s, n * n, 0.0, buf0);
  if (e != hipSuccess) return e;
  csr_to_dense_kernel<<<(unsigned)((n * 64 + 255) / 256), 256, 0, s>>>(n, J0.row_ptr, J0.col, J0.val, buf0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int32_t* q = perm;
  int32_t* used = perm + n;
  if ((e = launch_fill_i32(s, n, 0, used)) != hipSuccess) return e;
  double* a = buf0;
  double* b = buf1;
  // R rows x NB panel columns per thread: R * NB <= 64 doubles
  const int64_t R = (n + CT - 1) / CT;
  if (R <= 4) e = run_blocked<4, 16>(s, n, &a, &b, q, used, status);
  else if (R <= 8) e = run_blocked<8, 8>(s, n, &a, &b, q, used, status);
  else e = run_blocked<16, 4>(s, n, &a, &b, q, used, status);
  *result = a;
  return e;
}

hipError_t launch_coarse_apply(hipStream_t s, int64_t n, const double* W, const int32_t* q, const double* x,
                               double* y) {
  coarse_apply_kernel<<<(unsigned)((n * 64 + 255) / 256), 256, 0, s>>>(n, W, q, x, y);
  return hipGetLastError();
}

hipError_t launch_coarse_export(hipStream_t s, int64_t n, const double* W, const int32_t* q, double* out) {
  int64_t g = (n * n + 255) / 256;
  if (g > 8192) g = 8192;
  coarse_export_kernel<<<(unsigned)g, 256, 0, s>>>(n, W, q, out);
  return hipGetLastError();
}
