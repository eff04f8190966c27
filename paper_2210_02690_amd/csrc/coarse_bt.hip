// Direct solve of a wide directly solved block through its block-tridiagonal structure (Sec. 3: a
// direct solver for J_0 d_0 = b_0 on T_0; the paper names no method).
//
// Breadth-first level sets of the block's symmetrised sparsity graph, started from a
// pseudo-peripheral vertex, couple only to themselves and to the neighbouring sets.  Consecutive
// level sets are grouped into blocks of at least VK_BT_MIN_BLOCK unknowns; in that order the block is
// block tridiagonal, with diagonal blocks D_i and couplings U_i (block i to i + 1) and L_i (block i
// to i - 1).  The factorisation is block Gaussian elimination in that order:
//   S_0 = D_0,   X_i = S_i^{-1} U_i,   S_{i+1} = D_{i+1} - L_{i+1} X_i,
// each S_i inverted densely by the blocked Gauss-Jordan kernels (implicit partial pivoting inside
// the block); the solve runs forward, y_0 = S_0^{-1} b_0, y_i = S_i^{-1} (b_i - L_i y_{i-1}), and
// back, x_{nb-1} = y_{nb-1}, x_i = y_i - X_i x_{i+1}.  It computes J_0^{-1} b up to rounding like the
// dense inverse, with 2 sum s_i^3 + 4 sum s_i^2 s_{i+1} flop instead of 2 n^3, and a chain of nb
// small inversions instead of one wide one.  A block S_i with no nonzero pivot is reported like a
// singular dense block.
//
// Layout (carved from the level's dense-inverse buffer, which this path does not otherwise use):
// D_i and U_i column-major (the Gauss-Jordan input, overwritten, and the GEMM operand), S_i^{-1},
// L_i and X_i row-major (the solve reads them a row per wavefront).
#include <algorithm>
#include <climits>
#include <vector>

#include "vk_internal.h"

namespace {

__device__ inline int find_block(const int64_t* __restrict__ off, int nb, int64_t r) {
  int lo = 0, hi = nb;  // last block with off[b] <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

// One wavefront per row of the new order: the row's CSR entries go to D, U or L of its block.
// An entry coupling blocks more than one apart flags status (the plan makes that impossible).
__global__ __launch_bounds__(256) void bt_gather_kernel(int64_t n, int64_t r0, const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col, const double* __restrict__ val,
                                                        const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ iperm, int nb,
                                                        const int64_t* __restrict__ off, const int64_t* __restrict__ oD,
                                                        const int64_t* __restrict__ oU, const int64_t* __restrict__ oL,
                                                        double* D, double* U, double* Lc, int32_t* status) {
  const int64_t rn = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (rn >= n) return;
  const int b = find_block(off, nb, rn);
  const int64_t ri = rn - off[b], sb = off[b + 1] - off[b];
  const int64_t ro = r0 + perm[rn];
  for (int64_t e = row_ptr[ro] + lane; e < row_ptr[ro + 1]; e += 64) {
    const int64_t co = (int64_t)col[e] - r0;
    if (co < 0 || co >= n) {
      atomicOr(&status[1], 1);
      continue;
    }
    const int64_t cn = iperm[co];
    const int bc = find_block(off, nb, cn);
    const int64_t cj = cn - off[bc];
    if (bc == b) D[oD[b] + cj * sb + ri] = val[e];
    else if (bc == b + 1) U[oU[b] + cj * sb + ri] = val[e];
    else if (bc == b - 1) Lc[oL[b] + ri * (off[b] - off[b - 1]) + cj] = val[e];
    else atomicOr(&status[1], 2);
  }
}

// C += alpha A B for C (m x n, ldc), A (m x k, lda), B (k x n, ldb), each row-major (the *_ROW
// flag) or column-major.  64 x 64 tiles of C per 256-thread workgroup, 16-step chunks of k through
// LDS; thread (tx, ty) owns rows ty + 16 i and columns tx + 16 j (i, j < 4).
template <bool A_ROW, bool B_ROW, bool C_ROW>
__global__ __launch_bounds__(256) void bt_gemm_kernel(int64_t m, int64_t n, int64_t k, double alpha,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb, double* C,
                                                      int64_t ldc) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int row, kk;
      if (A_ROW) {
        kk = e & 15;
        row = e >> 4;
      } else {
        row = e & 63;
        kk = e >> 6;
      }
      const int64_t gr = m0 + row, gk = k0 + kk;
      const bool ok = gr < m && gk < k;
      As[kk][row] = ok ? (A_ROW ? A[gr * lda + gk] : A[gk * lda + gr]) : 0.0;
      int bk, bc;
      if (B_ROW) {
        bc = e & 63;
        bk = e >> 6;
      } else {
        bk = e & 15;
        bc = e >> 4;
      }
      const int64_t gc = n0 + bc, gk2 = k0 + bk;
      Bs[bk][bc] = (gc < n && gk2 < k) ? (B_ROW ? B[gk2 * ldb + gc] : B[gc * ldb + gk2]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = n0 + tx + 16 * j;
    if (c >= n) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = m0 + ty + 16 * i;
      if (r < m) (C_ROW ? C[r * ldc + c] : C[c * ldc + r]) += alpha * acc[i][j];
    }
  }
}

// y[r] = (base ? base[r] : 0) + alpha sum_j A[r lda + j] x[j], A (m x k) row-major: one wavefront
// per row, two loads in flight per lane.
__global__ __launch_bounds__(256) void bt_gemv_kernel(int64_t m, int64_t k, double alpha, const double* __restrict__ A,
                                                      int64_t lda, const double* __restrict__ x,
                                                      const double* __restrict__ base, double* __restrict__ y) {
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= m) return;
  const double* a = A + r * lda;
  double s0 = 0.0, s1 = 0.0;
  int64_t j = lane;
  for (; j + 64 < k; j += 128) {
    s0 = fma(a[j], x[j], s0);
    s1 = fma(a[j + 64], x[j + 64], s1);
  }
  if (j < k) s0 = fma(a[j], x[j], s0);
  double s = s0 + s1;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[r] = (base ? base[r] : 0.0) + alpha * s;
}

// gather (out[i] = in[idx[i]]) or scatter (out[idx[i]] = in[i])
__global__ void bt_permute_kernel(int64_t n, const int32_t* __restrict__ idx, const double* __restrict__ in,
                                  double* __restrict__ out, bool scatter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (scatter) out[idx[i]] = in[i];
  else out[i] = in[idx[i]];
}

unsigned grid_of(int64_t threads) { return (unsigned)((threads + 255) / 256); }

template <bool A_ROW, bool B_ROW, bool C_ROW>
hipError_t gemm(hipStream_t s, int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                const double* B, int64_t ldb, double* C, int64_t ldc) {
  bt_gemm_kernel<A_ROW, B_ROW, C_ROW><<<dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64)), 256, 0, s>>>(
      m, n, k, alpha, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t gemv(hipStream_t s, int64_t m, int64_t k, double alpha, const double* A, const double* x,
                const double* base, double* y) {
  bt_gemv_kernel<<<grid_of(m * 64), 256, 0, s>>>(m, k, alpha, A, k, x, base, y);
  return hipGetLastError();
}

// breadth-first levels from `start` over the symmetric adjacency (adj_ptr, adj); returns the
// number of levels, -1 if some vertex is unreached
int bfs_levels(int64_t n, const std::vector<int64_t>& ap, const std::vector<int32_t>& aj, int32_t start,
               std::vector<int32_t>& level, int32_t* last) {
  level.assign(n, -1);
  std::vector<int32_t> frontier{start}, next;
  level[start] = 0;
  int nl = 0;
  int64_t seen = 1;
  while (!frontier.empty()) {
    ++nl;
    next.clear();
    for (int32_t v : frontier)
      for (int64_t e = ap[v]; e < ap[v + 1]; ++e) {
        const int32_t u = aj[e];
        if (level[u] < 0) {
          level[u] = nl;
          next.push_back(u);
        }
      }
    if (next.empty()) {
      // lowest-index vertex of the last level: deterministic
      *last = *std::min_element(frontier.begin(), frontier.end());
    }
    seen += (int64_t)next.size();
    frontier.swap(next);
  }
  return seen == n ? nl : -1;
}

}  // namespace

bool vk_bt_plan(vk_level& L) {
  vk_bt& T = L.bt;
  T = vk_bt();
  T.planned = true;
  if (L.cb_rows.size() != 2) return false;
  const int64_t r0 = L.cb_rows[0], n = L.cb_rows[1] - L.cb_rows[0];
  if (n <= VK_TOURNEY_MIN_N) return false;
  // the block's pattern on the host
  std::vector<int64_t> rp(n + 1);
  if (hipMemcpy(rp.data(), L.J.row_ptr + r0, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const int64_t e0 = rp[0], nnz = rp[n] - e0;
  std::vector<int32_t> cj(nnz);
  if (nnz > 0 &&
      hipMemcpy(cj.data(), L.J.col + e0, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  // symmetric adjacency (pattern of A + A^T, no self loops)
  std::vector<int64_t> deg(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = rp[r] - e0; e < rp[r + 1] - e0; ++e) {
      const int64_t c = (int64_t)cj[e] - r0;
      if (c < 0 || c >= n) return false;  // a coupling outside the block: the dense path reports it
      if (c != r) {
        ++deg[r + 1];
        ++deg[c + 1];
      }
    }
  for (int64_t r = 0; r < n; ++r) deg[r + 1] += deg[r];
  std::vector<int32_t> adj(deg[n]);
  std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = rp[r] - e0; e < rp[r + 1] - e0; ++e) {
      const int64_t c = (int64_t)cj[e] - r0;
      if (c != r) {
        adj[fill[r]++] = (int32_t)c;
        adj[fill[c]++] = (int32_t)r;
      }
    }
  // pseudo-peripheral start: the last level's vertex of a search from vertex 0, then the levels
  // of a search from there
  std::vector<int32_t> level;
  int32_t far = 0;
  if (bfs_levels(n, deg, adj, 0, level, &far) < 0) return false;
  const int nl = bfs_levels(n, deg, adj, far, level, &far);
  if (nl < 0) return false;
  std::vector<int64_t> lsize(nl, 0);
  for (int64_t v = 0; v < n; ++v) ++lsize[level[v]];
  // consecutive levels into blocks of at least VK_BT_MIN_BLOCK unknowns (the remainder joins the last)
  std::vector<int32_t> lblock(nl);
  std::vector<int64_t> bsize;
  int64_t cur = 0;
  for (int l = 0; l < nl; ++l) {
    if (bsize.empty() || cur >= VK_BT_MIN_BLOCK) {
      bsize.push_back(0);
      cur = 0;
    }
    lblock[l] = (int32_t)bsize.size() - 1;
    bsize.back() += lsize[l];
    cur += lsize[l];
  }
  if (bsize.size() > 1 && bsize.back() < VK_BT_MIN_BLOCK) {
    const int64_t tail = bsize.back();
    bsize.pop_back();
    bsize.back() += tail;
    for (int l = 0; l < nl; ++l)
      if (lblock[l] == (int32_t)bsize.size()) lblock[l] = (int32_t)bsize.size() - 1;
  }
  const int nb = (int)bsize.size();
  int64_t smax = 0;
  for (int64_t sz : bsize) smax = std::max(smax, sz);
  if (nb < 3 || smax > VK_BT_MAX_BLOCK) return false;
  // the new order: by block, then by row
  T.off.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) T.off[b + 1] = T.off[b] + bsize[b];
  std::vector<int64_t> pos(T.off.begin(), T.off.end() - 1);
  std::vector<int32_t> perm(n), iperm(n);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t p = pos[lblock[level[v]]]++;
    perm[p] = (int32_t)v;
    iperm[v] = (int32_t)p;
  }
  // element offsets and the carve of the dense-inverse buffer (doubles)
  T.nb = nb;
  T.smax = smax;
  T.oD.assign(nb, 0);
  T.oU.assign(nb, 0);
  T.oL.assign(nb, 0);
  int64_t sD = 0, sU = 0, sL = 0;
  for (int b = 0; b < nb; ++b) {
    T.oD[b] = sD;
    sD += bsize[b] * bsize[b];
    T.oU[b] = sU;
    if (b + 1 < nb) sU += bsize[b] * bsize[b + 1];
    T.oL[b] = sL;
    if (b > 0) sL += bsize[b] * bsize[b - 1];
  }
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  const int64_t ints = up((3 * n + 1) / 2 + 1);                           // perm, iperm (as doubles)
  const int64_t idx = up(4 * (nb + 1) + 3 * nb + 2 * nb);                 // off, oD, oU, oL, rows
  const int64_t need = 2 * up(sD) + up(sU) * 2 + up(sL) + 3 * up(n) + up(smax) + ints + idx;
  if (need > L.cb_sq) return false;
  double* p = L.cb_a;
  T.D = p;    p += up(sD);
  T.Dinv = p; p += up(sD);
  T.U = p;    p += up(sU);
  T.X = p;    p += up(sU);
  T.Lc = p;   p += up(sL);
  T.bp = p;   p += up(n);
  T.y = p;    p += up(n);
  T.xp = p;   p += up(n);
  T.w = p;    p += up(smax);
  T.perm = reinterpret_cast<int32_t*>(p);
  T.iperm = T.perm + n;
  p += ints;
  int64_t* q = reinterpret_cast<int64_t*>(p);
  T.d_off = q;        q += nb + 1;
  T.d_oD = q;         q += nb;
  T.d_oU = q;         q += nb;
  T.d_oL = q;         q += nb;
  T.d_rows = q;       q += 2 * nb;
  std::vector<int64_t> rows(2 * nb);
  for (int b = 0; b < nb; ++b) {
    rows[2 * b] = 0;
    rows[2 * b + 1] = bsize[b];
  }
  if (hipMemcpy(T.perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.iperm, iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_off, T.off.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oD, T.oD.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oU, T.oU.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oL, T.oL.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_rows, rows.data(), sizeof(int64_t) * 2 * nb, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  T.flops = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double s = (double)bsize[b];
    T.flops += 2.0 * s * s * s;
    if (b + 1 < nb) T.flops += 4.0 * s * s * (double)bsize[b + 1];
  }
  T.active = true;
  return true;
}

hipError_t launch_bt_factor(hipStream_t s, const vk_level& L, int32_t* status) {
  const vk_bt& T = L.bt;
  const int64_t n = T.off[T.nb], r0 = L.cb_rows[0];
  hipError_t e;
  const int64_t nD = T.oD[T.nb - 1] + (T.off[T.nb] - T.off[T.nb - 1]) * (T.off[T.nb] - T.off[T.nb - 1]);
  const int64_t nU = T.oU[T.nb - 1], nL = T.oL[T.nb - 1] + (T.off[T.nb] - T.off[T.nb - 1]) *
                                                              (T.off[T.nb - 1] - T.off[T.nb - 2]);
  if ((e = launch_fill(s, nD, 0.0, T.D)) != hipSuccess) return e;
  if ((e = launch_fill(s, nU, 0.0, T.U)) != hipSuccess) return e;
  if ((e = launch_fill(s, nU, 0.0, T.X)) != hipSuccess) return e;
  if ((e = launch_fill(s, nL, 0.0, T.Lc)) != hipSuccess) return e;
  bt_gather_kernel<<<grid_of(n * 64), 256, 0, s>>>(n, r0, L.J.row_ptr, L.J.col, L.J.val, T.perm, T.iperm, T.nb,
                                                    T.d_off, T.d_oD, T.d_oU, T.d_oL, T.D, T.U, T.Lc, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int b = 0; b < T.nb; ++b) {
    const int64_t sb = T.off[b + 1] - T.off[b];
    // S_b (already the Schur complement) inverted in place, then exported in natural order
    vk_level V;
    V.cb_rows = {0, sb};
    V.cb_max = sb;
    V.cb_sq = sb * sb;
    V.d_cb_rows = T.d_rows + 2 * b;
    V.d_cb_woff = T.d_rows;  // {0, ...}: the one block starts at offset 0
    V.cb_a = T.D + T.oD[b];
    V.cb_W = V.cb_a;
    V.cb_q = L.cb_q;
    V.cb_used = L.cb_used;
    V.cb_gi = L.cb_gi;
    V.cb_go = L.cb_go;
    V.J.n_rows = sb;
    if ((e = launch_block_invert_dense_any(s, V, status)) != hipSuccess) return e;
    if ((e = launch_block_export(s, V, 0, T.Dinv + T.oD[b])) != hipSuccess) return e;
    if (b + 1 < T.nb) {
      const int64_t sn = T.off[b + 2] - T.off[b + 1];
      // X_b = S_b^{-1} U_b, then S_{b+1} = D_{b+1} - L_{b+1} X_b
      if ((e = gemm<true, false, true>(s, sb, sn, sb, 1.0, T.Dinv + T.oD[b], sb, T.U + T.oU[b], sb, T.X + T.oU[b],
                                       sn)) != hipSuccess)
        return e;
      if ((e = gemm<true, true, false>(s, sn, sn, sb, -1.0, T.Lc + T.oL[b + 1], sb, T.X + T.oU[b], sn,
                                       T.D + T.oD[b + 1], sn)) != hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_bt_solve(hipStream_t s, const vk_level& L, const double* b, double* x) {
  const vk_bt& T = L.bt;
  const int64_t n = T.off[T.nb], r0 = L.cb_rows[0];
  hipError_t e;
  bt_permute_kernel<<<grid_of(n), 256, 0, s>>>(n, T.perm, b + r0, T.bp, false);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // forward: y_i = S_i^{-1} (b_i - L_i y_{i-1})
  for (int i = 0; i < T.nb; ++i) {
    const int64_t si = T.off[i + 1] - T.off[i];
    const double* rhs = T.bp + T.off[i];
    if (i > 0) {
      const int64_t sp = T.off[i] - T.off[i - 1];
      if ((e = gemv(s, si, sp, -1.0, T.Lc + T.oL[i], T.y + T.off[i - 1], rhs, T.w)) != hipSuccess) return e;
      rhs = T.w;
    }
    if ((e = gemv(s, si, si, 1.0, T.Dinv + T.oD[i], rhs, nullptr, T.y + T.off[i])) != hipSuccess) return e;
  }
  // back: x_{nb-1} = y_{nb-1}, x_i = y_i - X_i x_{i+1}; each block scattered to the natural order
  const int64_t sl = T.off[T.nb] - T.off[T.nb - 1];
  bt_permute_kernel<<<grid_of(sl), 256, 0, s>>>(sl, T.perm + T.off[T.nb - 1], T.y + T.off[T.nb - 1], x + r0, true);
  for (int i = T.nb - 2; i >= 0; --i) {
    const int64_t si = T.off[i + 1] - T.off[i], sn = T.off[i + 2] - T.off[i + 1];
    const double* xn = (i + 1 == T.nb - 1) ? T.y + T.off[i + 1] : T.xp + T.off[i + 1];
    if ((e = gemv(s, si, sn, -1.0, T.X + T.oU[i], xn, T.y + T.off[i], T.xp + T.off[i])) != hipSuccess) return e;
    bt_permute_kernel<<<grid_of(si), 256, 0, s>>>(si, T.perm + T.off[i], T.xp + T.off[i], x + r0, true);
  }
  return hipGetLastError();
}
