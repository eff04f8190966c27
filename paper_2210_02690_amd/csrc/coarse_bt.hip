// Direct solve of a wide directly solved block through its block-tridiagonal structure (Sec. 3: a
// direct solver for J_0 d_0 = b_0 on T_0; the paper names no method).
//
// Breadth-first level sets of the block's symmetrised sparsity graph, started from a
// pseudo-peripheral vertex, couple only to themselves and to the neighbouring sets.  Consecutive
// level sets are grouped into blocks of at least VK_BT_MIN_BLOCK unknowns; in that order the block is
// block tridiagonal, with diagonal blocks D_i and couplings U_i (block i to i + 1) and L_i (block i
// to i - 1).  The factorisation is block Gaussian elimination from both ends towards a middle block
// c, so the two chains run side by side (one launch sequence inverts a block of each):
//   left,  i < c:  S_0 = D_0,         X_i = S_i^{-1} U_i,  S_{i+1} = D_{i+1} - L_{i+1} X_i,
//   right, i > c:  T_{nb-1} = D_{nb-1}, Y_i = T_i^{-1} L_i,  T_{i-1} = D_{i-1} - U_{i-1} Y_i,
//   middle:        S_c = D_c - L_c X_{c-1} - U_c Y_{c+1},
// each S_i, T_i inverted densely by the blocked Gauss-Jordan kernels (implicit partial pivoting
// inside the block).  The solve runs inwards, y_0 = S_0^{-1} b_0, y_i = S_i^{-1} (b_i - L_i y_{i-1});
// z_{nb-1} = T_{nb-1}^{-1} b_{nb-1}, z_i = T_i^{-1} (b_i - U_i z_{i+1}); x_c = S_c^{-1} (b_c - L_c
// y_{c-1} - U_c z_{c+1}); and outwards, x_i = y_i - X_i x_{i+1} (i < c), x_i = z_i - Y_i x_{i-1}
// (i > c).  It computes J_0^{-1} b up to rounding like the dense inverse, with 2 sum s_i^3 + 4 sum
// s_i^2 s_{i+/-1} flop instead of 2 n^3, and about nb / 2 steps of small inversions instead of one
// wide one.  A block with no nonzero pivot is reported like a singular dense block.
//
// Layout (carved from the level's dense-inverse buffer, which this path does not otherwise use):
// D_i column-major (the Gauss-Jordan input, overwritten); the inverses, U_i, L_i, X_i and Y_i
// row-major (GEMM operands, and the solve reads them a row per wavefront).
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
    else if (bc == b + 1) U[oU[b] + ri * (off[b + 2] - off[b + 1]) + cj] = val[e];
    else if (bc == b - 1) Lc[oL[b] + ri * (off[b] - off[b - 1]) + cj] = val[e];
    else atomicOr(&status[1], 2);
  }
}

// C += alpha A B for C (m x n, ldc), A (m x k, lda), B (k x n, ldb), each row-major (the *_ROW
// flag) or column-major.  64 x 64 tiles of C per 256-thread workgroup, 16-step chunks of k through
// LDS; thread (tx, ty) owns rows ty + 16 i and columns tx + 16 j (i, j < 4).  Up to two independent
// products per launch (blockIdx.z), for the two elimination chains.
struct GemmP {
  int64_t m, n, k;
  double alpha;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
};

template <bool A_ROW, bool B_ROW, bool C_ROW>
__global__ __launch_bounds__(256) void bt_gemm_kernel(GemmP p0, GemmP p1) {
  const GemmP& p = blockIdx.z ? p1 : p0;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
  if (m0 >= p.m || n0 >= p.n) return;  // uniform: the grid covers the larger product
  const int64_t m = p.m, n = p.n, k = p.k, lda = p.lda, ldb = p.ldb;
  const double* __restrict__ A = p.A;
  const double* __restrict__ B = p.B;
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
  double* C = p.C;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = n0 + tx + 16 * j;
    if (c >= n) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = m0 + ty + 16 * i;
      if (r < m) (C_ROW ? C[r * p.ldc + c] : C[c * p.ldc + r]) += p.alpha * acc[i][j];
    }
  }
}

// y[r] = (base ? base[r] : 0) + alpha sum_j A[r lda + j] x[j], A (m x k) row-major: one wavefront
// per row, two loads in flight per lane.  Up to two independent products per launch (blockIdx.y).
struct GemvP {
  int64_t m, k;
  double alpha;
  const double* A;
  const double* x;
  const double* base;
  double* y;
};

__global__ __launch_bounds__(256) void bt_gemv_kernel(GemvP p0, GemvP p1) {
  const GemvP& p = blockIdx.y ? p1 : p0;
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= p.m) return;
  const int64_t k = p.k;
  const double* __restrict__ a = p.A + r * k;
  const double* __restrict__ x = p.x;
  double s0 = 0.0, s1 = 0.0;
  int64_t j = lane;
  for (; j + 64 < k; j += 128) {
    s0 = fma(a[j], x[j], s0);
    s1 = fma(a[j + 64], x[j + 64], s1);
  }
  if (j < k) s0 = fma(a[j], x[j], s0);
  double s = s0 + s1;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) p.y[r] = (p.base ? p.base[r] : 0.0) + p.alpha * s;
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

// one or two products (np = 1, 2) in one launch
template <bool A_ROW, bool B_ROW, bool C_ROW>
hipError_t gemm2(hipStream_t s, int np, const GemmP& p0, const GemmP& p1) {
  const int64_t m = np > 1 ? std::max(p0.m, p1.m) : p0.m, n = np > 1 ? std::max(p0.n, p1.n) : p0.n;
  bt_gemm_kernel<A_ROW, B_ROW, C_ROW><<<dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64), (unsigned)np),
                                        256, 0, s>>>(p0, np > 1 ? p1 : p0);
  return hipGetLastError();
}

hipError_t gemv2(hipStream_t s, int np, const GemvP& p0, const GemvP& p1) {
  const int64_t m = np > 1 ? std::max(p0.m, p1.m) : p0.m;
  bt_gemv_kernel<<<dim3(grid_of(m * 64), (unsigned)np), 256, 0, s>>>(p0, np > 1 ? p1 : p0);
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
  // two pseudo-peripheral ends: s1, the last level's vertex of a search from vertex 0, and s2,
  // the last level's vertex of a search from s1; d1, d2 the distances from them.  With D =
  // d1(s2) and h = D / 2, the left part {d1 < h} and the right part {d2 < D - h} share no edge
  // (d1 + d2 >= D, and an edge changes each by at most one); the rest is the middle block.
  // Each part is cut into blocks of consecutive levels of its own search, from its end inwards,
  // so both chains start at a corner of the mesh (a block there is a whole neighbourhood of
  // cells, not one thin layer of level sets, whose principal submatrix can be singular).
  std::vector<int32_t> d1, d2;
  int32_t s1 = 0, s2 = 0;
  if (bfs_levels(n, deg, adj, 0, d1, &s1) < 0) return false;
  if (bfs_levels(n, deg, adj, s1, d1, &s2) < 0) return false;
  int32_t tmp = 0;
  if (bfs_levels(n, deg, adj, s2, d2, &tmp) < 0) return false;
  const int dist = d1[s2];
  const int h1 = dist / 2, h2 = dist - h1;
  if (h1 < 1 || h2 < 1) return false;
  // part of each vertex (0 left, 1 middle, 2 right) and its level within the part
  std::vector<int64_t> lcnt(h1, 0), rcnt(h2, 0);
  int64_t nmid = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (d1[v] < h1) ++lcnt[d1[v]];
    else if (d2[v] < h2) ++rcnt[d2[v]];
    else ++nmid;
  }
  // consecutive levels into blocks of at least VK_BT_MIN_BLOCK unknowns, from the end inwards
  // (a remainder joins the block before it)
  auto group = [](const std::vector<int64_t>& cnt, std::vector<int32_t>& lblk, std::vector<int64_t>& bs) {
    lblk.assign(cnt.size(), 0);
    bs.clear();
    int64_t cur = 0;
    for (size_t l = 0; l < cnt.size(); ++l) {
      if (bs.empty() || cur >= VK_BT_MIN_BLOCK) {
        bs.push_back(0);
        cur = 0;
      }
      lblk[l] = (int32_t)bs.size() - 1;
      bs.back() += cnt[l];
      cur += cnt[l];
    }
    if (bs.size() > 1 && bs.back() < VK_BT_MIN_BLOCK) {
      const int64_t tail = bs.back();
      bs.pop_back();
      bs.back() += tail;
      for (size_t l = 0; l < cnt.size(); ++l)
        if (lblk[l] == (int32_t)bs.size()) lblk[l] = (int32_t)bs.size() - 1;
    }
  };
  std::vector<int32_t> lb, rb;
  std::vector<int64_t> lsz, rsz;
  group(lcnt, lb, lsz);
  group(rcnt, rb, rsz);
  if (lsz.empty() || rsz.empty() || nmid == 0) return false;
  // the order: left blocks from s1's end, the middle, right blocks towards s2's end
  const int nl = (int)lsz.size(), nr = (int)rsz.size();
  const int nb = nl + 1 + nr;
  std::vector<int64_t> bsize(nb);
  for (int i = 0; i < nl; ++i) bsize[i] = lsz[i];
  bsize[nl] = nmid;
  for (int i = 0; i < nr; ++i) bsize[nb - 1 - i] = rsz[i];
  int64_t smax = 0;
  for (int64_t sz : bsize) smax = std::max(smax, sz);
  if (smax > VK_BT_MAX_BLOCK) return false;
  // the new order: by block, then by row
  T.off.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) T.off[b + 1] = T.off[b] + bsize[b];
  std::vector<int64_t> pos(T.off.begin(), T.off.end() - 1);
  std::vector<int32_t> perm(n), iperm(n);
  for (int64_t v = 0; v < n; ++v) {
    const int blk = d1[v] < h1 ? lb[d1[v]] : (d2[v] < h2 ? nb - 1 - rb[d2[v]] : nl);
    const int64_t p = pos[blk]++;
    perm[p] = (int32_t)v;
    iperm[v] = (int32_t)p;
  }
  T.c = nl;
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
  // the elimination steps: the left chain 0 .. c-1 and the right chain nb-1 .. c+1 side by side,
  // then the middle block c
  const int nsteps = std::max(T.c, nb - 1 - T.c) + 1;
  T.pa.assign(nsteps, -1);
  T.pb.assign(nsteps, -1);
  for (int k = 0; k + 1 < nsteps; ++k) {
    if (k < T.c) T.pa[k] = k;
    if (nb - 1 - k > T.c) T.pb[k] = nb - 1 - k;
  }
  T.pa[nsteps - 1] = T.c;
  std::vector<int64_t> prows(3 * nsteps), pwoff(2 * nsteps);
  for (int k = 0; k < nsteps; ++k) {
    const int a = T.pa[k] >= 0 ? T.pa[k] : T.pb[k], b = T.pa[k] >= 0 ? T.pb[k] : -1;
    prows[3 * k] = 0;
    prows[3 * k + 1] = bsize[a];
    prows[3 * k + 2] = bsize[a] + (b >= 0 ? bsize[b] : 0);
    pwoff[2 * k] = T.oD[a];
    pwoff[2 * k + 1] = b >= 0 ? T.oD[b] : 0;
  }
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  const int64_t ints = up((3 * n + 1) / 2 + 1);                           // perm, iperm (as doubles)
  const int64_t idx = up(4 * nb + 1 + 5 * nsteps);                        // off, oD, oU, oL, prows, pwoff
  const int64_t need = 2 * up(sD) + up(sU) * 2 + up(sL) * 2 + 3 * up(n) + up(2 * smax) + ints + idx;
  if (need > L.cb_sq) return false;
  double* p = L.cb_a;
  T.D = p;    p += up(sD);
  T.Dinv = p; p += up(sD);
  T.U = p;    p += up(sU);
  T.X = p;    p += up(sU);
  T.Lc = p;   p += up(sL);
  T.Y = p;    p += up(sL);
  T.bp = p;   p += up(n);
  T.y = p;    p += up(n);
  T.xp = p;   p += up(n);
  T.w = p;    p += up(2 * smax);
  T.perm = reinterpret_cast<int32_t*>(p);
  T.iperm = T.perm + n;
  p += ints;
  int64_t* q = reinterpret_cast<int64_t*>(p);
  T.d_off = q;        q += nb + 1;
  T.d_oD = q;         q += nb;
  T.d_oU = q;         q += nb;
  T.d_oL = q;         q += nb;
  T.d_prows = q;      q += 3 * nsteps;
  T.d_pwoff = q;      q += 2 * nsteps;
  if (hipMemcpy(T.perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.iperm, iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_off, T.off.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oD, T.oD.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oU, T.oU.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_oL, T.oL.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_prows, prows.data(), sizeof(int64_t) * 3 * nsteps, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(T.d_pwoff, pwoff.data(), sizeof(int64_t) * 2 * nsteps, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  // inversions 2 s_i^3; per chain step the coupling product (2 s_i^2 s_j) and the Schur update of
  // the next block (2 s_j^2 s_i), j the next block inwards
  T.flops = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double sb = (double)bsize[b];
    T.flops += 2.0 * sb * sb * sb;
    const int j = b < T.c ? b + 1 : (b > T.c ? b - 1 : -1);
    if (j >= 0) {
      const double sj = (double)bsize[j];
      T.flops += 2.0 * sb * sb * sj + 2.0 * sj * sj * sb;
    }
  }
  T.active = true;
  return true;
}

hipError_t launch_bt_factor(hipStream_t s, const vk_level& L, int32_t* status) {
  const vk_bt& T = L.bt;
  const int nb = T.nb, c = T.c, nsteps = (int)T.pa.size();
  const int64_t n = T.off[nb], r0 = L.cb_rows[0];
  auto sz = [&](int b) { return T.off[b + 1] - T.off[b]; };
  hipError_t e;
  const int64_t nD = T.oD[nb - 1] + sz(nb - 1) * sz(nb - 1);
  const int64_t nU = T.oU[nb - 1], nL = T.oL[nb - 1] + sz(nb - 1) * sz(nb - 2);
  if ((e = launch_fill(s, nD, 0.0, T.D)) != hipSuccess) return e;
  if ((e = launch_fill(s, nU, 0.0, T.U)) != hipSuccess) return e;
  if ((e = launch_fill(s, nU, 0.0, T.X)) != hipSuccess) return e;
  if ((e = launch_fill(s, nL, 0.0, T.Lc)) != hipSuccess) return e;
  if ((e = launch_fill(s, nL, 0.0, T.Y)) != hipSuccess) return e;
  bt_gather_kernel<<<grid_of(n * 64), 256, 0, s>>>(n, r0, L.J.row_ptr, L.J.col, L.J.val, T.perm, T.iperm, nb,
                                                    T.d_off, T.d_oD, T.d_oU, T.d_oL, T.D, T.U, T.Lc, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k = 0; k < nsteps; ++k) {
    // the step's blocks (already Schur complements), inverted in place by one launch sequence,
    // then exported in natural order
    const int bl[2] = {T.pa[k] >= 0 ? T.pa[k] : T.pb[k], T.pa[k] >= 0 ? T.pb[k] : -1};
    const int nbk = bl[1] >= 0 ? 2 : 1;
    vk_level V;
    V.cb_rows = {0, sz(bl[0])};
    if (nbk == 2) V.cb_rows.push_back(sz(bl[0]) + sz(bl[1]));
    V.cb_max = nbk == 2 ? std::max(sz(bl[0]), sz(bl[1])) : sz(bl[0]);
    V.cb_sq = sz(bl[0]) * sz(bl[0]) + (nbk == 2 ? sz(bl[1]) * sz(bl[1]) : 0);
    V.d_cb_rows = T.d_prows + 3 * k;
    V.d_cb_woff = T.d_pwoff + 2 * k;
    V.cb_a = T.D;
    V.cb_W = T.D;
    V.cb_q = L.cb_q;
    V.cb_used = L.cb_used;
    V.cb_gi = L.cb_gi;
    V.cb_go = L.cb_go;
    V.J.n_rows = V.cb_rows[nbk];
    if ((e = launch_block_invert_dense_any(s, V, status)) != hipSuccess) return e;
    for (int i = 0; i < nbk; ++i) {
      vk_level V1;
      V1.cb_rows = {0, sz(bl[i])};
      V1.cb_W = T.D + T.oD[bl[i]];
      V1.cb_q = L.cb_q + V.cb_rows[i];
      if ((e = launch_block_export(s, V1, 0, T.Dinv + T.oD[bl[i]])) != hipSuccess) return e;
    }
    // the couplings and the Schur complements of the next blocks inwards
    const int a = T.pa[k], b = T.pb[k];
    GemmP cp[2], up[2];
    int np = 0;
    if (a >= 0 && a < c) {  // X_a = S_a^{-1} U_a;  D_{a+1} -= L_{a+1} X_a
      const int64_t sa = sz(a), sn = sz(a + 1);
      cp[np] = GemmP{sa, sn, sa, 1.0, T.Dinv + T.oD[a], sa, T.U + T.oU[a], sn, T.X + T.oU[a], sn};
      up[np] = GemmP{sn, sn, sa, -1.0, T.Lc + T.oL[a + 1], sa, T.X + T.oU[a], sn, T.D + T.oD[a + 1], sn};
      ++np;
    }
    if (b > c) {  // Y_b = T_b^{-1} L_b;  D_{b-1} -= U_{b-1} Y_b
      const int64_t sb = sz(b), sp = sz(b - 1);
      cp[np] = GemmP{sb, sp, sb, 1.0, T.Dinv + T.oD[b], sb, T.Lc + T.oL[b], sp, T.Y + T.oL[b], sp};
      up[np] = GemmP{sp, sp, sb, -1.0, T.U + T.oU[b - 1], sb, T.Y + T.oL[b], sp, T.D + T.oD[b - 1], sp};
      ++np;
    }
    if (np == 0) continue;
    if ((e = gemm2<true, true, true>(s, np, cp[0], cp[np - 1])) != hipSuccess) return e;
    if (np == 2 && up[0].C == up[1].C) {  // both chains end on the middle block: one after the other
      if ((e = gemm2<true, true, false>(s, 1, up[0], up[0])) != hipSuccess) return e;
      if ((e = gemm2<true, true, false>(s, 1, up[1], up[1])) != hipSuccess) return e;
    } else if ((e = gemm2<true, true, false>(s, np, up[0], up[np - 1])) != hipSuccess) {
      return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_bt_solve(hipStream_t s, const vk_level& L, const double* b, double* x) {
  const vk_bt& T = L.bt;
  const int nb = T.nb, c = T.c, nsteps = (int)T.pa.size();
  const int64_t n = T.off[nb], r0 = L.cb_rows[0];
  auto sz = [&](int i) { return T.off[i + 1] - T.off[i]; };
  double* wL = T.w;
  double* wR = T.w + T.smax;
  hipError_t e;
  bt_permute_kernel<<<grid_of(n), 256, 0, s>>>(n, T.perm, b + r0, T.bp, false);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // inwards: y_i = S_i^{-1} (b_i - L_i y_{i-1}) on the left, z_i = T_i^{-1} (b_i - U_i z_{i+1}) on
  // the right, a block of each per launch
  for (int k = 0; k + 1 < nsteps; ++k) {
    const int a = T.pa[k], r = T.pb[k];
    GemvP cp[2], ip[2];
    int nc = 0, ni = 0;
    if (a >= 0) {
      const double* rhs = T.bp + T.off[a];
      if (a > 0) {
        cp[nc++] = GemvP{sz(a), sz(a - 1), -1.0, T.Lc + T.oL[a], T.y + T.off[a - 1], rhs, wL};
        rhs = wL;
      }
      ip[ni++] = GemvP{sz(a), sz(a), 1.0, T.Dinv + T.oD[a], rhs, nullptr, T.y + T.off[a]};
    }
    if (r >= 0) {
      const double* rhs = T.bp + T.off[r];
      if (r < nb - 1) {
        cp[nc++] = GemvP{sz(r), sz(r + 1), -1.0, T.U + T.oU[r], T.y + T.off[r + 1], rhs, wR};
        rhs = wR;
      }
      ip[ni++] = GemvP{sz(r), sz(r), 1.0, T.Dinv + T.oD[r], rhs, nullptr, T.y + T.off[r]};
    }
    if (nc > 0 && (e = gemv2(s, nc, cp[0], cp[nc - 1])) != hipSuccess) return e;
    if (ni > 0 && (e = gemv2(s, ni, ip[0], ip[ni - 1])) != hipSuccess) return e;
  }
  // the middle block: x_c = S_c^{-1} (b_c - L_c y_{c-1} - U_c z_{c+1})  (0 < c < nb - 1)
  const int64_t scc = sz(c);
  GemvP m1{scc, sz(c - 1), -1.0, T.Lc + T.oL[c], T.y + T.off[c - 1], T.bp + T.off[c], wL};
  GemvP m2{scc, sz(c + 1), -1.0, T.U + T.oU[c], T.y + T.off[c + 1], wL, wR};
  GemvP m3{scc, scc, 1.0, T.Dinv + T.oD[c], wR, nullptr, T.xp + T.off[c]};
  if ((e = gemv2(s, 1, m1, m1)) != hipSuccess) return e;
  if ((e = gemv2(s, 1, m2, m2)) != hipSuccess) return e;
  if ((e = gemv2(s, 1, m3, m3)) != hipSuccess) return e;
  // outwards: x_i = y_i - X_i x_{i+1} (i < c), x_i = z_i - Y_i x_{i-1} (i > c)
  for (int k = 0; k < std::max(c, nb - 1 - c); ++k) {
    const int i = c - 1 - k, j = c + 1 + k;
    GemvP bp[2];
    int np = 0;
    if (i >= 0) bp[np++] = GemvP{sz(i), sz(i + 1), -1.0, T.X + T.oU[i], T.xp + T.off[i + 1], T.y + T.off[i], T.xp + T.off[i]};
    if (j < nb) bp[np++] = GemvP{sz(j), sz(j - 1), -1.0, T.Y + T.oL[j], T.xp + T.off[j - 1], T.y + T.off[j], T.xp + T.off[j]};
    if ((e = gemv2(s, np, bp[0], bp[np - 1])) != hipSuccess) return e;
  }
  // back to the natural order
  bt_permute_kernel<<<grid_of(n), 256, 0, s>>>(n, T.perm, T.xp, x + r0, true);
  return hipGetLastError();
}
