// Grouped CSR of a level's J: the plan (host) and the choice between it and CSR for the J products.
// The format itself and its kernel are described with spmv_g_kernel in sparse.hip.
#include <vector>

#include "vk_internal.h"

// LPR lanes per group from the mean row length of the groups' rows
int vk_pick_lpr_g(int64_t nnz, int64_t n_rows) {
  const double avg = n_rows > 0 ? (double)nnz / (double)n_rows : 0.0;
  if (avg >= 128) return 32;
  if (avg >= 48) return 16;
  if (avg >= 16) return 8;
  return 4;
}

// Greedy over the rows in order: a group takes the largest G in {4, 3, 2} for which the next G
// rows have the first row's length and columns col[r][j] + c d_j (d_j in {0, 1}), else G = 1.
// Copies the pattern to the host once; returns false (CSR stays) if the pattern needs more column
// words or groups than reserved, or a copy fails.
bool vk_gcsr_plan(vk_level& L) {
  vk_gcsr& G = L.gJ;
  G.planned = true;
  G.active = false;
  G.n_groups = 0;
  const vk_csr& A = L.J;
  const int64_t n = A.n_rows, nnz = A.nnz;
  if (!G.gcol || !G.g_v0 || n <= 0 || nnz < VK_GCSR_MIN_NNZ || A.n_cols > INT32_MAX) return false;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> col(nnz);
  if (hipMemcpy(rp.data(), A.row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(col.data(), A.col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  std::vector<int32_t> grow;
  std::vector<int64_t> gcoff, gv0;
  std::vector<uint32_t> words;
  grow.reserve(n / 2 + 2);
  gcoff.reserve(n / 2 + 2);
  gv0.reserve(n / 2 + 2);
  words.reserve(G.cap_words);
  int64_t r = 0;
  while (r < n) {
    const int64_t e0 = rp[r], m = rp[r + 1] - e0;
    int best = 1;
    for (int g = 4; g >= 2 && best == 1; --g) {
      if (r + g > n) continue;
      bool ok = true;
      for (int c = 1; c < g && ok; ++c) ok = rp[r + c + 1] - rp[r + c] == m;
      for (int64_t j = 0; j < m && ok; ++j) {
        const int64_t base = col[e0 + j], d = (int64_t)col[e0 + m + j] - base;
        ok = d == 0 || d == 1;
        for (int c = 2; c < g && ok; ++c) ok = (int64_t)col[e0 + c * m + j] == base + c * d;
      }
      if (ok) best = g;
    }
    if ((int64_t)words.size() + m > G.cap_words) return false;
    grow.push_back((int32_t)r);
    gcoff.push_back((int64_t)words.size());
    gv0.push_back(e0);
    for (int64_t j = 0; j < m; ++j) {
      const uint32_t d = best > 1 ? (uint32_t)(col[e0 + m + j] - col[e0 + j]) : 0u;
      words.push_back((uint32_t)col[e0 + j] | (d << 31));
    }
    r += best;
  }
  grow.push_back((int32_t)n);
  gcoff.push_back((int64_t)words.size());
  gv0.push_back(nnz);
  const int64_t ng = (int64_t)grow.size() - 1;
  if (ng > G.cap_groups) return false;
  if (hipMemcpy(G.g_row, grow.data(), sizeof(int32_t) * (ng + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.g_coff, gcoff.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.g_v0, gv0.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.gcol, words.data(), sizeof(uint32_t) * words.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  G.n_groups = ng;
  G.active = true;
  return true;
}

hipError_t launch_spmv_J(hipStream_t s, const vk_level& L, double alpha, const double* x, double beta,
                         const double* z, double* y) {
  if (L.use_gJ && L.gJ.active) return launch_spmv_g(s, L.J, L.gJ, L.lpr_gJ, alpha, x, beta, z, y);
  return launch_spmv(s, L.J, L.lpr_J, alpha, x, beta, z, y);
}
