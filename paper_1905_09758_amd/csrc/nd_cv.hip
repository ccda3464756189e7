// Learned control variate (not part of the paper's method): per-node
// structural features, a 5 -> 128 -> 128 -> n_out MLP (ReLU, ReLU, linear),
// its mean-squared-error gradient and the Adam update, all in fp32 with
// fixed-order reductions (bit-identical across runs).
//
// Parameter layout (flat float vector):
//   W1 [5][128], b1 [128], W2 [128][128], b2 [128], W3 [128][n_out], b3 [n_out]
// with W[k][c] the weight from input k to output c.
#include <cmath>

#include "nd_common.h"

namespace nd {
namespace {

constexpr int kFeat = 5;
constexpr int kWidth = 128;

struct Layout {
  int64_t w1, b1, w2, b2, w3, b3, total;
  __host__ __device__ explicit Layout(int n_out) {
    w1 = 0;
    b1 = w1 + kFeat * kWidth;
    w2 = b1 + kWidth;
    b2 = w2 + kWidth * kWidth;
    w3 = b2 + kWidth;
    b3 = w3 + static_cast<int64_t>(kWidth) * n_out;
    total = b3 + n_out;
  }
};

// ------------------------------------------------------------------ features
// One block per node i (grid-stride).  Bitmap A marks N(i), bitmap B the
// nodes at distance exactly 2.  They live in LDS when the graph fits
// (2 x N bits <= kLdsBitmapBytes), otherwise in the block's own slice of a
// device workspace; either way a block clears its bitmaps once, then clears
// only the words a node touched, and the distance-2 count comes from the
// atomicOr return values, so node i costs O(d_i + sum_{j in N(i)} d_j).
// Each wavefront walks the neighbour list of some j in N(i); a k in N(j)
// that is also in N(i) closes a triangle (each counted twice).
//
// Optionally (diag != null) the same walk gives the exact diagonal of the
// first Chebyshev polynomials of H = D^{-1/2} A D^{-1/2} (no self loops):
//   T_0(H)_ii = 1,  T_1(H)_ii = H_ii = 0,
//   T_2(H)_ii = 2 (H^2)_ii - 1 = 2 sum_{j in N(i)} 1 / (d_i d_j) - 1,
//   T_3(H)_ii = 4 (H^3)_ii - 3 H_ii = 4 sum_{j in N(i)} sum_{k in N(i) & N(j)} 1 / (d_i d_j d_k),
// written to diag[i * ld + m] for m < n_diag (<= 4).  All sums have a fixed
// order (per lane, then lanes and wavefronts in a fixed tree).
constexpr size_t kLdsBitmapBytes = 128 * 1024;

template <bool LDS>
__device__ inline uint32_t bm_or(uint32_t* p, uint32_t bit) {
  if constexpr (LDS) return atomicOr(p, bit);
  else return __hip_atomic_fetch_or(p, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__device__ inline uint32_t bm_get(const uint32_t* p) {
  if constexpr (LDS) return *p;
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__device__ inline void bm_clear(uint32_t* p) {
  if constexpr (LDS) *p = 0u;
  else __hip_atomic_store(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__global__ __launch_bounds__(kBlock) void k_features(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, int64_t n, int64_t words,
                                                     uint32_t* __restrict__ gbm, const float* __restrict__ mean,
                                                     const float* __restrict__ sdev, float* __restrict__ feat,
                                                     float* __restrict__ diag, int64_t ld, int n_diag) {
  extern __shared__ uint32_t lbm[];
  uint32_t* A = LDS ? lbm : gbm + static_cast<int64_t>(blockIdx.x) * 2 * words;
  uint32_t* B = A + words;
  constexpr int NW = kBlock / kWave;
  __shared__ unsigned long long red_u[3][NW];
  __shared__ long long red_max[NW];
  __shared__ double red_d[2][NW];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const bool want_two = feat != nullptr;
  for (int64_t w = tid; w < 2 * words; w += kBlock) bm_clear<LDS>(A + w);
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1], d = e1 - e0;
    unsigned long long dsum = 0;
    long long dmax = 0;
    double inv_sum = 0.0;
    for (int64_t t = e0 + tid; t < e1; t += kBlock) {
      const int32_t j = col[t];
      bm_or<LDS>(&A[j >> 5], 1u << (j & 31));
      const long long dj = row_ptr[j + 1] - row_ptr[j];
      dsum += static_cast<unsigned long long>(dj);
      dmax = dj > dmax ? dj : dmax;
      inv_sum += 1.0 / static_cast<double>(dj);
    }
    __syncthreads();
    unsigned long long tri = 0, two = 0;
    double tri_w = 0.0;
    for (int64_t t = e0 + wid; t < e1; t += NW) {
      const int32_t j = col[t];
      const int64_t u0 = row_ptr[j], u1 = row_ptr[j + 1];
      const double inv_dj = 1.0 / static_cast<double>(u1 - u0);
      for (int64_t u = u0 + lane; u < u1; u += kWave) {
        const int32_t k = col[u];
        const uint32_t bit = 1u << (k & 31);
        if (bm_get<LDS>(&A[k >> 5]) & bit) {
          tri++;
          if (diag) tri_w += inv_dj / static_cast<double>(row_ptr[k + 1] - row_ptr[k]);
        } else if (want_two && k != i) {
          if (!(bm_or<LDS>(&B[k >> 5], bit) & bit)) two++;
        }
      }
    }
    __syncthreads();
    // clear what this node set
    for (int64_t t = e0 + tid; t < e1; t += kBlock) bm_clear<LDS>(&A[col[t] >> 5]);
    if (want_two)
      for (int64_t t = e0 + wid; t < e1; t += NW) {
        const int32_t j = col[t];
        for (int64_t u = row_ptr[j] + lane; u < row_ptr[j + 1]; u += kWave) bm_clear<LDS>(&B[col[u] >> 5]);
      }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      dsum += __shfl_xor(dsum, off, kWave);
      tri += __shfl_xor(tri, off, kWave);
      two += __shfl_xor(two, off, kWave);
      inv_sum += __shfl_xor(inv_sum, off, kWave);
      tri_w += __shfl_xor(tri_w, off, kWave);
      const long long o = __shfl_xor(dmax, off, kWave);
      dmax = o > dmax ? o : dmax;
    }
    if (lane == 0) {
      red_u[0][wid] = dsum;
      red_u[1][wid] = tri;
      red_u[2][wid] = two;
      red_max[wid] = dmax;
      red_d[0][wid] = inv_sum;
      red_d[1][wid] = tri_w;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long S = 0, T = 0, W = 0;
      long long X = 0;
      double IS = 0.0, TW = 0.0;
      for (int w = 0; w < NW; ++w) {
        S += red_u[0][w];
        T += red_u[1][w];
        W += red_u[2][w];
        X = red_max[w] > X ? red_max[w] : X;
        IS += red_d[0][w];
        TW += red_d[1][w];
      }
      const double dd = static_cast<double>(d);
      if (feat) {
        const double t_i = static_cast<double>(T) / 2.0;
        double f[kFeat];
        f[0] = log1p(dd);
        f[1] = log1p(static_cast<double>(S) / dd);
        f[2] = log1p(static_cast<double>(X));
        f[3] = log1p(d >= 2 ? 2.0 * t_i / (dd * (dd - 1.0)) : 0.0);
        f[4] = log1p(static_cast<double>(W));
        for (int c = 0; c < kFeat; ++c) {
          float v = static_cast<float>(f[c]);
          if (mean) v = (v - mean[c]) / sdev[c];
          feat[i * kFeat + c] = v;
        }
      }
      if (diag) {
        const double t[4] = {1.0, 0.0, 2.0 * IS / dd - 1.0, 4.0 * TW / dd};
        for (int m = 0; m < n_diag; ++m) diag[i * ld + m] = static_cast<float>(t[m]);
      }
    }
    __syncthreads();
  }
}

// Launch of k_features: LDS bitmaps when they fit, else per-block slices of
// a device workspace of at most kGlobalBitmapBytes (fewer blocks then).
constexpr size_t kGlobalBitmapBytes = size_t(4) << 30;

nd_status launch_features(const nd_graph* g, const float* mean, const float* sdev, float* feat, float* diag,
                          int64_t ld, int n_diag, hipStream_t st) {
  const int64_t n = g->n;
  if (n == 0) return ND_OK;
  const int64_t words = (n + 31) / 32;
  const size_t per_block = static_cast<size_t>(2) * words * sizeof(uint32_t);
  if (per_block <= kLdsBitmapBytes) {
    ND_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_features<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(per_block)));
    const int grid = static_cast<int>(n < 4096 ? n : 4096);
    hipLaunchKernelGGL(k_features<true>, dim3(grid), dim3(kBlock), per_block, st, g->row_ptr, g->col, n, words,
                       static_cast<uint32_t*>(nullptr), mean, sdev, feat, diag, ld, n_diag);
    ND_LAUNCH_CHECK();
    return ND_OK;
  }
  int64_t grid = static_cast<int64_t>(kGlobalBitmapBytes / per_block);
  if (grid > 1024) grid = 1024;
  if (grid > n) grid = n;
  if (grid < 1) {
    set_error("node features: %lld nodes need %zu bytes of bitmaps per block, more than the %zu-byte workspace",
              (long long)n, per_block, kGlobalBitmapBytes);
    return ND_EUNSUPPORTED;
  }
  Tmp t;
  uint32_t* gbm = nullptr;
  ND_CHECK(t.get(&gbm, static_cast<size_t>(grid) * 2 * words));
  hipLaunchKernelGGL(k_features<false>, dim3(static_cast<int>(grid)), dim3(kBlock), 0, st, g->row_ptr, g->col, n,
                     words, gbm, mean, sdev, feat, diag, ld, n_diag);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

// ------------------------------------------------------------------ estimator variance
// Per-probe variance of the per-node estimates from one run's first and
// second probe moments (ldos = mean_j v_ij, ldos_sq = mean_j v_ij^2):
// s2_im = k/(k-1) (ldos_sq - ldos^2).  Block b sums rows [b R, (b+1) R) of
// each column in row order; the final pass adds the blocks in order.
constexpr int kVarBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_var_partial(const double* __restrict__ ld, const double* __restrict__ sq,
                                                        int64_t n, int M, double scale, int64_t rows_per_block,
                                                        double* __restrict__ part) {
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  for (int m = threadIdx.x; m < M; m += kBlock) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double a = ld[r * M + m];
      s += scale * (sq[r * M + m] - a * a);
    }
    part[static_cast<int64_t>(blockIdx.x) * M + m] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_var_final(const double* __restrict__ part, int blocks, int64_t n, int M,
                                                      int m_lo, double* __restrict__ per_m, double* __restrict__ out) {
  __shared__ double col[1024];
  for (int m = threadIdx.x; m < M; m += kBlock) {
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += part[static_cast<int64_t>(b) * M + m];
    col[m] = s / static_cast<double>(n);
    if (per_m) per_m[m] = col[m];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int m = m_lo; m < M; ++m) s += col[m];
    out[0] = s / static_cast<double>(M - m_lo);
  }
}

// ------------------------------------------------------------------ column statistics
constexpr int kStatBlocks = 256;
constexpr int kMaxCols = 16;

__global__ __launch_bounds__(kBlock) void k_col_partial(const float* __restrict__ x, int64_t n, int nc,
                                                        double* __restrict__ part) {
  __shared__ double s1[kBlock][kMaxCols + 1];
  double a[kMaxCols], b[kMaxCols];
  for (int c = 0; c < nc; ++c) a[c] = b[c] = 0.0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < n;
       r += static_cast<int64_t>(gridDim.x) * kBlock)
    for (int c = 0; c < nc; ++c) {
      const double v = x[r * nc + c];
      a[c] += v;
      b[c] += v * v;
    }
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = 0; c < nc; ++c) s1[threadIdx.x][c] = pass ? b[c] : a[c];
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < nc) {
      double s = 0.0;
      for (int t = 0; t < kBlock; ++t) s += s1[t][threadIdx.x];
      part[(static_cast<int64_t>(blockIdx.x) * 2 + pass) * nc + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

__global__ void k_col_final(const double* __restrict__ part, int blocks, int64_t n, int nc, float* __restrict__ mean,
                            float* __restrict__ sdev) {
  const int c = threadIdx.x;
  if (c >= nc) return;
  double s = 0.0, s2 = 0.0;
  for (int b = 0; b < blocks; ++b) {
    s += part[(static_cast<int64_t>(b) * 2) * nc + c];
    s2 += part[(static_cast<int64_t>(b) * 2 + 1) * nc + c];
  }
  const double m = s / static_cast<double>(n);
  double var = s2 / static_cast<double>(n) - m * m;
  if (var < 1e-12) var = 1e-12;
  mean[c] = static_cast<float>(m);
  sdev[c] = static_cast<float>(sqrt(var));
}

// ------------------------------------------------------------------ MLP forward
constexpr int kFwdRows = 64;

__global__ __launch_bounds__(kBlock) void k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ feat,
                                                    int64_t n, int n_out, float* __restrict__ out) {
  __shared__ float xs[kFwdRows][kFeat];
  __shared__ float h1[kFwdRows][kWidth];
  __shared__ float h2[kFwdRows][kWidth];
  const Layout Lo(n_out);
  const int t = threadIdx.x, c = t % kWidth, rg = t / kWidth;  // rg in {0, 1}
  constexpr int RPT = kFwdRows / 2;                             // rows per thread
  for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * kFwdRows; r0 < n; r0 += static_cast<int64_t>(gridDim.x) * kFwdRows) {
    for (int e = t; e < kFwdRows * kFeat; e += kBlock) {
      const int r = e / kFeat, k = e % kFeat;
      xs[r][k] = (r0 + r < n) ? feat[(r0 + r) * kFeat + k] : 0.f;
    }
    __syncthreads();
    for (int i = 0; i < RPT; ++i) {
      const int r = rg + 2 * i;
      float a = P[Lo.b1 + c];
      for (int k = 0; k < kFeat; ++k) a += xs[r][k] * P[Lo.w1 + k * kWidth + c];
      h1[r][c] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    {
      float acc[RPT];
      const float bb = P[Lo.b2 + c];
      for (int i = 0; i < RPT; ++i) acc[i] = bb;
      for (int k = 0; k < kWidth; ++k) {
        const float w = P[Lo.w2 + k * kWidth + c];
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc[i] += h1[rg + 2 * i][k] * w;
      }
      for (int i = 0; i < RPT; ++i) h2[rg + 2 * i][c] = acc[i] > 0.f ? acc[i] : 0.f;
    }
    __syncthreads();
    if (c < n_out) {
      float acc[RPT];
      const float bb = P[Lo.b3 + c];
      for (int i = 0; i < RPT; ++i) acc[i] = bb;
      for (int k = 0; k < kWidth; ++k) {
        const float w = P[Lo.w3 + static_cast<int64_t>(k) * n_out + c];
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc[i] += h2[rg + 2 * i][k] * w;
      }
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = r0 + rg + 2 * i;
        if (r < n) out[r * n_out + c] = acc[i];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ MLP gradient
// One block per tile of 32 rows: forward, output residual, backward, and the
// tile's partial parameter gradient (written to its own slot; summed over
// tiles in order afterwards).
constexpr int kGradRows = 32;

__global__ __launch_bounds__(kBlock) void k_mlp_grad_tile(const float* __restrict__ P, const float* __restrict__ feat,
                                                          const float* __restrict__ target, int ld_target,
                                                          const int32_t* __restrict__ idx, int64_t n, int n_out,
                                                          float scale, float* __restrict__ part,
                                                          float* __restrict__ loss_part) {
  __shared__ float xs[kGradRows][kFeat];
  __shared__ float a1[kGradRows][kWidth];
  __shared__ float a2[kGradRows][kWidth];
  __shared__ float d3[kGradRows][kWidth];  // output residual, later d1
  __shared__ float d2[kGradRows][kWidth];
  __shared__ float lred[kBlock];
  const Layout Lo(n_out);
  const int t = threadIdx.x, c = t % kWidth, rg = t / kWidth;
  constexpr int RPT = kGradRows / 2;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kGradRows;
  float* g = part + static_cast<int64_t>(blockIdx.x) * Lo.total;
  auto src_row = [&](int r) -> int64_t {
    const int64_t b = r0 + r;
    if (b >= n) return -1;
    return idx ? static_cast<int64_t>(idx[b]) : b;
  };
  for (int e = t; e < kGradRows * kFeat; e += kBlock) {
    const int r = e / kFeat, k = e % kFeat;
    const int64_t s = src_row(r);
    xs[r][k] = s >= 0 ? feat[s * kFeat + k] : 0.f;
  }
  __syncthreads();
  // forward
  for (int i = 0; i < RPT; ++i) {
    const int r = rg + 2 * i;
    float a = P[Lo.b1 + c];
    for (int k = 0; k < kFeat; ++k) a += xs[r][k] * P[Lo.w1 + k * kWidth + c];
    a1[r][c] = a;
  }
  __syncthreads();
  {
    float acc[RPT];
    for (int i = 0; i < RPT; ++i) acc[i] = P[Lo.b2 + c];
    for (int k = 0; k < kWidth; ++k) {
      const float w = P[Lo.w2 + k * kWidth + c];
#pragma unroll
      for (int i = 0; i < RPT; ++i) acc[i] += fmaxf(a1[rg + 2 * i][k], 0.f) * w;
    }
    for (int i = 0; i < RPT; ++i) a2[rg + 2 * i][c] = acc[i];
  }
  __syncthreads();
  float lsum = 0.f;
  if (c < n_out) {
    float acc[RPT];
    for (int i = 0; i < RPT; ++i) acc[i] = P[Lo.b3 + c];
    for (int k = 0; k < kWidth; ++k) {
      const float w = P[Lo.w3 + static_cast<int64_t>(k) * n_out + c];
#pragma unroll
      for (int i = 0; i < RPT; ++i) acc[i] += fmaxf(a2[rg + 2 * i][k], 0.f) * w;
    }
    for (int i = 0; i < RPT; ++i) {
      const int r = rg + 2 * i;
      const int64_t s = src_row(r);
      float res = 0.f;
      if (s >= 0) {
        res = acc[i] - target[s * ld_target + c];
        lsum += res * res;
      }
      d3[r][c] = scale * res;  // d loss / d out, loss = mean of squared residuals
    }
  }
  lred[t] = lsum;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
    for (int u = 0; u < kBlock; ++u) s += lred[u];
    loss_part[blockIdx.x] = s;
  }
  // gradients of layer 3
  for (int o = t; o < kWidth * n_out; o += kBlock) {
    const int k = o / n_out, cc = o % n_out;
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += fmaxf(a2[r][k], 0.f) * d3[r][cc];
    g[Lo.w3 + o] = s;
  }
  for (int cc = t; cc < n_out; cc += kBlock) {
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += d3[r][cc];
    g[Lo.b3 + cc] = s;
  }
  // d2 = (d3 W3^T) * relu'(a2)
  for (int i = 0; i < RPT; ++i) {
    const int r = rg + 2 * i;
    float s = 0.f;
    for (int cc = 0; cc < n_out; ++cc) s += d3[r][cc] * P[Lo.w3 + static_cast<int64_t>(c) * n_out + cc];
    d2[r][c] = a2[r][c] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // gradients of layer 2
  for (int o = t; o < kWidth * kWidth; o += kBlock) {
    const int k = o / kWidth, cc = o % kWidth;
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += fmaxf(a1[r][k], 0.f) * d2[r][cc];
    g[Lo.w2 + o] = s;
  }
  if (t < kWidth) {
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += d2[r][t];
    g[Lo.b2 + t] = s;
  }
  // d1 = (d2 W2^T) * relu'(a1), into d3
  for (int i = 0; i < RPT; ++i) {
    const int r = rg + 2 * i;
    float s = 0.f;
    for (int cc = 0; cc < kWidth; ++cc) s += d2[r][cc] * P[Lo.w2 + c * kWidth + cc];
    d3[r][c] = a1[r][c] > 0.f ? s : 0.f;
  }
  __syncthreads();
  for (int o = t; o < kFeat * kWidth; o += kBlock) {
    const int k = o / kWidth, cc = o % kWidth;
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += xs[r][k] * d3[r][cc];
    g[Lo.w1 + o] = s;
  }
  if (t < kWidth) {
    float s = 0.f;
    for (int r = 0; r < kGradRows; ++r) s += d3[r][t];
    g[Lo.b1 + t] = s;
  }
}

// grad[p] = sum over tiles in order; loss = sum of tile losses * loss_scale.
__global__ __launch_bounds__(kBlock) void k_grad_reduce(const float* __restrict__ part, int tiles, int64_t np,
                                                        float* __restrict__ grad, const float* __restrict__ loss_part,
                                                        float loss_scale, float* __restrict__ loss) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < np;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    float s = 0.f;
    for (int b = 0; b < tiles; ++b) s += part[static_cast<int64_t>(b) * np + p];
    grad[p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < tiles; ++b) s += loss_part[b];
    *loss = static_cast<float>(s * loss_scale);
  }
}

__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                                 const float* __restrict__ g, int64_t n, float lr, float bc1,
                                                 float bc2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

Scratch& grad_scratch() {
  static Scratch s;
  return s;
}

}  // namespace
}  // namespace nd

extern "C" {

nd_status nd_node_features(const nd_graph* g, const float* mean, const float* std, float* feat, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(g != nullptr && feat != nullptr, "nd_node_features: graph or feat is NULL");
  ND_REQUIRE((mean == nullptr) == (std == nullptr), "nd_node_features: give both mean and std, or neither");
  return launch_features(g, mean, std, feat, nullptr, 0, 0, as_stream(stream));
}

nd_status nd_cv_exact_diag(const nd_graph* g, float* cv_g, int64_t ld, int32_t n_cols, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(g != nullptr && cv_g != nullptr, "nd_cv_exact_diag: graph or cv_g is NULL");
  ND_REQUIRE(n_cols >= 1 && n_cols <= 4, "nd_cv_exact_diag: n_cols=%d must be 1..4", n_cols);
  ND_REQUIRE(ld >= n_cols, "nd_cv_exact_diag: ld=%lld < n_cols=%d", (long long)ld, n_cols);
  return launch_features(g, nullptr, nullptr, nullptr, cv_g, ld, n_cols, as_stream(stream));
}

nd_status nd_column_stats(const float* x, int64_t n_rows, int32_t n_cols, float* mean, float* std, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(x && mean && std, "nd_column_stats: NULL pointer");
  ND_REQUIRE(n_rows >= 1 && n_cols >= 1 && n_cols <= kMaxCols, "nd_column_stats: n_rows=%lld n_cols=%d",
             (long long)n_rows, n_cols);
  hipStream_t st = as_stream(stream);
  double* part = nullptr;
  ND_CHECK(dalloc_t(&part, static_cast<size_t>(kStatBlocks) * 2 * n_cols));
  hipLaunchKernelGGL(k_col_partial, dim3(kStatBlocks), dim3(kBlock), 0, st, x, n_rows, n_cols, part);
  hipLaunchKernelGGL(k_col_final, dim3(1), dim3(64), 0, st, part, kStatBlocks, n_rows, n_cols, mean, std);
  nd_status s = hipGetLastError() == hipSuccess ? ND_OK : ND_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) s = ND_EDEVICE;
  dfree(part);
  if (s != ND_OK) set_error("nd_column_stats: kernel failure");
  return s;
}

nd_status nd_mlp_forward(const float* params, const float* feat, int64_t n, int32_t n_out, float* g, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(params && feat && g, "nd_mlp_forward: NULL pointer");
  ND_REQUIRE(n >= 0 && n_out >= 1 && n_out <= kWidth, "nd_mlp_forward: n=%lld n_out=%d", (long long)n, n_out);
  if (n == 0) return ND_OK;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_for(n, kFwdRows)), dim3(kBlock), 0, as_stream(stream), params, feat, n,
                     n_out, g);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

nd_status nd_mlp_grad(const float* params, const float* feat, const float* target, int32_t ld_target,
                      const int32_t* idx, int64_t n, int32_t n_out, float* grad, float* loss, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(params && feat && target && grad && loss, "nd_mlp_grad: NULL pointer");
  ND_REQUIRE(n >= 1 && n_out >= 1 && n_out <= kWidth && ld_target >= n_out,
             "nd_mlp_grad: n=%lld n_out=%d ld_target=%d", (long long)n, n_out, ld_target);
  const Layout Lo(n_out);
  const int64_t tiles = ceil_div(n, kGradRows);
  ND_REQUIRE(tiles <= 1 << 20, "nd_mlp_grad: batch of %lld rows is too large", (long long)n);
  Scratch& sc = grad_scratch();
  ND_CHECK(sc.ensure(static_cast<size_t>(tiles) * (Lo.total + 1) * sizeof(float)));
  float* part = sc.as<float>();
  float* loss_part = part + tiles * Lo.total;
  hipStream_t st = as_stream(stream);
  const float scale = 2.0f / static_cast<float>(static_cast<double>(n) * n_out);
  hipLaunchKernelGGL(k_mlp_grad_tile, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, params, feat, target,
                     ld_target, idx, n, n_out, scale, part, loss_part);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(Lo.total, kBlock)), dim3(kBlock), 0, st, part,
                     static_cast<int>(tiles), Lo.total, grad, loss_part,
                     static_cast<float>(1.0 / (static_cast<double>(n) * n_out)), loss);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

nd_status nd_adam_step(float* params, float* m, float* v, const float* grad, int64_t n_params, int32_t t, float lr,
                       void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(params && m && v && grad, "nd_adam_step: NULL pointer");
  ND_REQUIRE(n_params >= 1 && t >= 1, "nd_adam_step: n_params=%lld t=%d", (long long)n_params, t);
  const float bc1 = static_cast<float>(1.0 - std::pow(0.9, t));
  const float bc2 = static_cast<float>(1.0 - std::pow(0.999, t));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n_params, kBlock)), dim3(kBlock), 0, as_stream(stream), params, m, v, grad,
                     n_params, lr, bc1, bc2);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

}  // extern "C"

nd_status nd_ldos_variance(const double* ldos, const double* ldos_sq, int64_t n, int32_t n_moments, int32_t m_lo,
                           int32_t n_probes, double* out, double* per_m, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(ldos != nullptr && ldos_sq != nullptr && out != nullptr, "nd_ldos_variance: a buffer is NULL");
  ND_REQUIRE(n >= 1, "nd_ldos_variance: n=%lld must be >= 1", (long long)n);
  ND_REQUIRE(n_moments >= 1 && n_moments <= 1024, "nd_ldos_variance: n_moments=%d must be 1..1024", n_moments);
  ND_REQUIRE(m_lo >= 0 && m_lo < n_moments, "nd_ldos_variance: m_lo=%d not in [0, %d)", m_lo, n_moments);
  ND_REQUIRE(n_probes >= 2, "nd_ldos_variance: n_probes=%d must be >= 2", n_probes);
  hipStream_t st = as_stream(stream);
  const int64_t rpb = ceil_div(n, static_cast<int64_t>(kVarBlocks));
  const int blocks = static_cast<int>(ceil_div(n, rpb));
  Tmp t;
  double* part = nullptr;
  ND_CHECK(t.get(&part, static_cast<size_t>(blocks) * n_moments));
  const double scale = static_cast<double>(n_probes) / (n_probes - 1.0);
  hipLaunchKernelGGL(k_var_partial, dim3(blocks), dim3(kBlock), 0, st, ldos, ldos_sq, n, n_moments, scale, rpb, part);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_var_final, dim3(1), dim3(kBlock), 0, st, part, blocks, n, n_moments, m_lo, per_m, out);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

nd_status nd_motif_diag(const nd_motifs* motifs, float* cv_g, int64_t ld, int32_t n_cols, double scale,
                        void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(motifs != nullptr && cv_g != nullptr, "nd_motif_diag: motifs or cv_g is NULL");
  ND_REQUIRE(n_cols >= 1 && ld >= n_cols, "nd_motif_diag: n_cols=%d, ld=%lld (need 1 <= n_cols <= ld)", n_cols,
             (long long)ld);
  if (motifs->n_classes == 0) return ND_OK;
  hipLaunchKernelGGL(k_motif_diag<float>, dim3(grid_for(motifs->n_members, kBlock)), dim3(kBlock), 0,
                     as_stream(stream), motifs->class_ptr, motifs->members, motifs->class_lambda,
                     motifs->class_paired, motifs->n_classes, motifs->n_members, ld, n_cols, scale, cv_g);
  ND_LAUNCH_CHECK();
  return ND_OK;
}
