// Density reconstruction from Chebyshev moments, in fp64 (Sec. 2.2, 3.1, 4.1).
//
// With damping factors g_m (Jackson, or 1), theta = arccos x and weight
// 1/(pi sqrt(1-x^2)) (eqn orth), the density is
//   rho(x) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi sqrt(1 - x^2))
// and its integral over [a, b] is (F(theta_a) - F(theta_b)) / pi with
//   F(theta) = g_0 mu_0 theta + 2 sum_{m>=1} g_m mu_m sin(m theta) / m.
// Both are a small dense product of the moment rows with a table that
// depends only on (M, bins or points); the table is built once per call.
#include <cmath>
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

__device__ inline double jackson_g(int m, int M) {
  const double a = M_PI / static_cast<double>(M + 1);
  return (static_cast<double>(M - m + 1) * cos(a * m) + sin(a * m) * cos(a) / sin(a)) / static_cast<double>(M + 1);
}

// Column tiles of the product: kTC columns, kKC moments per LDS stage.
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTR = 64;  // rows per block
constexpr int kTC = 64;  // columns per launch
constexpr int kKC = 32;  // moments per stage

// Table Wt[m][c] (m < Mp, c < cpad; zero beyond M and beyond the columns):
// columns 0..n_edges-1 are the bin-edge integrals F, then n_points density
// columns at the Chebyshev nodes.  Moment-major, so that a stage of kKC
// moments of a column tile is one contiguous block.
__global__ __launch_bounds__(kBlock) void k_recon_table(int M, int Mp, int kernel, int n_bins, double lo, double hi,
                                                        int n_points, int cpad, double* __restrict__ Wt) {
  const int n_edges = n_bins > 0 ? n_bins + 1 : 0;
  const int64_t total = static_cast<int64_t>(Mp) * cpad;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int m = static_cast<int>(idx / cpad), c = static_cast<int>(idx % cpad);
    double w = 0.0;
    if (m < M && c < n_edges + n_points) {
      const double g = kernel ? jackson_g(m, M) : 1.0;
      if (c < n_edges) {
        double x = lo + (hi - lo) * static_cast<double>(c) / static_cast<double>(n_bins);
        x = x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x);
        const double th = acos(x);
        w = (m == 0) ? th : 2.0 * sin(static_cast<double>(m) * th) / static_cast<double>(m);
      } else {
        const int k = c - n_edges;
        const double th = M_PI * (static_cast<double>(k) + 0.5) / static_cast<double>(n_points);
        w = ((m == 0) ? 1.0 : 2.0 * cos(static_cast<double>(m) * th)) / (M_PI * sin(th));
      }
      w *= g;
    }
    Wt[idx] = w;
  }
}

// out[row][c] = sum_m mu[row][m] Wt[m][c0 + c] - corr[c0 + c], c < ncols, for
// one tile of kTC table columns: a block owns kTR rows and stages kKC moments
// of its rows and of the column tile in LDS; each wavefront multiplies a
// 32 x 32 quarter of the tile on the fp64 matrix cores, four
// v_mfma_f64_16x16x4f64 per 4 moments.  Their operand layout (any other
// reading fails the reconstruction parity tests): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16], and element
// i of its result is D[4 i + l / 16][l % 16].
// With `hist` set, the tile holds all n_bins + 1 edge columns and the block
// writes the bin masses hist[row][b] = (F_b - F_{b+1}) / pi + spikes directly.
__global__ __launch_bounds__(kBlock) void k_recon_gemm(const double* __restrict__ mu, int64_t n_rows, int M,
                                                       const double* __restrict__ Wt, int cpad, int c0, int ncols,
                                                       const double* __restrict__ corr, double* __restrict__ out,
                                                       int ld_out, double* __restrict__ hist,
                                                       const int32_t* __restrict__ sbin,
                                                       const double* __restrict__ sw, int n_spikes) {
  constexpr int kLdA = kKC + 1;
  __shared__ double lds[kTR * (kTC + 1)];  // >= kTR * kLdA + kKC * kTC
  static_assert(kTR * (kTC + 1) >= kTR * kLdA + kKC * kTC, "LDS tile too small");
  double* sa = lds;                // [kTR][kLdA]
  double* sb = lds + kTR * kLdA;   // [kKC][kTC]
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;  // the wavefront's quarter of the tile
  const int lr = lane % 16, lk = lane / 16;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kTR;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  // stage loads go through registers: the next stage's moments and table
  // entries are in flight while the current stage is multiplied
  constexpr int kPA = kTR * kKC / kBlock, kPB = kKC * kTC / kBlock;
  static_assert(kPA * kBlock == kTR * kKC && kPB * kBlock == kKC * kTC, "stage tile / block size");
  double ra[kPA], rb[kPB];
  auto fetch = [&](int m0) {
    const int mm = M - m0 < kKC ? M - m0 : kKC;
#pragma unroll
    for (int u = 0; u < kPA; ++u) {
      const int t = threadIdx.x + u * kBlock, r = t / kKC, k = t % kKC;
      ra[u] = (r0 + r < n_rows && k < mm) ? mu[(r0 + r) * M + m0 + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPB; ++u) {
      const int t = threadIdx.x + u * kBlock, k = t / kTC, c = t % kTC;
      // only the launch's ncols columns exist past c0 (a tile that starts
      // inside the table, e.g. at the density points, ends before cpad)
      rb[u] = c < ncols ? Wt[static_cast<int64_t>(m0 + k) * cpad + c0 + c] : 0.0;
    }
  };
  fetch(0);
  for (int m0 = 0; m0 < M; m0 += kKC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPA; ++u) {
      const int t = threadIdx.x + u * kBlock;
      sa[(t / kKC) * kLdA + t % kKC] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < kPB; ++u) sb[threadIdx.x + u * kBlock] = rb[u];
    __syncthreads();
    if (m0 + kKC < M) fetch(m0 + kKC);
#pragma unroll
    for (int k0 = 0; k0 < kKC; k0 += 4) {
      double x[2], y[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) x[t] = sa[(wr + 16 * t + lr) * kLdA + k0 + lk];
#pragma unroll
      for (int t = 0; t < 2; ++t) y[t] = sb[(k0 + lk) * kTC + wc + 16 * t + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], y[j], acc[i][j], 0, 0, 0);
    }
  }
  if (!hist) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t r = r0 + wr + 16 * i + 4 * e + lk;
          const int c = wc + 16 * j + lr;
          if (r < n_rows && c < ncols) out[r * ld_out + c] = corr ? acc[i][j][e] - corr[c0 + c] : acc[i][j][e];
        }
    return;
  }
  // fused bins: F tile through LDS, then the differences of adjacent edges
  constexpr int kLdF = kTC + 1;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr + 16 * i + 4 * e + lk, c = wc + 16 * j + lr;
        lds[r * kLdF + c] = corr && c < ncols ? acc[i][j][e] - corr[c] : acc[i][j][e];
      }
  __syncthreads();
  const int nb = ncols - 1;
  for (int t = threadIdx.x; t < kTR * nb; t += kBlock) {
    const int r = t / nb, b = t % nb;
    if (r0 + r >= n_rows) break;
    double h = (lds[r * kLdF + b] - lds[r * kLdF + b + 1]) / M_PI;
    for (int s = 0; s < n_spikes; ++s)
      if (sbin[s] == b) h += sw[s];
    hist[(r0 + r) * nb + b] = h;
  }
}

// corr[c] = sum_s w_s sum_m T_m(lambda_s) Wt[m][c]: the part of column c that
// the point masses contribute when the moments include them.
__global__ __launch_bounds__(kBlock) void k_spike_corr(const double* __restrict__ Wt, int cpad, int ncols, int M,
                                                       const double* __restrict__ lam, const double* __restrict__ w,
                                                       int n_spikes, double* __restrict__ corr) {
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < ncols; c += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int s = 0; s < n_spikes; ++s) {
      const double x = lam[s] < -1.0 ? -1.0 : (lam[s] > 1.0 ? 1.0 : lam[s]);
      const double th = acos(x);
      double t = 0.0;
      for (int m = 0; m < M; ++m)
        t = fma(cos(static_cast<double>(m) * th), Wt[static_cast<int64_t>(m) * cpad + c], t);
      acc += w[s] * t;
    }
    corr[c] = acc;
  }
}

// hist[row][b] = (F[b] - F[b+1]) / pi + spikes; F rows are n_bins+1 wide.
__global__ __launch_bounds__(kBlock) void k_recon_bins(const double* __restrict__ F, int64_t n_rows, int n_bins,
                                                       const int32_t* __restrict__ sbin,
                                                       const double* __restrict__ sw, int n_spikes,
                                                       double* __restrict__ hist) {
  const int64_t total = n_rows * n_bins;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t r = idx / n_bins;
    const int b = static_cast<int>(idx % n_bins);
    const double* f = F + r * (n_bins + 1);
    double h = (f[b] - f[b + 1]) / M_PI;
    for (int s = 0; s < n_spikes; ++s)
      if (sbin[s] == b) h += sw[s];
    hist[idx] = h;
  }
}

}  // namespace
}  // namespace nd

extern "C" nd_status nd_reconstruct(const double* mu, int64_t n_rows, int32_t n_moments, uint32_t kernel,
                                    const double* spike_lambda, const double* spike_weight, int32_t n_spikes,
                                    int32_t n_bins, double lo, double hi, double* hist, int32_t n_points,
                                    double* rho, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(mu != nullptr, "nd_reconstruct: mu is NULL");
  ND_REQUIRE(n_rows >= 1 && n_moments >= 1, "nd_reconstruct: n_rows=%lld n_moments=%d", (long long)n_rows,
             n_moments);
  const bool spikes_in = (kernel & ND_SPIKES_IN_MOMENTS) != 0;
  kernel &= ~ND_SPIKES_IN_MOMENTS;
  ND_REQUIRE(kernel == ND_KERNEL_NONE || kernel == ND_KERNEL_JACKSON, "nd_reconstruct: unknown kernel %u", kernel);
  ND_REQUIRE(hist || rho, "nd_reconstruct: hist and rho are both NULL");
  ND_REQUIRE(!hist || (n_bins >= 1 && n_bins <= 4096), "nd_reconstruct: n_bins=%d not in [1, 4096]", n_bins);
  ND_REQUIRE(!rho || (n_points >= 1 && n_points <= 4096), "nd_reconstruct: n_points=%d not in [1, 4096]",
             n_points);
  ND_REQUIRE(!hist || (lo >= -1.0 && hi <= 1.0 && lo < hi), "nd_reconstruct: need -1 <= lo < hi <= 1");
  ND_REQUIRE(n_spikes >= 0 && n_spikes <= 1024, "nd_reconstruct: n_spikes=%d not in [0, 1024]", n_spikes);
  ND_REQUIRE(n_spikes == 0 || (spike_lambda && spike_weight), "nd_reconstruct: spike arrays are NULL");
  hipStream_t st = as_stream(stream);
  const int nb = hist ? n_bins : 0, np = rho ? n_points : 0;
  const int n_edges = nb ? nb + 1 : 0;
  const int ncols = n_edges + np;
  // spike bins on the host with the same edge formula as the kernels
  std::vector<int32_t> sbin;
  std::vector<double> sw;
  for (int s = 0; s < n_spikes && nb; ++s) {
    const double lam = spike_lambda[s];
    const double e_lo = lo, e_hi = lo + (hi - lo) * static_cast<double>(nb) / static_cast<double>(nb);
    if (lam < e_lo || lam > e_hi) continue;
    int b = nb - 1;
    for (int t = 0; t < nb; ++t) {
      const double e_next = lo + (hi - lo) * static_cast<double>(t + 1) / static_cast<double>(nb);
      if (lam < e_next) {
        b = t;
        break;
      }
    }
    sbin.push_back(b);
    sw.push_back(spike_weight[s]);
  }
  const int cpad = static_cast<int>(ceil_div(ncols, kTC)) * kTC;
  const int Mp = static_cast<int>(ceil_div(n_moments, kKC)) * kKC;
  // bins fused into the product when all edge columns fit one tile
  const bool fused = nb > 0 && n_edges <= kTC;
  double *W = nullptr, *F = nullptr, *sw_d = nullptr, *corr = nullptr, *all_d = nullptr;
  int32_t* sb_d = nullptr;
  nd_status s = dalloc_t(&W, static_cast<size_t>(Mp) * cpad);
  if (s == ND_OK && spikes_in && n_spikes > 0) {
    s = dalloc_t(&corr, static_cast<size_t>(ncols));
    if (s == ND_OK) s = dalloc_t(&all_d, static_cast<size_t>(2 * n_spikes));
    if (s == ND_OK &&
        (hipMemcpyAsync(all_d, spike_lambda, n_spikes * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
         hipMemcpyAsync(all_d + n_spikes, spike_weight, n_spikes * 8, hipMemcpyHostToDevice, st) != hipSuccess)) {
      set_error("nd_reconstruct: copy of spikes failed");
      s = ND_EDEVICE;
    }
  }
  if (s == ND_OK && nb && !fused) s = dalloc_t(&F, static_cast<size_t>(n_rows) * n_edges);
  if (s == ND_OK && !sbin.empty()) s = dalloc_t(&sb_d, sbin.size());
  if (s == ND_OK && !sw.empty()) s = dalloc_t(&sw_d, sw.size());
  if (s == ND_OK && !sbin.empty()) {
    if (hipMemcpyAsync(sb_d, sbin.data(), sbin.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(sw_d, sw.data(), sw.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
      set_error("nd_reconstruct: copy of spikes failed");
      s = ND_EDEVICE;
    }
  }
  if (s == ND_OK) {
    hipLaunchKernelGGL(k_recon_table, dim3(grid_for(static_cast<int64_t>(Mp) * cpad, kBlock)), dim3(kBlock), 0, st,
                       n_moments, Mp, static_cast<int>(kernel), nb, lo, hi, np, cpad, W);
    if (corr)
      hipLaunchKernelGGL(k_spike_corr, dim3(grid_for(ncols, kBlock)), dim3(kBlock), 0, st, W, cpad, ncols, n_moments,
                         all_d, all_d + n_spikes, n_spikes, corr);
    const dim3 grid(static_cast<unsigned>(ceil_div(n_rows, kTR)));
    bool ok = hipGetLastError() == hipSuccess;
    // product over the table columns [c_begin, c_end), tile by tile, into o
    // (row stride ld; its column 0 is table column c_begin)
    auto apply = [&](int c_begin, int c_end, double* o, int ld) {
      for (int c0 = c_begin; c0 < c_end && ok; c0 += kTC) {
        const int cc = c_end - c0 < kTC ? c_end - c0 : kTC;
        hipLaunchKernelGGL(k_recon_gemm, grid, dim3(kBlock), 0, st, mu, n_rows, n_moments, W, cpad, c0, cc, corr,
                           o + (c0 - c_begin), ld, nullptr, nullptr, nullptr, 0);
        ok = hipGetLastError() == hipSuccess;
      }
    };
    if (fused) {
      hipLaunchKernelGGL(k_recon_gemm, grid, dim3(kBlock), 0, st, mu, n_rows, n_moments, W, cpad, 0, n_edges, corr,
                         nullptr, 0, hist, sb_d, sw_d, static_cast<int>(sbin.size()));
      ok = ok && hipGetLastError() == hipSuccess;
    } else if (nb) {
      apply(0, n_edges, F, n_edges);
      if (ok) {
        hipLaunchKernelGGL(k_recon_bins, dim3(grid_for(n_rows * nb, kBlock)), dim3(kBlock), 0, st, F, n_rows, nb,
                           sb_d, sw_d, static_cast<int>(sbin.size()), hist);
        ok = hipGetLastError() == hipSuccess;
      }
    }
    if (np) apply(n_edges, n_edges + np, rho, np);
    if (!ok) {
      set_error("nd_reconstruct: launch failed");
      s = ND_EDEVICE;
    }
  }
  // temporaries are released once the stream has consumed them
  if (hipStreamSynchronize(st) != hipSuccess && s == ND_OK) {
    set_error("nd_reconstruct: stream failure");
    s = ND_EDEVICE;
  }
  dfree(W);
  dfree(F);
  dfree(sb_d);
  dfree(sw_d);
  dfree(corr);
  dfree(all_d);
  return s;
}
