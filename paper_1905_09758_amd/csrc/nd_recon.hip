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

// W[e][m] for the bin integral table (n_edges rows) followed by the density
// table (n_points rows).
__global__ __launch_bounds__(kBlock) void k_recon_table(int M, int kernel, int n_bins, double lo, double hi,
                                                        int n_points, double* __restrict__ W) {
  const int n_edges = n_bins > 0 ? n_bins + 1 : 0;
  const int64_t total = static_cast<int64_t>(n_edges + n_points) * M;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int r = static_cast<int>(idx / M), m = static_cast<int>(idx % M);
    const double g = kernel ? jackson_g(m, M) : 1.0;
    double w;
    if (r < n_edges) {
      double x = lo + (hi - lo) * static_cast<double>(r) / static_cast<double>(n_bins);
      x = x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x);
      const double th = acos(x);
      w = (m == 0) ? th : 2.0 * sin(static_cast<double>(m) * th) / static_cast<double>(m);
    } else {
      const int k = r - n_edges;
      const double th = M_PI * (static_cast<double>(k) + 0.5) / static_cast<double>(n_points);
      w = ((m == 0) ? 1.0 : 2.0 * cos(static_cast<double>(m) * th)) / (M_PI * sin(th));
    }
    W[idx] = g * w;
  }
}

// out[row][c] = sum_m mu[row][m] W[c][m] for c < ncols (fixed order in m).
// A block handles kRows rows; their moment rows are staged in LDS.
constexpr int kRows = 8;
constexpr int kMaxStage = 1024;  // moments staged per pass

__global__ __launch_bounds__(kBlock) void k_recon_apply(const double* __restrict__ mu, int64_t n_rows, int M,
                                                        const double* __restrict__ W, int ncols,
                                                        double* __restrict__ out, int ld_out,
                                                        const double* __restrict__ corr) {
  __shared__ double smu[kRows][kMaxStage];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRows;
  const int work = kRows * ncols;
  // each thread owns up to ceil(work / kBlock) (row, col) outputs
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int per = (work + kBlock - 1) / kBlock;  // <= 4 enforced by the host
  for (int m0 = 0; m0 < M; m0 += kMaxStage) {
    const int mm = M - m0 < kMaxStage ? M - m0 : kMaxStage;
    __syncthreads();
    for (int t = threadIdx.x; t < kRows * mm; t += kBlock) {
      const int rr = t / mm, m = t % mm;
      smu[rr][m] = (r0 + rr < n_rows) ? mu[(r0 + rr) * M + m0 + m] : 0.0;
    }
    __syncthreads();
    for (int u = 0; u < per; ++u) {
      const int w = threadIdx.x + u * kBlock;
      if (w >= work) break;
      const int rr = w / ncols, c = w % ncols;
      const double* wr = W + static_cast<int64_t>(c) * M + m0;
      double s = acc[u];
      for (int m = 0; m < mm; ++m) s = fma(smu[rr][m], wr[m], s);
      acc[u] = s;
    }
  }
  for (int u = 0; u < per; ++u) {
    const int w = threadIdx.x + u * kBlock;
    if (w >= work) break;
    const int rr = w / ncols, c = w % ncols;
    if (r0 + rr < n_rows) out[(r0 + rr) * ld_out + c] = corr ? acc[u] - corr[c] : acc[u];
  }
}

// corr[c] = sum_s w_s sum_m T_m(lambda_s) W[c][m]: the part of column c that
// the point masses contribute when the moments include them.
__global__ __launch_bounds__(kBlock) void k_spike_corr(const double* __restrict__ W, int ncols, int M,
                                                       const double* __restrict__ lam, const double* __restrict__ w,
                                                       int n_spikes, double* __restrict__ corr) {
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < ncols; c += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int s = 0; s < n_spikes; ++s) {
      const double x = lam[s] < -1.0 ? -1.0 : (lam[s] > 1.0 ? 1.0 : lam[s]);
      const double th = acos(x);
      double t = 0.0;
      for (int m = 0; m < M; ++m) t = fma(cos(static_cast<double>(m) * th), W[static_cast<int64_t>(c) * M + m], t);
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
  ND_REQUIRE(n_spikes >= 0 && n_spikes <= 64, "nd_reconstruct: n_spikes=%d not in [0, 64]", n_spikes);
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
  double *W = nullptr, *F = nullptr, *sw_d = nullptr, *corr = nullptr, *all_d = nullptr;
  int32_t* sb_d = nullptr;
  nd_status s = dalloc_t(&W, static_cast<size_t>(ncols) * n_moments);
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
  if (s == ND_OK && nb) s = dalloc_t(&F, static_cast<size_t>(n_rows) * n_edges);
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
    hipLaunchKernelGGL(k_recon_table, dim3(grid_for(static_cast<int64_t>(ncols) * n_moments, kBlock)), dim3(kBlock),
                       0, st, n_moments, static_cast<int>(kernel), nb, lo, hi, np, W);
    if (corr)
      hipLaunchKernelGGL(k_spike_corr, dim3(grid_for(ncols, kBlock)), dim3(kBlock), 0, st, W, ncols, n_moments, all_d,
                         all_d + n_spikes, n_spikes, corr);
    // products: bins then points, each in column groups that fit a block
    // products: bin-edge columns then point columns, in groups that fit a block
    auto apply = [&](const double* Wc, const double* cc_corr, int cols, double* out) -> bool {
      const int per_grp = (4 * kBlock) / kRows;
      for (int c0 = 0; c0 < cols; c0 += per_grp) {
        const int cc = cols - c0 < per_grp ? cols - c0 : per_grp;
        hipLaunchKernelGGL(k_recon_apply, dim3(static_cast<unsigned>(ceil_div(n_rows, kRows))), dim3(kBlock), 0, st,
                           mu, n_rows, n_moments, Wc + static_cast<int64_t>(c0) * n_moments, cc, out + c0, cols,
                           cc_corr ? cc_corr + c0 : nullptr);
        if (hipGetLastError() != hipSuccess) return false;
      }
      return true;
    };
    bool ok = true;
    if (nb) ok = apply(W, corr, n_edges, F);
    if (ok && np) ok = apply(W + static_cast<int64_t>(n_edges) * n_moments, corr ? corr + n_edges : nullptr, np, rho);
    if (!ok) {
      set_error("nd_reconstruct: launch failed");
      s = ND_EDEVICE;
    }
    if (s == ND_OK && nb) {
      hipLaunchKernelGGL(k_recon_bins, dim3(grid_for(n_rows * nb, kBlock)), dim3(kBlock), 0, st, F, n_rows, nb, sb_d,
                         sw_d, static_cast<int>(sbin.size()), hist);
      if (hipGetLastError() != hipSuccess) {
        set_error("nd_reconstruct: launch failed");
        s = ND_EDEVICE;
      }
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
