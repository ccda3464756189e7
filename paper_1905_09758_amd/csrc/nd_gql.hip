// Gauss quadrature and Lanczos, GQL (Sec. 3.2): per probe, the K-node Gauss
// rule of the measure sum_i (q_i^T z)^2 delta(lambda - lambda_i), from the
// Lanczos coefficients computed on the sparse step kernels.  The rule's nodes
// are the eigenvalues of the Lanczos tridiagonal Gamma_K, its weights the
// squared first components of the eigenvectors (Golub-Welsch), scaled by
// |z|^2 / N; averaged over probes they estimate the DOS, and their Chebyshev
// moments equal the KPM estimates of the same probes up to degree 2K - 1.
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

// Eigenvalues of the symmetric tridiagonal (diagonal a[0..n), subdiagonal
// b[0..n-1), destroyed) by implicit QR steps with the Wilkinson shift and
// deflation (Golub & Van Loan, Matrix Computations, Sec. 8.3), accumulating
// only the first row q0 of the eigenvector matrix.  On return a holds the
// eigenvalues (unordered) and q0 the first components.  Returns false if an
// iteration cap of 60 n steps is reached.
__device__ bool tridiag_rule(double* a, double* b, double* q0, int n) {
  for (int i = 0; i < n; ++i) q0[i] = (i == 0) ? 1.0 : 0.0;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iters = 0;
  while (hi > 0) {
    if (fabs(b[hi - 1]) <= eps * (fabs(a[hi - 1]) + fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    // unreduced block [lo, hi]
    int lo = hi - 1;
    while (lo > 0 && fabs(b[lo - 1]) > eps * (fabs(a[lo - 1]) + fabs(a[lo]))) --lo;
    if (lo > 0) b[lo - 1] = 0.0;
    if (++iters > 60 * n) return false;
    const double dlt = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double mu = a[hi] - bb * bb / (dlt + copysign(hypot(dlt, bb), dlt == 0.0 ? 1.0 : dlt));
    // chase the bulge with rotations G = [c s; -s c] on (p, p+1)
    double x = a[lo] - mu, z = b[lo], bulge = 0.0;
    for (int p = lo; p < hi; ++p) {
      const int q = p + 1;
      const double r = hypot(x, z);
      const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? -z / r : 0.0;
      if (p > lo) b[p - 1] = c * b[p - 1] - s * bulge;
      const double ap = a[p], aq = a[q], bp = b[p];
      a[p] = c * c * ap - 2.0 * c * s * bp + s * s * aq;
      a[q] = s * s * ap + 2.0 * c * s * bp + c * c * aq;
      b[p] = c * s * (ap - aq) + (c * c - s * s) * bp;
      if (q < hi) {
        bulge = -s * b[q];
        b[q] = c * b[q];
        x = b[p];
        z = bulge;
      }
      const double u = q0[p], v = q0[q];
      q0[p] = c * u - s * v;
      q0[q] = s * u + c * v;
    }
  }
  return true;
}

// One thread per probe: nodes[j][i], weights[j][i] (i < steps[j]; zeros beyond).
__global__ void k_gql_rule(int k, int K, const double* __restrict__ alpha, const double* __restrict__ beta,
                           const double* __restrict__ norm2, const int32_t* __restrict__ steps,
                           double* __restrict__ sub, double* __restrict__ nodes, double* __restrict__ weights,
                           int32_t* __restrict__ failed) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const int n = steps[j];
  double* a = nodes + static_cast<int64_t>(j) * K;
  double* w = weights + static_cast<int64_t>(j) * K;
  double* b = sub + static_cast<int64_t>(j) * K;
  for (int i = 0; i < K; ++i) {
    a[i] = i < n ? alpha[static_cast<int64_t>(j) * K + i] : 0.0;
    b[i] = i + 1 < n ? beta[static_cast<int64_t>(j) * K + i] : 0.0;
    w[i] = 0.0;
  }
  if (n <= 0) return;
  if (!tridiag_rule(a, b, w, n)) atomicAdd(failed, 1);
  for (int i = 0; i < n; ++i) w[i] = w[i] * w[i] * norm2[j];
}

// mu[m] = (1/k) sum_j sum_i w_ji T_m(tau_ji), fixed order.
__global__ __launch_bounds__(kBlock) void k_gql_moments(int k, int K, const double* __restrict__ nodes,
                                                        const double* __restrict__ weights, int M,
                                                        double* __restrict__ mu) {
  for (int m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock) {
    double s = 0.0;
    for (int64_t t = 0; t < static_cast<int64_t>(k) * K; ++t) {
      const double w = weights[t];
      if (w == 0.0) continue;
      const double x = nodes[t] < -1.0 ? -1.0 : (nodes[t] > 1.0 ? 1.0 : nodes[t]);
      s += w * cos(static_cast<double>(m) * acos(x));
    }
    mu[m] = s / static_cast<double>(k);
  }
}

// hist[b] = (1/k) sum of the weights of the nodes in bin b (bins of [lo, hi]
// half-open except the last), fixed order.  Nodes are clamped to [-1, 1],
// the interval that holds the spectrum of H (fp32 Lanczos can place the
// node of the eigenvalue 1 a rounding error beyond it).
__global__ __launch_bounds__(kBlock) void k_gql_hist(int k, int K, const double* __restrict__ nodes,
                                                     const double* __restrict__ weights, int nb, double lo, double hi,
                                                     double* __restrict__ hist) {
  for (int bin = blockIdx.x * kBlock + threadIdx.x; bin < nb; bin += gridDim.x * kBlock) {
    const double e0 = lo + (hi - lo) * static_cast<double>(bin) / static_cast<double>(nb);
    const double e1 = lo + (hi - lo) * static_cast<double>(bin + 1) / static_cast<double>(nb);
    double s = 0.0;
    for (int64_t t = 0; t < static_cast<int64_t>(k) * K; ++t) {
      const double w = weights[t];
      if (w == 0.0) continue;
      const double x = nodes[t] < -1.0 ? -1.0 : (nodes[t] > 1.0 ? 1.0 : nodes[t]);
      if (x >= e0 && (x < e1 || (bin == nb - 1 && x <= e1))) s += w;
    }
    hist[bin] = s / static_cast<double>(k);
  }
}

// Lanczos coefficients, then one Gauss rule per probe (unit probes when
// unit_nodes is given).
nd_status gql_impl(const nd_graph* g, const nd_motifs* motifs, const int32_t* unit_nodes, int32_t n_probes,
                   int32_t n_steps, uint64_t probe_seed, uint32_t flags, double* nodes, double* weights,
                   int32_t* steps, double* alpha, double* beta, hipStream_t st) {
  const size_t kk = static_cast<size_t>(n_probes) * n_steps;
  Tmp t;
  double *al = alpha, *be = beta, *norm2, *sub;
  int32_t *stp = steps, *failed;
  if (!al) ND_CHECK(t.get(&al, kk));
  if (!be) ND_CHECK(t.get(&be, kk));
  if (!stp) ND_CHECK(t.get(&stp, static_cast<size_t>(n_probes)));
  ND_CHECK(t.get(&norm2, static_cast<size_t>(n_probes)));
  ND_CHECK(t.get(&sub, kk));
  ND_CHECK(t.get(&failed, 1));
  ND_HIP(hipMemsetAsync(al, 0, kk * 8, st));
  ND_HIP(hipMemsetAsync(be, 0, kk * 8, st));
  ND_HIP(hipMemsetAsync(failed, 0, 4, st));
  ND_CHECK(lanczos_coefficients(const_cast<nd_graph*>(g), motifs, unit_nodes, n_probes, n_steps, probe_seed, flags, al,
                                be, norm2, stp, st));
  hipLaunchKernelGGL(k_gql_rule, dim3(static_cast<unsigned>(ceil_div(n_probes, 64))), dim3(64), 0, st, n_probes,
                     n_steps, al, be, norm2, stp, sub, nodes, weights, failed);
  ND_LAUNCH_CHECK();
  int32_t hf = 0;
  ND_HIP(hipMemcpyAsync(&hf, failed, 4, hipMemcpyDeviceToHost, st));
  ND_HIP(hipStreamSynchronize(st));
  ND_REQUIRE(hf == 0, "nd_gql: the tridiagonal eigensolver did not converge for %d probes", hf);
  return ND_OK;
}

}  // namespace
}  // namespace nd

extern "C" {

nd_status nd_gql(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_steps, uint64_t probe_seed,
                 uint32_t flags, double* nodes, double* weights, int32_t* steps, double* alpha, double* beta,
                 void* stream) {
  using namespace nd;
  clear_error();
  ND_CHECK(check_moment_args(g, motifs, n_probes, n_steps, flags, "nd_gql"));
  ND_REQUIRE((flags & ND_MOMENT_DOUBLING) == 0, "nd_gql: ND_MOMENT_DOUBLING does not apply");
  ND_REQUIRE(nodes != nullptr && weights != nullptr, "nd_gql: nodes/weights are NULL");
  ND_REQUIRE(n_steps <= 4096, "nd_gql: n_steps=%d exceeds 4096", n_steps);
  return gql_impl(g, motifs, nullptr, n_probes, n_steps, probe_seed, flags, nodes, weights, steps, alpha, beta,
                  as_stream(stream));
}

nd_status nd_gql_pdos(const nd_graph* g, const int32_t* vertices, int32_t n_vertices, int32_t n_steps,
                      uint32_t flags, double* nodes, double* weights, int32_t* steps, void* stream) {
  using namespace nd;
  clear_error();
  ND_CHECK(check_moment_args(g, nullptr, n_vertices, n_steps, flags, "nd_gql_pdos"));
  ND_REQUIRE((flags & ~(ND_STATE_FP64 | ND_TIME_STEPS)) == 0, "nd_gql_pdos: flags 0x%x (only ND_STATE_FP64, "
             "ND_TIME_STEPS apply)", flags);
  ND_REQUIRE(vertices != nullptr && nodes != nullptr && weights != nullptr, "nd_gql_pdos: NULL argument");
  ND_REQUIRE(n_steps <= 4096, "nd_gql_pdos: n_steps=%d exceeds 4096", n_steps);
  hipStream_t st = as_stream(stream);
  {
    std::vector<int32_t> h(static_cast<size_t>(n_vertices));
    ND_HIP(hipMemcpyAsync(h.data(), vertices, h.size() * 4, hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
    for (int32_t v : h) ND_REQUIRE(v >= 0 && v < g->n, "nd_gql_pdos: node id %d not in [0, %lld)", v, (long long)g->n);
  }
  return gql_impl(g, nullptr, vertices, n_vertices, n_steps, 0, flags, nodes, weights, steps, nullptr, nullptr, st);
}

nd_status nd_gql_density(const double* nodes, const double* weights, int32_t n_probes, int32_t n_steps,
                         int32_t n_moments, double* mu, int32_t n_bins, double lo, double hi, double* hist,
                         void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(nodes != nullptr && weights != nullptr, "nd_gql_density: nodes/weights are NULL");
  ND_REQUIRE(n_probes >= 1 && n_steps >= 1, "nd_gql_density: n_probes=%d n_steps=%d", n_probes, n_steps);
  ND_REQUIRE(mu || hist, "nd_gql_density: mu and hist are both NULL");
  ND_REQUIRE(!mu || n_moments >= 1, "nd_gql_density: n_moments=%d", n_moments);
  ND_REQUIRE(!hist || (n_bins >= 1 && n_bins <= 4096 && lo < hi), "nd_gql_density: bad bins");
  hipStream_t st = as_stream(stream);
  if (mu) {
    hipLaunchKernelGGL(k_gql_moments, dim3(grid_for(n_moments, kBlock)), dim3(kBlock), 0, st, n_probes, n_steps,
                       nodes, weights, n_moments, mu);
    ND_LAUNCH_CHECK();
  }
  if (hist) {
    hipLaunchKernelGGL(k_gql_hist, dim3(grid_for(n_bins, kBlock)), dim3(kBlock), 0, st, n_probes, n_steps, nodes,
                       weights, n_bins, lo, hi, hist);
    ND_LAUNCH_CHECK();
  }
  return ND_OK;
}

}  // extern "C"
