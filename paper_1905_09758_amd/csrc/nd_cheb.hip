// KPM moments on the device (Sec. 3.1): probe block, optional twin projection
// (Sec. 3.4), the Chebyshev three-term recurrence (eq. cheb_3term) applied to
// the whole block with one sparse product per step, and the fused moment
// reductions of the trace estimator (eq. probe_trace) and the diagonal
// estimator (eq. probe_diag).
//
// The recurrence runs on X_m = D^{-1/2} Y_m, Y_m = T_m(H) Z, which satisfies
//   X_0 = D^{-1/2} Z,  X_1 = D^{-1} A X_0,  X_{m+1} = 2 D^{-1} A X_m - X_{m-1},
// since D^{-1/2} H D^{1/2} = D^{-1} A.  The gathered operand of each step is
// then a plain row of X (no per-neighbour scale), and Y_m = D^{1/2} X_m is
// formed in fp64 only inside the moment reductions.
//
// Layout: probe blocks are node-major [N][kp] (kp = padded probe count, a
// power of two), so the row of X gathered for one neighbour is one contiguous
// kp*sizeof(T)-byte load spread over L = kp*sizeof(T)/16 lanes of 16 bytes.
// X_{m+1} overwrites X_{m-1} in place: row i reads only its own old row.
#include <cmath>
#include <cstdlib>

#include "nd_common.h"

namespace nd {
namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
  using type = float4;
};
template <>
struct VecOf<double> {
  using type = double2;
};

template <typename T>
__device__ inline void load16(const T* p, T (&v)[16 / sizeof(T)]) {
  using V = typename VecOf<T>::type;
  const V x = *reinterpret_cast<const V*>(p);
  if constexpr (sizeof(T) == 4) {
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    v[0] = x.x; v[1] = x.y;
  }
}

template <typename T>
__device__ inline void store16(T* p, const T (&v)[16 / sizeof(T)]) {
  using V = typename VecOf<T>::type;
  V x;
  if constexpr (sizeof(T) == 4) {
    x.x = v[0]; x.y = v[1]; x.z = v[2]; x.w = v[3];
  } else {
    x.x = v[0]; x.y = v[1];
  }
  *reinterpret_cast<V*>(p) = x;
}

// Neumaier-compensated accumulation.
__device__ inline void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

struct StepArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  const int32_t* rows;
  int64_t n;
  int n_bins;
  int64_t bin_row_start[kMaxBins + 1];
  int64_t bin_item_start[kMaxBins + 1];
  int64_t n_items;
  const int64_t* split_chunk_ptr;
  const int32_t* chunk_owner;
  int32_t* split_counter;
  int64_t chunk_nnz;
  void* chunk_part;
  const void* xg;   // X_m, gathered
  void* xio;        // X_{m-1} in, X_{m+1} out
  const void* z;    // probe block (projected when filtering)
  int first;        // step m == 1: X_1 = D^{-1} A X_0
  int kp;           // padded probes per row
  int k_batch;      // real probes in this block
  double inv_k;     // 1 / (total probe count over all blocks)
  int m;            // moment index written by this launch
  double* partial;  // [gridDim.x + n_split][kp] per-probe partial sums for moment m
  int64_t n_split;  // rows split into chunks (one partial slot each)
  double* ldos;     // [n][ld] or null
  double* ldos_sq;  // [n][ld] or null
  int64_t ld;       // leading dimension of ldos / cv_g (= number of moments)
  int accumulate;   // add to ldos instead of overwriting (later probe blocks)
  const float* cv_g;
};

// Per-row epilogue: given Y_m(i, probes of this lane) in fp64, form the
// estimator terms v_ij = z_ij y_ij (+ g_im (1 - z_ij^2) with a control
// variate), add them to this lane's per-probe accumulators, and write the
// row's LDOS entry.  Called by every lane of the wavefront; `own` selects the
// lanes that hold a row's values.
// With `direct` set (rows split over several wavefronts) the terms go to that
// row's own partial slot instead, so the summation order does not depend on
// which wavefront finished the row.
template <typename T, int L>
__device__ inline void emit_moments(const StepArgs& a, bool own, int64_t r, const double (&y)[16 / sizeof(T)],
                                    int q, double (&acc_s)[16 / sizeof(T)], double (&acc_c)[16 / sizeof(T)],
                                    double* direct = nullptr) {
  constexpr int PPL = 16 / sizeof(T);
  double s1 = 0.0, s2 = 0.0;
  if (own) {
    T z[PPL];
    load16<T>(reinterpret_cast<const T*>(a.z) + r * a.kp + q * PPL, z);
    const double g = a.cv_g ? static_cast<double>(a.cv_g[r * a.ld + a.m]) : 0.0;
#pragma unroll
    for (int c = 0; c < PPL; ++c) {
      const double zc = static_cast<double>(z[c]);
      double v = zc * y[c];
      if (a.cv_g) v += g * (1.0 - zc * zc);
      if (q * PPL + c >= a.k_batch) v = 0.0;
      if (direct)
        direct[q * PPL + c] = v;
      else
        neumaier(acc_s[c], acc_c[c], v);
      s1 += v;
      s2 += v * v;
    }
  }
  if (a.ldos) {
#pragma unroll
    for (int off = 1; off < L; off <<= 1) {
      s1 += __shfl_xor(s1, off, kWave);
      s2 += __shfl_xor(s2, off, kWave);
    }
    if (own && q == 0) {
      double* p = a.ldos + r * a.ld + a.m;
      *p = (a.accumulate ? *p : 0.0) + s1 * a.inv_k;
      if (a.ldos_sq) {
        double* p2 = a.ldos_sq + r * a.ld + a.m;
        *p2 = (a.accumulate ? *p2 : 0.0) + s2 * a.inv_k;
      }
    }
  }
}

// Finish row r: X_{m+1} = 2/d * acc - X_{m-1} (or acc/d on the first step),
// store it in place, then the moment epilogue on Y = sqrt(d) X.
template <typename T, int L, typename A>
__device__ inline void finish_row(const StepArgs& a, bool own, int64_t r, int64_t d, const A (&acc)[16 / sizeof(T)],
                                  int q, double (&acc_s)[16 / sizeof(T)], double (&acc_c)[16 / sizeof(T)],
                                  double* direct = nullptr) {
  constexpr int PPL = 16 / sizeof(T);
  double y[PPL];
  if (own) {
    T* xo = reinterpret_cast<T*>(a.xio) + r * a.kp + q * PPL;
    T xn[PPL];
    const A invd = A(1) / static_cast<A>(d);
    if (a.first) {
#pragma unroll
      for (int c = 0; c < PPL; ++c) xn[c] = static_cast<T>(acc[c] * invd);
    } else {
      T xp[PPL];
      load16<T>(xo, xp);
      const A two_invd = A(2) * invd;
#pragma unroll
      for (int c = 0; c < PPL; ++c) xn[c] = static_cast<T>(two_invd * acc[c] - static_cast<A>(xp[c]));
    }
    store16<T>(xo, xn);
    const double sd = sqrt(static_cast<double>(d));
#pragma unroll
    for (int c = 0; c < PPL; ++c) y[c] = static_cast<double>(xn[c]) * sd;
  } else {
#pragma unroll
    for (int c = 0; c < PPL; ++c) y[c] = 0.0;
  }
  emit_moments<T, L>(a, own, r, y, q, acc_s, acc_c, direct);
}

// Rows of a sub-wave bin: P nonzero slots per row, 64/(P*L) rows per wavefront.
template <typename T, int L, int P>
__device__ inline void rows_item(const StepArgs& a, int bin, int64_t local_item, int lane,
                                 double (&acc_s)[16 / sizeof(T)], double (&acc_c)[16 / sizeof(T)]) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int G = P * L;
  constexpr int RPW = kWave / G;
  const int grp = lane / G, sub = (lane % G) / L, q = lane % L;
  const int64_t ridx = a.bin_row_start[bin] + local_item * RPW + grp;
  const bool active = ridx < a.bin_row_start[bin + 1];
  const int64_t r = active ? a.rows[ridx] : 0;
  const int64_t e0 = active ? a.row_ptr[r] : 0, e1 = active ? a.row_ptr[r + 1] : 0;
  T acc[PPL];
#pragma unroll
  for (int c = 0; c < PPL; ++c) acc[c] = T(0);
  const T* xg = reinterpret_cast<const T*>(a.xg);
  for (int64_t e = e0 + sub; e < e1; e += P) {
    const int64_t j = a.col[e];
    T v[PPL];
    load16<T>(xg + j * a.kp + q * PPL, v);
#pragma unroll
    for (int c = 0; c < PPL; ++c) acc[c] += v[c];
  }
#pragma unroll
  for (int off = L; off < G; off <<= 1)
#pragma unroll
    for (int c = 0; c < PPL; ++c) acc[c] += __shfl_xor(acc[c], off, kWave);
  finish_row<T, L, T>(a, active && sub == 0, r, e1 - e0, acc, q, acc_s, acc_c);
}

// One chunk of a long row; the wavefront that completes the row's last chunk
// sums the chunk partials in chunk order and finishes the row.
template <typename T, int L>
__device__ inline void chunk_item(const StepArgs& a, int64_t c, int lane, double (&acc_s)[16 / sizeof(T)],
                                  double (&acc_c)[16 / sizeof(T)]) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int P = kWave / L;
  const int sub = lane / L, q = lane % L;
  const int64_t s = a.chunk_owner[c];
  const int64_t r = a.rows[a.bin_row_start[a.n_bins] + s];
  const int64_t c0 = a.split_chunk_ptr[s], nch = a.split_chunk_ptr[s + 1] - c0;
  const int64_t rb = a.row_ptr[r], re = a.row_ptr[r + 1];
  const int64_t e0 = rb + (c - c0) * a.chunk_nnz;
  const int64_t e1 = e0 + a.chunk_nnz < re ? e0 + a.chunk_nnz : re;
  T acc[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) acc[k] = T(0);
  const T* xg = reinterpret_cast<const T*>(a.xg);
  for (int64_t e = e0 + sub; e < e1; e += P) {
    const int64_t j = a.col[e];
    T v[PPL];
    load16<T>(xg + j * a.kp + q * PPL, v);
#pragma unroll
    for (int k = 0; k < PPL; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int off = L; off < kWave; off <<= 1)
#pragma unroll
    for (int k = 0; k < PPL; ++k) acc[k] += __shfl_xor(acc[k], off, kWave);
  // chunk partials are kept in fp64: a long row sums many of them
  double* part = reinterpret_cast<double*>(a.chunk_part);
  if (sub == 0) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) part[c * a.kp + q * PPL + k] = static_cast<double>(acc[k]);
  }
  __threadfence();
  int old = 0;
  if (lane == 0) old = atomicAdd(&a.split_counter[s], 1);
  old = __shfl(old, 0, kWave);
  if (old == nch - 1) {
    __threadfence();
    double tot[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) tot[k] = 0.0;
    if (sub == 0) {
      for (int64_t cc = 0; cc < nch; ++cc) {
#pragma unroll
        for (int k = 0; k < PPL; ++k) tot[k] += part[(c0 + cc) * a.kp + q * PPL + k];
      }
    }
    finish_row<T, L, double>(a, sub == 0, r, re - rb, tot, q, acc_s, acc_c,
                             a.partial + (static_cast<int64_t>(gridDim.x) + s) * a.kp);
    if (lane == 0) a.split_counter[s] = 0;
  }
}

// Block-level fixed-order reduction of the per-lane probe accumulators into
// partial[blockIdx.x][0..kp).
template <typename T, int L>
__device__ inline void block_partials(const StepArgs& a, const double (&acc_s)[16 / sizeof(T)],
                                      const double (&acc_c)[16 / sizeof(T)]) {
  constexpr int PPL = 16 / sizeof(T);
  __shared__ double red[kBlock][PPL];
#pragma unroll
  for (int c = 0; c < PPL; ++c) red[threadIdx.x][c] = acc_s[c] + acc_c[c];
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < a.kp) {
    const int j = threadIdx.x, qq = j / PPL, cc = j % PPL;
    double s = 0.0, comp = 0.0;
    for (int t = qq; t < kBlock; t += L) neumaier(s, comp, red[t][cc]);
    a.partial[static_cast<int64_t>(blockIdx.x) * a.kp + j] = s + comp;
  }
}

template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_cheb_step(StepArgs a) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int PMAX = kWave / L;
  const int lane = threadIdx.x & (kWave - 1);
  double acc_s[PPL], acc_c[PPL];
#pragma unroll
  for (int c = 0; c < PPL; ++c) acc_s[c] = acc_c[c] = 0.0;
  const int64_t n_waves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  for (int64_t it = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave; it < a.n_items;
       it += n_waves) {
    int b = 0;
    while (b < a.n_bins && it >= a.bin_item_start[b + 1]) ++b;
    if (b < a.n_bins) {
      const int64_t li = it - a.bin_item_start[b];
      switch (b) {
#define ND_BIN(B) \
  case B:         \
    if constexpr ((1 << B) <= PMAX) rows_item<T, L, (1 << B)>(a, b, li, lane, acc_s, acc_c); \
    break;
        ND_BIN(0)
        ND_BIN(1)
        ND_BIN(2)
        ND_BIN(3)
        ND_BIN(4)
        ND_BIN(5)
        ND_BIN(6)
#undef ND_BIN
        default:
          break;
      }
    } else {
      chunk_item<T, L>(a, it - a.bin_item_start[a.n_bins], lane, acc_s, acc_c);
    }
  }
  block_partials<T, L>(a, acc_s, acc_c);
}

// Moment 0: Y_0 = Z.  Rows in natural order, 64/L rows per wavefront.
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_moment0(StepArgs a) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int RPW = kWave / L;
  const int lane = threadIdx.x & (kWave - 1), q = lane % L, grp = lane / L;
  double acc_s[PPL], acc_c[PPL];
#pragma unroll
  for (int c = 0; c < PPL; ++c) acc_s[c] = acc_c[c] = 0.0;
  const int64_t n_waves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  const int64_t items = ceil_div(a.n, RPW);
  for (int64_t it = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave; it < items;
       it += n_waves) {
    const int64_t r = it * RPW + grp;
    const bool own = r < a.n;
    double y[PPL];
    if (own) {
      T z[PPL];
      load16<T>(reinterpret_cast<const T*>(a.z) + r * a.kp + q * PPL, z);
#pragma unroll
      for (int c = 0; c < PPL; ++c) y[c] = static_cast<double>(z[c]);
    } else {
#pragma unroll
      for (int c = 0; c < PPL; ++c) y[c] = 0.0;
    }
    emit_moments<T, L>(a, own, own ? r : 0, y, q, acc_s, acc_c);
  }
  // no split rows at moment 0: clear their slots
  double* sp = a.partial + static_cast<int64_t>(gridDim.x) * a.kp;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < a.n_split * a.kp;
       t += static_cast<int64_t>(gridDim.x) * kBlock)
    sp[t] = 0.0;
  block_partials<T, L>(a, acc_s, acc_c);
}

}  // namespace
}  // namespace nd

// ====================================================================== probes
namespace nd {
namespace {

// Probe entry (j, i): see nd_make_probes in nd.h for the definition.
__device__ inline float probe_value(uint64_t seed, int64_t j, int64_t i, bool gaussian) {
  const uint64_t key = splitmix64(seed, static_cast<uint64_t>(j) + 1);
  if (!gaussian) {
    const uint64_t b = splitmix64(key, static_cast<uint64_t>(i) + 1);
    return (b >> 63) ? -1.0f : 1.0f;
  }
  const uint64_t b1 = splitmix64(key, 2 * static_cast<uint64_t>(i) + 1);
  const uint64_t b2 = splitmix64(key, 2 * static_cast<uint64_t>(i) + 2);
  const double u1 = (static_cast<double>(b1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = static_cast<double>(b2 >> 11) * 0x1.0p-53;
  const double g = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  return static_cast<float>(g);
}

// Z[i][ld] (probes j0 .. j0+k_batch-1 in columns 0..k_batch-1, zeros beyond)
// and, when X0 is given, X0 = D^{-1/2} Z.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probes(int64_t n, int ld, int k_batch, int64_t j0, uint64_t seed,
                                                   int gaussian, const int64_t* __restrict__ row_ptr,
                                                   T* __restrict__ Z, T* __restrict__ X0) {
  const int64_t total = n * ld;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = idx / ld;
    const int j = static_cast<int>(idx - i * ld);
    const T z = j < k_batch ? static_cast<T>(probe_value(seed, j0 + j, i, gaussian != 0)) : T(0);
    Z[idx] = z;
    if (X0) {
      const double d = static_cast<double>(row_ptr[i + 1] - row_ptr[i]);
      X0[idx] = static_cast<T>(static_cast<double>(z) / sqrt(d));
    }
  }
}

// Twin projection Z <- P P^T Z (Sec. 3.4): each class's rows replaced by the
// class mean (fp64 sum in member order).  Members of a class share their
// neighbourhood and hence their degree.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_project(const int64_t* __restrict__ class_ptr,
                                                    const int32_t* __restrict__ members, int64_t n_classes,
                                                    int ld, int k_batch, const int64_t* __restrict__ row_ptr,
                                                    T* __restrict__ Z, T* __restrict__ X0) {
  const int64_t total = n_classes * k_batch;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t c = idx / k_batch;
    const int j = static_cast<int>(idx - c * k_batch);
    const int64_t p0 = class_ptr[c], p1 = class_ptr[c + 1];
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) s += static_cast<double>(Z[static_cast<int64_t>(members[p]) * ld + j]);
    const T mean = static_cast<T>(s / static_cast<double>(p1 - p0));
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t i = members[p];
      Z[i * ld + j] = mean;
      if (X0) {
        const double d = static_cast<double>(row_ptr[i + 1] - row_ptr[i]);
        X0[i * ld + j] = static_cast<T>(static_cast<double>(mean) / sqrt(d));
      }
    }
  }
}

// mu_pp[j0+j][m] = (1/N) sum over partial slots, for the `count` steps
// m0 .. m0+count-1 stored in consecutive partial blocks of `slots` slots.
// Thread t sums slots t/kp, t/kp + S, ... (S = 256/kp stripes) with
// compensation; the stripes are then combined in order: a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partial, int64_t slots,
                                                            int kp, int k_batch, int m0, double inv_n,
                                                            double* __restrict__ mu_pp, int M, int64_t j0) {
  __shared__ double red[kBlock];
  const int s = blockIdx.x;
  const double* p = partial + static_cast<int64_t>(s) * slots * kp;
  const int stripes = kBlock / kp;
  const int j = threadIdx.x % kp, st = threadIdx.x / kp;
  double sum = 0.0, comp = 0.0;
  if (st < stripes)
    for (int64_t b = st; b < slots; b += stripes) neumaier(sum, comp, p[b * kp + j]);
  red[threadIdx.x] = sum + comp;
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < k_batch) {
    double t = 0.0, c = 0.0;
    for (int q = 0; q < stripes; ++q) neumaier(t, c, red[q * kp + threadIdx.x]);
    mu_pp[(j0 + threadIdx.x) * M + m0 + s] = (t + c) * inv_n;
  }
}

// mu[m] = (1/k) sum_j mu_pp[j][m] + w T_m(0).
__global__ __launch_bounds__(kBlock) void k_mu_final(const double* __restrict__ mu_pp, int k, int M, double w,
                                                     double* __restrict__ mu) {
  for (int m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock) {
    double sum = 0.0, comp = 0.0;
    for (int j = 0; j < k; ++j) neumaier(sum, comp, mu_pp[static_cast<int64_t>(j) * M + m]);
    const double t0 = (m & 1) ? 0.0 : ((m & 2) ? -1.0 : 1.0);
    mu[m] = (sum + comp) / static_cast<double>(k) + w * t0;
  }
}

// ldos[i][m] += (1 - 1/|C|) T_m(0) for every member i of a class C.
__global__ __launch_bounds__(kBlock) void k_ldos_spike(const int64_t* __restrict__ class_ptr,
                                                       const int32_t* __restrict__ members, int64_t n_classes,
                                                       int64_t n_members, int M, double* __restrict__ ldos) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n_members;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    int64_t lo = 0, hi = n_classes;  // class c with class_ptr[c] <= p < class_ptr[c+1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (class_ptr[mid] <= p) lo = mid; else hi = mid;
    }
    const double w = 1.0 - 1.0 / static_cast<double>(class_ptr[lo + 1] - class_ptr[lo]);
    double* row = ldos + static_cast<int64_t>(members[p]) * M;
    for (int m = 0; m < M; m += 2) row[m] += (m & 2) ? -w : w;
  }
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

int step_grid_cap() {
  static int cap = [] {
    const char* e = std::getenv("ND_STEP_GRID");
    int v = e ? std::atoi(e) : 0;
    return v > 0 ? v : 2048;
  }();
  return cap;
}

struct MomentJob {
  const nd_motifs* motifs = nullptr;
  int k = 0, M = 0;
  uint64_t seed = 0;
  bool gaussian = false;
  const float* cv_g = nullptr;
  double* ldos = nullptr;
  double* ldos_sq = nullptr;
  double* mu = nullptr;
  double* mu_pp = nullptr;
  double spike_w = 0.0;  // added to mu as w T_m(0)
};

template <typename T, int L>
nd_status launch_step_kernels(const StepArgs& base, int grid, bool moment0, hipStream_t st) {
  if (moment0)
    hipLaunchKernelGGL((k_moment0<T, L>), dim3(grid), dim3(kBlock), 0, st, base);
  else
    hipLaunchKernelGGL((k_cheb_step<T, L>), dim3(grid), dim3(kBlock), 0, st, base);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

template <typename T>
nd_status launch_step(int L, const StepArgs& a, int grid, bool moment0, hipStream_t st) {
  switch (L) {
    case 1: return launch_step_kernels<T, 1>(a, grid, moment0, st);
    case 2: return launch_step_kernels<T, 2>(a, grid, moment0, st);
    case 4: return launch_step_kernels<T, 4>(a, grid, moment0, st);
    case 8: return launch_step_kernels<T, 8>(a, grid, moment0, st);
    case 16: return launch_step_kernels<T, 16>(a, grid, moment0, st);
    case 32:
      if constexpr (sizeof(T) == 8) return launch_step_kernels<T, 32>(a, grid, moment0, st);
      break;
    default: break;
  }
  set_error("internal: unsupported lane count %d", L);
  return ND_EUNSUPPORTED;
}

template <typename T>
nd_status run_moments(nd_graph* g, const MomentJob& job, hipStream_t st) {
  constexpr int PPL = 16 / sizeof(T);
  const int64_t N = g->n;
  const int M = job.M;
  double* mu_pp = job.mu_pp;
  if (!mu_pp) {
    ND_CHECK(g->ws_misc.ensure(static_cast<size_t>(job.k) * M * sizeof(double)));
    mu_pp = g->ws_misc.as<double>();
  }
  for (int j0 = 0; j0 < job.k; j0 += 64) {
    const int kb = job.k - j0 < 64 ? job.k - j0 : 64;
    const int kp = pow2_at_least(kb < PPL ? PPL : kb);
    const int L = kp * static_cast<int>(sizeof(T)) / 16;
    Schedule* sc = nullptr;
    ND_CHECK(get_schedule(g, L, st, &sc));
    const size_t blk = static_cast<size_t>(N) * kp * sizeof(T);
    ND_CHECK(g->ws_state.ensure(3 * blk));
    ND_CHECK(g->ws_chunk.ensure(static_cast<size_t>(sc->n_chunks > 0 ? sc->n_chunks : 1) * kp * sizeof(double)));
    T* Z = g->ws_state.as<T>();
    T* A = Z + static_cast<int64_t>(N) * kp;
    T* B = A + static_cast<int64_t>(N) * kp;
    const int grid = grid_for(sc->n_items > 0 ? sc->n_items : 1, kWavesPerBlock, step_grid_cap());
    const int64_t slots = static_cast<int64_t>(grid) + sc->n_split;
    const int64_t per_step = slots * kp;
    int R = static_cast<int>((int64_t(64) << 20) / (per_step * 8));
    if (R < 1) R = 1;
    if (R > M) R = M;
    ND_CHECK(g->ws_partial.ensure(static_cast<size_t>(R) * per_step * sizeof(double)));
    double* partial = g->ws_partial.as<double>();

    hipLaunchKernelGGL(k_probes<T>, dim3(grid_for(N * kp, kBlock)), dim3(kBlock), 0, st, N, kp, kb,
                       static_cast<int64_t>(j0), job.seed, job.gaussian ? 1 : 0, g->row_ptr, Z, A);
    ND_LAUNCH_CHECK();
    if (job.motifs && job.motifs->n_classes > 0) {
      hipLaunchKernelGGL(k_project<T>, dim3(grid_for(job.motifs->n_classes * kb, kBlock)), dim3(kBlock), 0, st,
                         job.motifs->class_ptr, job.motifs->members, job.motifs->n_classes, kp, kb, g->row_ptr,
                         Z, A);
      ND_LAUNCH_CHECK();
    }
    StepArgs a{};
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.rows = sc->rows;
    a.n = N;
    a.n_bins = sc->n_bins;
    for (int b = 0; b <= kMaxBins; ++b) {
      a.bin_row_start[b] = sc->bin_row_start[b];
      a.bin_item_start[b] = sc->bin_item_start[b];
    }
    a.n_items = sc->n_items;
    a.split_chunk_ptr = sc->split_chunk_ptr;
    a.chunk_owner = sc->chunk_owner;
    a.split_counter = sc->split_counter;
    a.chunk_nnz = sc->chunk_nnz;
    a.n_split = sc->n_split;
    a.chunk_part = g->ws_chunk.p;
    a.z = Z;
    a.kp = kp;
    a.k_batch = kb;
    a.inv_k = 1.0 / static_cast<double>(job.k);
    a.ldos = job.ldos;
    a.ldos_sq = job.ldos_sq;
    a.ld = M;
    a.accumulate = j0 > 0 ? 1 : 0;
    a.cv_g = job.cv_g;
    for (int m = 0; m < M; ++m) {
      a.m = m;
      a.partial = partial + static_cast<int64_t>(m % R) * per_step;
      if (m == 0) {
        ND_CHECK(launch_step<T>(L, a, grid, true, st));
      } else {
        a.first = (m == 1) ? 1 : 0;
        a.xg = (m & 1) ? A : B;
        a.xio = (m & 1) ? B : A;
        ND_CHECK(launch_step<T>(L, a, grid, false, st));
      }
      if ((m + 1) % R == 0 || m == M - 1) {
        const int m0 = m - (m % R);
        hipLaunchKernelGGL(k_reduce_partials, dim3(m - m0 + 1), dim3(kBlock), 0, st, partial, slots, kp, kb, m0,
                           1.0 / static_cast<double>(N), mu_pp, M, static_cast<int64_t>(j0));
        ND_LAUNCH_CHECK();
      }
    }
  }
  if (job.mu) {
    hipLaunchKernelGGL(k_mu_final, dim3(grid_for(M, kBlock)), dim3(kBlock), 0, st, mu_pp, job.k, M, job.spike_w,
                       job.mu);
    ND_LAUNCH_CHECK();
  }
  if (job.ldos && job.motifs && job.motifs->n_classes > 0) {
    hipLaunchKernelGGL(k_ldos_spike, dim3(grid_for(job.motifs->n_members, kBlock)), dim3(kBlock), 0, st,
                       job.motifs->class_ptr, job.motifs->members, job.motifs->n_classes, job.motifs->n_members, M,
                       job.ldos);
    ND_LAUNCH_CHECK();
  }
  return ND_OK;
}

nd_status check_common(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                       uint32_t flags, const char* who) {
  ND_REQUIRE(g != nullptr, "%s: graph is NULL", who);
  ND_REQUIRE(g->n > 0, "%s: the graph has no edges (no node survives)", who);
  ND_REQUIRE(n_probes >= 1, "%s: n_probes=%d must be >= 1", who, n_probes);
  ND_REQUIRE(n_moments >= 1, "%s: n_moments=%d must be >= 1", who, n_moments);
  ND_REQUIRE((flags & ~(ND_PROBE_GAUSSIAN | ND_STATE_FP64)) == 0, "%s: unknown flags 0x%x", who, flags);
  ND_REQUIRE(motifs == nullptr || motifs->n == g->n, "%s: motifs belong to another graph", who);
  int dev = -1;
  ND_HIP(hipGetDevice(&dev));
  ND_REQUIRE(dev == g->device, "%s: graph lives on device %d, current device is %d", who, g->device, dev);
  return ND_OK;
}

}  // namespace
}  // namespace nd

// ====================================================================== C ABI
extern "C" {

nd_status nd_make_probes(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, uint64_t seed,
                         uint32_t flags, void* Z, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, 1, flags, "nd_make_probes"));
  ND_REQUIRE(Z != nullptr, "nd_make_probes: Z is NULL");
  hipStream_t st = nd::as_stream(stream);
  const bool gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  const int64_t total = g->n * n_probes;
  if (flags & ND_STATE_FP64) {
    hipLaunchKernelGGL(nd::k_probes<double>, dim3(nd::grid_for(total, nd::kBlock)), dim3(nd::kBlock), 0, st, g->n,
                       n_probes, n_probes, int64_t(0), seed, gaussian ? 1 : 0, g->row_ptr,
                       static_cast<double*>(Z), static_cast<double*>(nullptr));
  } else {
    hipLaunchKernelGGL(nd::k_probes<float>, dim3(nd::grid_for(total, nd::kBlock)), dim3(nd::kBlock), 0, st, g->n,
                       n_probes, n_probes, int64_t(0), seed, gaussian ? 1 : 0, g->row_ptr,
                       static_cast<float*>(Z), static_cast<float*>(nullptr));
  }
  ND_LAUNCH_CHECK();
  if (motifs && motifs->n_classes > 0) {
    const int64_t t2 = motifs->n_classes * n_probes;
    if (flags & ND_STATE_FP64)
      hipLaunchKernelGGL(nd::k_project<double>, dim3(nd::grid_for(t2, nd::kBlock)), dim3(nd::kBlock), 0, st,
                         motifs->class_ptr, motifs->members, motifs->n_classes, n_probes, n_probes, g->row_ptr,
                         static_cast<double*>(Z), static_cast<double*>(nullptr));
    else
      hipLaunchKernelGGL(nd::k_project<float>, dim3(nd::grid_for(t2, nd::kBlock)), dim3(nd::kBlock), 0, st,
                         motifs->class_ptr, motifs->members, motifs->n_classes, n_probes, n_probes, g->row_ptr,
                         static_cast<float*>(Z), static_cast<float*>(nullptr));
    ND_LAUNCH_CHECK();
  }
  return ND_OK;
}

nd_status nd_cheb_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                          uint64_t probe_seed, uint32_t flags, double* mu, double* mu_pp, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, n_moments, flags, "nd_cheb_moments"));
  ND_REQUIRE(mu != nullptr || mu_pp != nullptr, "nd_cheb_moments: mu and mu_pp are both NULL");
  nd::MomentJob job;
  job.motifs = motifs;
  job.k = n_probes;
  job.M = n_moments;
  job.seed = probe_seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.mu = mu;
  job.mu_pp = mu_pp;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (flags & ND_STATE_FP64) return nd::run_moments<double>(gm, job, nd::as_stream(stream));
  return nd::run_moments<float>(gm, job, nd::as_stream(stream));
}

nd_status nd_ldos_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                          uint64_t probe_seed, uint32_t flags, const float* cv_g, double* ldos, double* ldos_sq,
                          double* mu, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, n_moments, flags, "nd_ldos_moments"));
  ND_REQUIRE(ldos != nullptr, "nd_ldos_moments: ldos is NULL");
  nd::MomentJob job;
  job.motifs = motifs;
  job.k = n_probes;
  job.M = n_moments;
  job.seed = probe_seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.cv_g = cv_g;
  job.ldos = ldos;
  job.ldos_sq = ldos_sq;
  job.mu = mu;
  job.spike_w = motifs ? motifs->spike_weight : 0.0;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (flags & ND_STATE_FP64) return nd::run_moments<double>(gm, job, nd::as_stream(stream));
  return nd::run_moments<float>(gm, job, nd::as_stream(stream));
}

}  // extern "C"
