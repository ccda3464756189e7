// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <vector>

#include "nd.h"

namespace nd {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per block in every kernel of the library
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

void set_error(const char* fmt, ...);
void clear_error();

#define ND_HIP(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      nd::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return ND_EDEVICE;                                                                  \
    }                                                                                     \
  } while (0)

#define ND_CHECK(expr)                   \
  do {                                   \
    nd_status s_ = (expr);               \
    if (s_ != ND_OK) return s_;          \
  } while (0)

#define ND_REQUIRE(cond, ...)            \
  do {                                   \
    if (!(cond)) {                       \
      nd::set_error(__VA_ARGS__);        \
      return ND_EINVAL;                  \
    }                                    \
  } while (0)

#define ND_LAUNCH_CHECK()                                                                     \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) {                                                                   \
      nd::set_error("kernel launch: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
      return ND_EDEVICE;                                                                      \
    }                                                                                         \
  } while (0)

// Device allocation with an optional process-wide cap (environment variable
// ND_ALLOC_LIMIT_BYTES) so that out-of-memory paths can be exercised.
nd_status dalloc(void** p, size_t bytes);
void dfree(void* p);

template <typename T>
nd_status dalloc_t(T** p, size_t count) {
  return dalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

// Temporaries of one call, freed together (hipFree waits for the device).
struct Tmp {
  std::vector<void*> ptrs;
  template <typename T>
  nd_status get(T** p, size_t count) {
    ND_CHECK(dalloc_t(p, count));
    ptrs.push_back(*p);
    return ND_OK;
  }
  ~Tmp() {
    for (void* p : ptrs) dfree(p);
  }
};

// A device buffer that only grows; freed with its owner.
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
  nd_status ensure(size_t need) {
    if (need <= bytes) return ND_OK;
    dfree(p);
    p = nullptr;
    bytes = 0;
    size_t want = need + need / 8;
    nd_status s = dalloc(&p, want);
    if (s != ND_OK) return s;
    bytes = want;
    return ND_OK;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
  ~Scratch() { dfree(p); }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int grid_for(int64_t work_items, int64_t per_block, int64_t cap = 65536) {
  int64_t g = ceil_div(work_items, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// ---------------------------------------------------------------- primitives
// Exclusive prefix sum of n int64 values (in may alias out); returns the total
// through *total_dev (device int64) when non-null.
nd_status exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_dev,
                             hipStream_t st);
// Same over int32 input, int64 output.
nd_status exclusive_scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total_dev,
                                 hipStream_t st);

// Stable LSD radix sort of n 64-bit keys on bits [0, nbits), with an optional
// 32-bit payload.  keys/vals are sorted in place; alt_* are scratch buffers of
// the same size (may be swapped internally; results always end in keys/vals).
nd_status radix_sort_u64(uint64_t* keys, uint64_t* alt_keys, uint32_t* vals, uint32_t* alt_vals,
                         int64_t n, int nbits, hipStream_t st);

// ---------------------------------------------------------------- schedule
// The sparse product runs on an internal numbering of the rows by descending
// degree (ties by ascending id): long rows first, then rows of decreasing
// length, so that rows of one length class are a contiguous range and the
// most-gathered rows (the high-degree ones) share cache lines.
struct Internal {
  int32_t* perm = nullptr;     // [n] internal row -> compact node id
  int32_t* inv = nullptr;      // [n] compact node id -> internal row
  int64_t* row_ptr = nullptr;  // [n+1]
  int32_t* col = nullptr;      // [nnz] internal column ids
  ~Internal();
};

// Row-to-wavefront mapping for a gathered row of L 16-byte lanes.  A row of
// degree d gets P = 2^b nonzero slots, b = clamp(ceil(log2(ceil(d/S))), 0,
// log2(64/L)) with S nonzeros per slot (the gathers one lane keeps in
// flight), so one wavefront covers 64/(P*L) rows; rows longer than one
// chunk (kChunkIters iterations of a full wavefront) are split into chunks
// whose fp64 partial sums a second kernel combines in a fixed order.
constexpr int kChunkIters = 32;
constexpr int kMaxBins = 8;

struct Schedule {
  int L = 0;
  int slot_nnz = 8;                    // nonzeros per slot: P = ceil(d / slot_nnz) (pow2)
  int n_bins = 0;                      // non-empty bins, in internal row order
  int bin_log2p[kMaxBins] = {0};
  int64_t bin_row_start[kMaxBins + 1] = {0};   // internal row ranges
  int64_t bin_item_start[kMaxBins + 1] = {0};  // wavefront items after the chunks
  int64_t chunk_nnz = 0;
  int64_t n_split = 0, n_chunks = 0;   // split rows are internal rows [0, n_split)
  int64_t n_items = 0;                 // n_chunks + bin items
  int64_t* split_chunk_ptr = nullptr;  // [n_split+1]
  int32_t* chunk_owner = nullptr;      // [n_chunks]
  ~Schedule();
};

}  // namespace nd

// ---------------------------------------------------------------- handles
struct nd_graph {
  int device = 0;
  int64_t n = 0, nnz = 0, max_deg = 0;
  int64_t* row_ptr = nullptr;  // [n+1]
  int32_t* col = nullptr;      // [nnz]
  int32_t* old_id = nullptr;   // [n]
  float* dinv_sqrt = nullptr;  // [n]
  std::unique_ptr<nd::Internal> internal;              // built on first use
  std::map<int, std::unique_ptr<nd::Schedule>> sched;  // keyed by L
  nd::Scratch ws_state, ws_partial, ws_chunk, ws_misc, ws_zcls, ws_stage, ws_zbits;  // moment workspaces
  // ND_TIME_STEPS: HIP-event time of the sparse-product step launches of the
  // last moment call (the launches of moment 1 .. M-1 of every probe block)
  double step_ms = 0.0;
  int64_t step_launches = 0;
  ~nd_graph();
};

struct nd_motifs {
  int device = 0;
  int64_t n = 0;            // nodes of the graph it belongs to
  int64_t n_classes = 0, n_members = 0;
  int64_t* class_ptr = nullptr;  // [n_classes+1]
  int32_t* members = nullptr;    // [n_members]
  double* class_lambda = nullptr;  // [n_classes] eigenvalue removed by each class
  int32_t* class_paired = nullptr; // [n_classes] 1: the class holds +-class_lambda, half each
  // distinct removed eigenvalues (ascending) and their DOS mass sum (|C|-1)/n
  std::vector<double> spike_lambda, spike_weight;
  double* spikes_d = nullptr;    // device copy: lambdas then weights
  ~nd_motifs();
};

namespace nd {
// out[i * ld + m] += scale (1 - 1/|C|) T_m(lambda_C), m < n_cols, for every
// member i of a motif class C: the part of T_m(H)_ii that the class's removed
// eigenvectors carry (Sec. 3.4).  A paired class (eigenvalues +-lambda_C,
// half each) adds (1 - 1/|C|) (T_m(lambda) + T_m(-lambda)) / 2, i.e.
// T_m(lambda) at even m and nothing at odd m.  T_m by the three-term
// recurrence in fp64.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_motif_diag(const int64_t* __restrict__ class_ptr,
                                                       const int32_t* __restrict__ members,
                                                       const double* __restrict__ class_lambda,
                                                       const int32_t* __restrict__ class_paired, int64_t n_classes,
                                                       int64_t n_members, int64_t ld, int n_cols, double scale,
                                                       T* __restrict__ out) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n_members;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    int64_t lo = 0, hi = n_classes;  // class c with class_ptr[c] <= p < class_ptr[c+1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (class_ptr[mid] <= p) lo = mid; else hi = mid;
    }
    const double w = scale * (1.0 - 1.0 / static_cast<double>(class_ptr[lo + 1] - class_ptr[lo]));
    const double x = class_lambda[lo];
    const bool pair = class_paired[lo] != 0;
    T* row = out + static_cast<int64_t>(members[p]) * ld;
    double t0 = 1.0, t1 = x;
    for (int m = 0; m < n_cols; ++m) {
      if (!pair || (m & 1) == 0) row[m] = static_cast<T>(static_cast<double>(row[m]) + w * t0);
      const double t2 = 2.0 * x * t1 - t0;
      t0 = t1;
      t1 = t2;
    }
  }
}

nd_status get_internal(nd_graph* g, hipStream_t st, Internal** out);
nd_status get_schedule(nd_graph* g, int L, hipStream_t st, Schedule** out);
// Lanczos coefficients of every probe (Sec. 3.2), on the sparse step kernels:
// alpha, beta device [n_probes][n_steps], norm2 device [n_probes] (|z|^2/N,
// or 1 for unit probes), steps device int32 [n_probes].  With unit_nodes
// (device int32 [n_probes]) probe j is the unit vector of that node.
nd_status lanczos_coefficients(nd_graph* g, const nd_motifs* motifs, const int32_t* unit_nodes, int32_t n_probes,
                               int32_t n_steps, uint64_t seed, uint32_t flags, double* alpha, double* beta,
                               double* norm2, int32_t* steps, hipStream_t st);
nd_status check_moment_args(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                            uint32_t flags, const char* who);
}

// ---------------------------------------------------------------- device helpers
namespace nd {
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Output n (1-based) of the SplitMix64 stream seeded with s.
__host__ __device__ inline uint64_t splitmix64(uint64_t s, uint64_t n) { return mix64(s + n * kGamma); }
}  // namespace nd
