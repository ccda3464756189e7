// Graph construction on the device (the graph and operator of Sec. 2.1):
// symmetrise, drop self-loops, deduplicate, drop isolated nodes, renumber by
// ascending input id, CSR with ascending columns, fp32(1/sqrt(fp64 degree)).
// Also the error/allocation helpers and the row schedule of the sparse product.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>

#include "nd_common.h"

namespace nd {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

// ------------------------------------------------------------------ allocation
static size_t alloc_limit() {
  static size_t lim = [] {
    const char* e = std::getenv("ND_ALLOC_LIMIT_BYTES");
    return e ? static_cast<size_t>(std::strtoull(e, nullptr, 10)) : static_cast<size_t>(0);
  }();
  return lim;
}

// Device memory is cached per device: freed blocks stay mapped in a pool and
// are handed out again to requests of their size class (graphs rebuilt in a
// loop, workspaces regrown, temporaries of every call), so the steady state
// makes no hipMalloc/hipFree calls.  A cached block is reused only after the
// device has drained (hipDeviceSynchronize), so work still queued on any
// stream never sees its memory change hands.  When hipMalloc fails, the cache
// is released and the allocation retried.  The pool lives until the process
// ends; ND_POOL_BYTES caps the cached total (default 32 GiB).
namespace {

struct Pool {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> free_blocks;  // device -> (size class, block)
  std::unordered_map<void*, std::pair<int, size_t>> owned;  // block -> (device, size class)
  size_t cached = 0;
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: no HIP calls after the runtime shuts down
  return *p;
}

size_t pool_cap() {
  static size_t cap = [] {
    const char* e = std::getenv("ND_POOL_BYTES");
    return e ? static_cast<size_t>(std::strtoull(e, nullptr, 10)) : (size_t(32) << 30);
  }();
  return cap;
}

// Size classes: powers of two up to 1 MiB, then multiples of 2 MiB.
size_t size_class(size_t bytes) {
  if (bytes <= (size_t(1) << 20)) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t g = size_t(2) << 20;
  return (bytes + g - 1) / g * g;
}

void release_cached(Pool& P) {
  for (auto& dev : P.free_blocks) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev.first);
    for (auto& kv : dev.second) {
      P.owned.erase(kv.second);
      (void)hipFree(kv.second);
    }
    dev.second.clear();
    (void)hipSetDevice(cur);
  }
  P.cached = 0;
}

}  // namespace

nd_status dalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  const size_t lim = alloc_limit();
  if (lim && bytes > lim) {
    set_error("allocation of %zu bytes exceeds ND_ALLOC_LIMIT_BYTES=%zu", bytes, lim);
    return ND_ENOMEM;
  }
  const size_t cls = size_class(bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipGetDevice failed");
    return ND_EDEVICE;
  }
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto& fl = P.free_blocks[dev];
    // small classes match exactly; large ones take a block up to twice the size
    auto it = fl.lower_bound(cls);
    if (it != fl.end() && (it->first == cls || (cls > (size_t(1) << 20) && it->first <= 2 * cls))) {
      void* q = it->second;
      P.cached -= it->first;
      fl.erase(it);
      if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        P.owned.erase(q);
        (void)hipFree(q);
        set_error("hipDeviceSynchronize failed before reusing device memory");
        return ND_EDEVICE;
      }
      *p = q;
      return ND_OK;
    }
  }
  hipError_t e = hipMalloc(p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.cached > 0) {
      (void)hipDeviceSynchronize();
      release_cached(P);
      e = hipMalloc(p, cls);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      set_error("hipMalloc(%zu bytes): %s", cls, hipGetErrorString(e));
      return ND_ENOMEM;
    }
  }
  std::lock_guard<std::mutex> lk(P.mu);
  P.owned[*p] = {dev, cls};
  return ND_OK;
}

void dfree(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.owned.find(p);
  if (it == P.owned.end()) {
    (void)hipFree(p);
    return;
  }
  const int dev = it->second.first;
  const size_t cls = it->second.second;
  if (P.cached + cls > pool_cap()) {
    P.owned.erase(it);
    (void)hipFree(p);
    return;
  }
  P.free_blocks[dev].emplace(cls, p);
  P.cached += cls;
}

namespace {

// ------------------------------------------------------------------ build kernels
__global__ __launch_bounds__(kBlock) void k_emit_keys(const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ dst, int64_t m,
                                                      int64_t n_nodes, int bits,
                                                      uint64_t* __restrict__ keys,
                                                      unsigned long long* __restrict__ counters) {
  const uint64_t sent = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1ull);
  unsigned long long bad = 0, loops = 0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < m;
       e += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t u = src[e], v = dst[e];
    uint64_t k0 = sent, k1 = sent;
    if (u < 0 || v < 0 || u >= n_nodes || v >= n_nodes) {
      bad++;
    } else if (u == v) {
      loops++;
    } else {
      k0 = (static_cast<uint64_t>(u) << bits) | static_cast<uint64_t>(v);
      k1 = (static_cast<uint64_t>(v) << bits) | static_cast<uint64_t>(u);
    }
    keys[2 * e] = k0;
    keys[2 * e + 1] = k1;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    bad += __shfl_xor(bad, off, kWave);
    loops += __shfl_xor(loops, off, kWave);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (bad) atomicAdd(&counters[0], bad);
    if (loops) atomicAdd(&counters[1], loops);
  }
}

__global__ __launch_bounds__(kBlock) void k_dedup_flags(const uint64_t* __restrict__ keys, int64_t n,
                                                        int32_t* __restrict__ flag) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_compact_mark(const uint64_t* __restrict__ keys, int64_t n,
                                                         const int32_t* __restrict__ flag,
                                                         const int64_t* __restrict__ pos, int bits,
                                                         uint64_t* __restrict__ ukeys,
                                                         int32_t* __restrict__ present) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (flag[i]) {
      const uint64_t k = keys[i];
      ukeys[pos[i]] = k;
      present[k >> bits] = 1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_old_id(const int32_t* __restrict__ present,
                                                   const int64_t* __restrict__ new_id, int64_t n_nodes,
                                                   int32_t* __restrict__ old_id) {
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; u < n_nodes;
       u += static_cast<int64_t>(gridDim.x) * kBlock)
    if (present[u]) old_id[new_id[u]] = static_cast<int32_t>(u);
}

__global__ __launch_bounds__(kBlock) void k_rows_cols(const uint64_t* __restrict__ ukeys, int64_t nnz,
                                                      int bits, const int64_t* __restrict__ new_id,
                                                      int64_t* __restrict__ row_ptr,
                                                      int32_t* __restrict__ col, int64_t n) {
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < nnz;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const uint64_t k = ukeys[p];
    const uint64_t u = k >> bits;
    col[p] = static_cast<int32_t>(new_id[k & mask]);
    if (p == 0 || (ukeys[p - 1] >> bits) != u) row_ptr[new_id[u]] = p;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) row_ptr[n] = nnz;
}

__global__ __launch_bounds__(kBlock) void k_dinv(const int64_t* __restrict__ row_ptr, int64_t n,
                                                 float* __restrict__ dinv,
                                                 unsigned long long* __restrict__ max_deg) {
  unsigned long long mx = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t d = row_ptr[i + 1] - row_ptr[i];
    dinv[i] = static_cast<float>(1.0 / sqrt(static_cast<double>(d)));
    if (static_cast<unsigned long long>(d) > mx) mx = static_cast<unsigned long long>(d);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(mx, off, kWave);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && mx) atomicMax(max_deg, mx);
}

int bit_length(int64_t x) {
  int b = 0;
  while (x > 0) {
    b++;
    x >>= 1;
  }
  return b;
}


nd_status build_impl(int64_t n_nodes, int64_t m, const int32_t* src_in, const int32_t* dst_in,
                     uint32_t flags, hipStream_t st, nd_graph* g) {
  Tmp t;
  const int32_t* src = src_in;
  const int32_t* dst = dst_in;
  if (!(flags & ND_INPUT_DEVICE) && m > 0) {
    int32_t *s2, *d2;
    ND_CHECK(t.get(&s2, static_cast<size_t>(m)));
    ND_CHECK(t.get(&d2, static_cast<size_t>(m)));
    ND_HIP(hipMemcpyAsync(s2, src_in, static_cast<size_t>(m) * 4, hipMemcpyHostToDevice, st));
    ND_HIP(hipMemcpyAsync(d2, dst_in, static_cast<size_t>(m) * 4, hipMemcpyHostToDevice, st));
    src = s2;
    dst = d2;
  }
  const int bits = bit_length(n_nodes);
  const int64_t nk = 2 * m;
  uint64_t *keys = nullptr, *alt = nullptr;
  unsigned long long* counters = nullptr;
  ND_CHECK(t.get(&counters, 4));
  ND_HIP(hipMemsetAsync(counters, 0, 4 * sizeof(unsigned long long), st));
  int64_t nnz = 0;
  if (m > 0) {
    ND_CHECK(t.get(&keys, static_cast<size_t>(nk)));
    hipLaunchKernelGGL(k_emit_keys, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, st, src, dst, m, n_nodes,
                       bits, keys, counters);
    ND_LAUNCH_CHECK();
    unsigned long long hc[2];
    ND_HIP(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
    if (hc[0]) {
      set_error("nd_build_csr: %llu edges have an endpoint outside [0, %lld)", hc[0], (long long)n_nodes);
      return ND_EINVAL;
    }
    const int64_t n_valid = nk - 2 * static_cast<int64_t>(hc[1]);
    ND_CHECK(t.get(&alt, static_cast<size_t>(nk)));
    ND_CHECK(radix_sort_u64(keys, alt, nullptr, nullptr, nk, 2 * bits, st));
    if (n_valid > 0) {
      int32_t* flag;
      int64_t *pos, *tot;
      ND_CHECK(t.get(&flag, static_cast<size_t>(n_valid)));
      ND_CHECK(t.get(&pos, static_cast<size_t>(n_valid)));
      ND_CHECK(t.get(&tot, 1));
      hipLaunchKernelGGL(k_dedup_flags, dim3(grid_for(n_valid, kBlock)), dim3(kBlock), 0, st, keys, n_valid,
                         flag);
      ND_LAUNCH_CHECK();
      ND_CHECK(exclusive_scan_i32_i64(flag, pos, n_valid, tot, st));
      ND_HIP(hipMemcpyAsync(&nnz, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      int32_t* present;
      ND_CHECK(t.get(&present, static_cast<size_t>(n_nodes)));
      ND_HIP(hipMemsetAsync(present, 0, static_cast<size_t>(n_nodes) * 4, st));
      hipLaunchKernelGGL(k_compact_mark, dim3(grid_for(n_valid, kBlock)), dim3(kBlock), 0, st, keys,
                         n_valid, flag, pos, bits, alt, present);
      ND_LAUNCH_CHECK();
      int64_t* new_id;
      ND_CHECK(t.get(&new_id, static_cast<size_t>(n_nodes)));
      ND_CHECK(exclusive_scan_i32_i64(present, new_id, n_nodes, tot, st));
      int64_t n = 0;
      ND_HIP(hipMemcpyAsync(&n, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      ND_HIP(hipStreamSynchronize(st));
      g->n = n;
      g->nnz = nnz;
      ND_CHECK(dalloc_t(&g->row_ptr, static_cast<size_t>(n + 1)));
      ND_CHECK(dalloc_t(&g->col, static_cast<size_t>(nnz)));
      ND_CHECK(dalloc_t(&g->old_id, static_cast<size_t>(n)));
      ND_CHECK(dalloc_t(&g->dinv_sqrt, static_cast<size_t>(n)));
      hipLaunchKernelGGL(k_old_id, dim3(grid_for(n_nodes, kBlock)), dim3(kBlock), 0, st, present, new_id,
                         n_nodes, g->old_id);
      ND_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_rows_cols, dim3(grid_for(nnz, kBlock)), dim3(kBlock), 0, st, alt, nnz, bits,
                         new_id, g->row_ptr, g->col, n);
      ND_LAUNCH_CHECK();
      // a grid-stride grid of 256 blocks: one max-degree atomic per wavefront
      hipLaunchKernelGGL(k_dinv, dim3(grid_for(n, kBlock, 256)), dim3(kBlock), 0, st, g->row_ptr, n, g->dinv_sqrt,
                         counters + 2);
      ND_LAUNCH_CHECK();
      unsigned long long mx = 0;
      ND_HIP(hipMemcpyAsync(&mx, counters + 2, sizeof(mx), hipMemcpyDeviceToHost, st));
      ND_HIP(hipStreamSynchronize(st));
      g->max_deg = static_cast<int64_t>(mx);
      return ND_OK;
    }
  }
  // no edge survives: the empty graph
  g->n = 0;
  g->nnz = 0;
  ND_CHECK(dalloc_t(&g->row_ptr, 1));
  ND_HIP(hipMemsetAsync(g->row_ptr, 0, sizeof(int64_t), st));
  ND_HIP(hipStreamSynchronize(st));
  return ND_OK;
}

}  // namespace

}  // namespace nd

nd_graph::~nd_graph() {
  nd::dfree(row_ptr);
  nd::dfree(col);
  nd::dfree(old_id);
  nd::dfree(dinv_sqrt);
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* nd_last_error(void) { return nd::g_err.c_str(); }

nd_status nd_build_csr(int64_t n_nodes, int64_t n_edges, const int32_t* src, const int32_t* dst,
                       uint32_t flags, void* stream, nd_graph** out) {
  nd::clear_error();
  ND_REQUIRE(out != nullptr, "nd_build_csr: out is NULL");
  *out = nullptr;
  ND_REQUIRE(n_nodes >= 1 && n_nodes < (int64_t(1) << 31), "nd_build_csr: n_nodes=%lld not in [1, 2^31)",
             (long long)n_nodes);
  ND_REQUIRE(n_edges >= 0 && n_edges < (int64_t(1) << 31), "nd_build_csr: n_edges=%lld not in [0, 2^31)",
             (long long)n_edges);
  ND_REQUIRE(n_edges == 0 || (src && dst), "nd_build_csr: src/dst is NULL");
  ND_REQUIRE((flags & ~ND_INPUT_DEVICE) == 0, "nd_build_csr: unknown flags 0x%x", flags);
  std::unique_ptr<nd_graph> g(new nd_graph());
  ND_HIP(hipGetDevice(&g->device));
  nd_status s = nd::build_impl(n_nodes, n_edges, src, dst, flags, nd::as_stream(stream), g.get());
  if (s != ND_OK) return s;
  *out = g.release();
  return ND_OK;
}

nd_status nd_graph_info(const nd_graph* g, int64_t* n, int64_t* nnz, int64_t* max_deg) {
  nd::clear_error();
  ND_REQUIRE(g != nullptr, "nd_graph_info: graph is NULL");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_deg) *max_deg = g->max_deg;
  return ND_OK;
}

nd_status nd_graph_export(const nd_graph* g, int64_t* row_ptr, int32_t* col, int32_t* old_id,
                          float* dinv_sqrt) {
  nd::clear_error();
  ND_REQUIRE(g != nullptr, "nd_graph_export: graph is NULL");
  ND_HIP(hipDeviceSynchronize());
  if (row_ptr) ND_HIP(hipMemcpy(row_ptr, g->row_ptr, static_cast<size_t>(g->n + 1) * 8, hipMemcpyDeviceToHost));
  if (col && g->nnz) ND_HIP(hipMemcpy(col, g->col, static_cast<size_t>(g->nnz) * 4, hipMemcpyDeviceToHost));
  if (old_id && g->n) ND_HIP(hipMemcpy(old_id, g->old_id, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToHost));
  if (dinv_sqrt && g->n)
    ND_HIP(hipMemcpy(dinv_sqrt, g->dinv_sqrt, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToHost));
  return ND_OK;
}

nd_status nd_graph_device_arrays(const nd_graph* g, const int64_t** row_ptr, const int32_t** col,
                                 const float** dinv_sqrt) {
  nd::clear_error();
  ND_REQUIRE(g != nullptr, "nd_graph_device_arrays: graph is NULL");
  if (row_ptr) *row_ptr = g->row_ptr;
  if (col) *col = g->col;
  if (dinv_sqrt) *dinv_sqrt = g->dinv_sqrt;
  return ND_OK;
}

nd_status nd_graph_step_timing(const nd_graph* g, double* total_ms, int64_t* launches) {
  nd::clear_error();
  ND_REQUIRE(g != nullptr, "nd_graph_step_timing: graph is NULL");
  if (total_ms) *total_ms = g->step_ms;
  if (launches) *launches = g->step_launches;
  return ND_OK;
}

void nd_graph_free(nd_graph* g) { delete g; }

}  // extern "C"
