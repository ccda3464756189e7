// Device-wide primitives used by graph construction and motif grouping:
// exclusive prefix sums over int64 and a stable LSD radix sort of 64-bit keys
// (8-bit digits) with an optional 32-bit payload.  Both are deterministic.
#include "nd_common.h"

namespace nd {

namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048 elements per block

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int64_t t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one int64 per thread; returns the prefix and
// writes the block total to *total.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int64_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <typename InT>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const InT* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ sums) {
  __shared__ int64_t red[kBlock / kWave];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) s += static_cast<int64_t>(in[i]);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

template <typename InT>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const InT* __restrict__ in, int64_t* out,
                                                      int64_t n, const int64_t* __restrict__ offs,
                                                      int64_t* total_dev) {
  __shared__ int64_t tile[kScanTile];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    tile[r * kBlock + threadIdx.x] = i < n ? static_cast<int64_t>(in[i]) : 0;
  }
  __syncthreads();
  int64_t loc[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    loc[r] = s;
    s += tile[threadIdx.x * kScanItems + r];
  }
  int64_t tot;
  int64_t pre = block_excl_scan(s, &tot);
  const int64_t off = offs ? offs[blockIdx.x] : 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) tile[threadIdx.x * kScanItems + r] = off + pre + loc[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) out[i] = tile[r * kBlock + threadIdx.x];
  }
  if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_dev = off + tot;
}

template <typename InT>
nd_status scan_impl(const InT* in, int64_t* out, int64_t n, int64_t* total_dev, hipStream_t st) {
  if (n <= 0) {
    if (total_dev) ND_HIP(hipMemsetAsync(total_dev, 0, sizeof(int64_t), st));
    return ND_OK;
  }
  const int64_t tiles = ceil_div(n, kScanTile);
  if (tiles > 0x7FFFFFFF) {
    set_error("scan: %lld elements is too many", (long long)n);
    return ND_EOVERFLOW;
  }
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan<InT>, dim3(1), dim3(kBlock), 0, st, in, out, n, nullptr, total_dev);
    ND_LAUNCH_CHECK();
    return ND_OK;
  }
  int64_t* sums = nullptr;
  ND_CHECK(dalloc_t(&sums, static_cast<size_t>(tiles)));
  hipLaunchKernelGGL(k_tile_sums<InT>, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, in, n, sums);
  nd_status s = ND_OK;
  if (hipGetLastError() != hipSuccess) s = ND_EDEVICE;
  if (s == ND_OK) s = scan_impl<int64_t>(sums, sums, tiles, nullptr, st);
  if (s == ND_OK) {
    hipLaunchKernelGGL(k_tile_scan<InT>, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, in,
                       out, n, sums, total_dev);
    if (hipGetLastError() != hipSuccess) s = ND_EDEVICE;
  }
  // the temporary is freed only after the stream has consumed it
  if (hipStreamSynchronize(st) != hipSuccess && s == ND_OK) s = ND_EDEVICE;
  dfree(sums);
  if (s == ND_EDEVICE) set_error("scan: kernel failure");
  return s;
}

// ------------------------------------------------------------------ radix sort
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;  // 4096 keys per tile

__device__ inline uint32_t digit_of(uint64_t k, int shift) {
  return static_cast<uint32_t>(k >> shift) & (kRadix - 1);
}

// counts[d * n_tiles + tile] = number of keys of the tile with digit d.
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                       int shift, uint32_t* __restrict__ counts,
                                                       int64_t n_tiles) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  counts[static_cast<int64_t>(threadIdx.x) * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: the tile's keys are loaded once into registers (all
// loads in flight together), ranked round by round (256 keys per round, in
// input order), placed sorted-by-digit in LDS, then written out so that keys
// with equal digits leave in consecutive addresses.
template <bool kVals>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, uint64_t* __restrict__ okeys,
    uint32_t* __restrict__ ovals, int64_t n, int shift, const int64_t* __restrict__ offs,
    int64_t n_tiles) {
  __shared__ uint64_t skeys[kSortTile];
  __shared__ uint32_t svals[kVals ? kSortTile : 1];
  __shared__ uint32_t tile_off[kRadix];   // exclusive prefix of the tile histogram
  __shared__ uint32_t running[kRadix];    // keys of each digit placed so far
  __shared__ uint32_t wcnt[kBlock / kWave][kRadix];
  __shared__ int64_t gbase[kRadix];       // output index of the tile's first key of each digit, minus tile_off

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
  const int64_t tile_n64 = n - base < kSortTile ? n - base : kSortTile;
  const int tile_n = static_cast<int>(tile_n64);

  uint64_t kr[kSortItems];
  uint32_t vr[kVals ? kSortItems : 1];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int li = r * kBlock + tid;
    kr[r] = li < tile_n ? keys[base + li] : 0;
    if constexpr (kVals) vr[r] = li < tile_n ? vals[base + li] : 0;
  }
  // tile histogram -> local exclusive offsets
  running[tid] = 0;
  for (int w = 0; w < kBlock / kWave; ++w) wcnt[w][tid] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r)
    if (r * kBlock + tid < tile_n) atomicAdd(&running[digit_of(kr[r], shift)], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t s = 0;
    for (int d = 0; d < kRadix; ++d) {
      tile_off[d] = s;
      s += running[d];
    }
  }
  __syncthreads();
  running[tid] = 0;
  gbase[tid] = offs[static_cast<int64_t>(tid) * n_tiles + blockIdx.x] - tile_off[tid];
  __syncthreads();

  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int li = r * kBlock + tid;
    const bool valid = li < tile_n;
    const uint64_t k = kr[r];
    uint32_t v = 0;
    if constexpr (kVals) v = vr[r];
    uint32_t d = digit_of(k, shift);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wid][d] = static_cast<uint32_t>(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t pre = running[d];
      for (int w = 0; w < wid; ++w) pre += wcnt[w][d];
      const uint32_t pos = tile_off[d] + pre + static_cast<uint32_t>(rank);
      skeys[pos] = k;
      if (kVals) svals[pos] = v;
    }
    __syncthreads();
    {
      uint32_t add = 0;
      for (int w = 0; w < kBlock / kWave; ++w) {
        add += wcnt[w][tid];
        wcnt[w][tid] = 0;
      }
      running[tid] += add;
    }
    __syncthreads();
  }
  // write out: LDS position p holds the p-th key of the tile in digit order
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    const int p = r * kBlock + tid;
    if (p < tile_n) {
      const uint64_t k = skeys[p];
      const int64_t dst = gbase[digit_of(k, shift)] + p;
      okeys[dst] = k;
      if (kVals) ovals[dst] = svals[p];
    }
  }
}

}  // namespace

nd_status exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_dev,
                             hipStream_t st) {
  return scan_impl<int64_t>(in, out, n, total_dev, st);
}

nd_status exclusive_scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total_dev,
                                 hipStream_t st) {
  return scan_impl<int32_t>(in, out, n, total_dev, st);
}

nd_status radix_sort_u64(uint64_t* keys, uint64_t* alt_keys, uint32_t* vals, uint32_t* alt_vals,
                         int64_t n, int nbits, hipStream_t st) {
  if (n <= 1 || nbits <= 0) return ND_OK;
  const int64_t n_tiles = ceil_div(n, kSortTile);
  if (n_tiles * kRadix > (int64_t(1) << 40) || n_tiles > 0x7FFFFFFF) {
    set_error("radix sort: %lld keys is too many", (long long)n);
    return ND_EOVERFLOW;
  }
  uint32_t* counts = nullptr;
  int64_t* offs = nullptr;
  ND_CHECK(dalloc_t(&counts, static_cast<size_t>(n_tiles * kRadix)));
  nd_status s = dalloc_t(&offs, static_cast<size_t>(n_tiles * kRadix));
  if (s != ND_OK) {
    dfree(counts);
    return s;
  }
  uint64_t *ka = keys, *kb = alt_keys;
  uint32_t *va = vals, *vb = alt_vals;
  const bool with_vals = vals != nullptr;
  for (int shift = 0; shift < nbits && s == ND_OK; shift += kRadixBits) {
    hipLaunchKernelGGL(k_radix_hist, dim3(static_cast<unsigned>(n_tiles)), dim3(kBlock), 0, st, ka, n,
                       shift, counts, n_tiles);
    if (hipGetLastError() != hipSuccess) {
      s = ND_EDEVICE;
      break;
    }
    s = exclusive_scan_i32_i64(reinterpret_cast<const int32_t*>(counts), offs, n_tiles * kRadix,
                               nullptr, st);
    if (s != ND_OK) break;
    if (with_vals)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(static_cast<unsigned>(n_tiles)), dim3(kBlock), 0, st,
                         ka, va, kb, vb, n, shift, offs, n_tiles);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3(static_cast<unsigned>(n_tiles)), dim3(kBlock), 0,
                         st, ka, va, kb, vb, n, shift, offs, n_tiles);
    if (hipGetLastError() != hipSuccess) {
      s = ND_EDEVICE;
      break;
    }
    uint64_t* tk = ka;
    ka = kb;
    kb = tk;
    uint32_t* tv = va;
    va = vb;
    vb = tv;
  }
  if (s == ND_OK && ka != keys) {
    if (hipMemcpyAsync(keys, ka, static_cast<size_t>(n) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
      s = ND_EDEVICE;
    if (s == ND_OK && with_vals &&
        hipMemcpyAsync(vals, va, static_cast<size_t>(n) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
      s = ND_EDEVICE;
  }
  if (hipStreamSynchronize(st) != hipSuccess && s == ND_OK) s = ND_EDEVICE;
  dfree(counts);
  dfree(offs);
  if (s == ND_EDEVICE) set_error("radix sort: kernel failure");
  return s;
}

}  // namespace nd
