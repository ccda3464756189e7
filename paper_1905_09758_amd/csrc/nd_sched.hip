// Internal row order and row-to-wavefront schedules of the sparse product.
//
// The graph's CSR (compact ids, ascending) is renumbered once per graph by
// descending degree, ties by ascending id, with a stable radix sort on the
// degree.  The sparse product then works on this internal CSR: every degree
// class is a contiguous row range (no row lists to read), the rows split into
// chunks come first, and the most-gathered rows -- the high-degree ones -- lie
// next to each other, so their cache lines are shared by hot rows only.
// Results do not depend on the numbering except through fp32 rounding order.
#include <cstdlib>

#include "nd_common.h"

namespace nd {

Internal::~Internal() {
  dfree(perm);
  dfree(inv);
  dfree(row_ptr);
  dfree(col);
}

Schedule::~Schedule() {
  dfree(split_chunk_ptr);
  dfree(chunk_owner);
}

namespace {

__global__ __launch_bounds__(kBlock) void k_deg_keys(const int64_t* __restrict__ row_ptr, int64_t n, int64_t max_deg,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ ids) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    keys[i] = static_cast<uint64_t>(max_deg - (row_ptr[i + 1] - row_ptr[i]));
    ids[i] = static_cast<uint32_t>(i);
  }
}

__global__ __launch_bounds__(kBlock) void k_inv_deg(const uint32_t* __restrict__ perm, const int64_t* __restrict__ row_ptr,
                                                    int64_t n, int32_t* __restrict__ inv, int64_t* __restrict__ deg_int) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = perm[p];
    inv[i] = static_cast<int32_t>(p);
    deg_int[p] = row_ptr[i + 1] - row_ptr[i];
  }
}

// One wavefront per internal row copies the row's neighbours, renumbered.
__global__ __launch_bounds__(kBlock) void k_internal_cols(const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                                                          const int64_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const int64_t* __restrict__ row_ptr_int, int64_t n,
                                                          int32_t* __restrict__ col_int) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t p = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; p < n;
       p += static_cast<int64_t>(gridDim.x) * (kBlock / kWave)) {
    const int64_t i = perm[p];
    const int64_t s0 = row_ptr[i], d = row_ptr[i + 1] - s0, o = row_ptr_int[p];
    for (int64_t t = lane; t < d; t += kWave) col_int[o + t] = inv[col[s0 + t]];
  }
}

__device__ inline int ceil_log2_dev(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) b++;
  return b;
}

// cnt[b] = rows with log2 P = b (b <= log2_pmax); cnt[log2_pmax + 1] = split rows.
// Each wavefront counts in registers over its grid-stride rows and adds its
// totals once at the end (the grid is a few hundred blocks).
__global__ __launch_bounds__(kBlock) void k_bin_count(const int64_t* __restrict__ row_ptr, int64_t n, int log2_pmax,
                                                      int64_t chunk_nnz, int slot_nnz,
                                                      unsigned long long* __restrict__ cnt) {
  unsigned long long wc[kMaxBins + 2] = {};
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock; base < n;
       base += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = base + threadIdx.x;
    int b = -1;
    if (i < n) {
      const int64_t d = row_ptr[i + 1] - row_ptr[i];
      if (d > chunk_nnz) {
        b = log2_pmax + 1;
      } else {
        b = ceil_log2_dev((d + slot_nnz - 1) / slot_nnz);
        if (b > log2_pmax) b = log2_pmax;
      }
    }
#pragma unroll
    for (int t = 0; t < kMaxBins + 2; ++t)
      if (t <= log2_pmax + 1) wc[t] += __popcll(__ballot(b == t));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int t = 0; t < kMaxBins + 2; ++t)
      if (t <= log2_pmax + 1 && wc[t]) atomicAdd(&cnt[t], wc[t]);
  }
}

__global__ __launch_bounds__(kBlock) void k_split_chunks(const int64_t* __restrict__ row_ptr, int64_t n_split,
                                                         int64_t chunk_nnz, int64_t* __restrict__ nch) {
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; s < n_split;
       s += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t d = row_ptr[s + 1] - row_ptr[s];
    nch[s] = (d + chunk_nnz - 1) / chunk_nnz;
  }
}

__global__ __launch_bounds__(kBlock) void k_chunk_owner(const int64_t* __restrict__ ptr, int64_t n_split,
                                                        int32_t* __restrict__ owner) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t s = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; s < n_split;
       s += static_cast<int64_t>(gridDim.x) * (kBlock / kWave))
    for (int64_t c = ptr[s] + lane; c < ptr[s + 1]; c += kWave) owner[c] = static_cast<int32_t>(s);
}

}  // namespace

nd_status get_internal(nd_graph* g, hipStream_t st, Internal** out) {
  if (g->internal) {
    *out = g->internal.get();
    return ND_OK;
  }
  const int64_t n = g->n, nnz = g->nnz;
  std::unique_ptr<Internal> in(new Internal());
  ND_CHECK(dalloc_t(&in->perm, static_cast<size_t>(n)));
  ND_CHECK(dalloc_t(&in->inv, static_cast<size_t>(n)));
  ND_CHECK(dalloc_t(&in->row_ptr, static_cast<size_t>(n + 1)));
  ND_CHECK(dalloc_t(&in->col, static_cast<size_t>(nnz > 0 ? nnz : 1)));
  {
    Tmp t;
    uint64_t *keys, *akeys;
    uint32_t* avals;
    int64_t *deg, *tot;
    ND_CHECK(t.get(&keys, n));
    ND_CHECK(t.get(&akeys, n));
    ND_CHECK(t.get(&avals, n));
    ND_CHECK(t.get(&deg, n));
    ND_CHECK(t.get(&tot, 1));
    uint32_t* perm = reinterpret_cast<uint32_t*>(in->perm);
    hipLaunchKernelGGL(k_deg_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, g->row_ptr, n, g->max_deg, keys,
                       perm);
    ND_LAUNCH_CHECK();
    int bits = 0;
    while ((int64_t(1) << bits) <= g->max_deg) bits++;
    ND_CHECK(radix_sort_u64(keys, akeys, perm, avals, n, bits, st));
    hipLaunchKernelGGL(k_inv_deg, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, perm, g->row_ptr, n, in->inv, deg);
    ND_LAUNCH_CHECK();
    ND_CHECK(exclusive_scan_i64(deg, in->row_ptr, n, tot, st));
    ND_HIP(hipMemcpyAsync(in->row_ptr + n, tot, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_internal_cols, dim3(grid_for(n * kWave, kBlock)), dim3(kBlock), 0, st, in->perm, in->inv,
                       g->row_ptr, g->col, in->row_ptr, n, in->col);
    ND_LAUNCH_CHECK();
    ND_HIP(hipStreamSynchronize(st));
  }
  *out = in.get();
  g->internal = std::move(in);
  return ND_OK;
}

nd_status get_schedule(nd_graph* g, int L, hipStream_t st, Schedule** out) {
  auto it = g->sched.find(L);
  if (it != g->sched.end()) {
    *out = it->second.get();
    return ND_OK;
  }
  Internal* in = nullptr;
  ND_CHECK(get_internal(g, st, &in));
  std::unique_ptr<Schedule> s(new Schedule());
  s->L = L;
  const int pmax = kWave / L;
  int log2_pmax = 0;
  while ((1 << log2_pmax) < pmax) log2_pmax++;
  s->chunk_nnz = static_cast<int64_t>(pmax) * kChunkIters;
  const int64_t n = g->n;
  unsigned long long cnt[kMaxBins + 1] = {0};
  if (n > 0) {
    Tmp t;
    unsigned long long* dcnt;
    ND_CHECK(t.get(&dcnt, kMaxBins + 1));
    ND_HIP(hipMemsetAsync(dcnt, 0, sizeof(cnt), st));
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(n, kBlock, 256)), dim3(kBlock), 0, st, in->row_ptr, n, log2_pmax,
                       s->chunk_nnz, s->slot_nnz, dcnt);
    ND_LAUNCH_CHECK();
    ND_HIP(hipMemcpyAsync(cnt, dcnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
  }
  s->n_split = static_cast<int64_t>(cnt[log2_pmax + 1]);
  // bins in internal order: decreasing P after the split rows
  int64_t row = s->n_split, item = 0;
  int nb = 0;
  for (int b = log2_pmax; b >= 0; --b) {
    if (cnt[b] == 0) continue;
    s->bin_log2p[nb] = b;
    s->bin_row_start[nb] = row;
    s->bin_item_start[nb] = item;
    const int64_t rpw = kWave / ((int64_t(1) << b) * L);
    row += static_cast<int64_t>(cnt[b]);
    item += ceil_div(static_cast<int64_t>(cnt[b]), rpw);
    nb++;
  }
  s->n_bins = nb;
  s->bin_row_start[nb] = row;
  s->bin_item_start[nb] = item;
  if (s->n_split > 0) {
    Tmp t;
    int64_t *nch, *tot;
    ND_CHECK(t.get(&nch, static_cast<size_t>(s->n_split)));
    ND_CHECK(t.get(&tot, 1));
    ND_CHECK(dalloc_t(&s->split_chunk_ptr, static_cast<size_t>(s->n_split + 1)));
    hipLaunchKernelGGL(k_split_chunks, dim3(grid_for(s->n_split, kBlock)), dim3(kBlock), 0, st, in->row_ptr,
                       s->n_split, s->chunk_nnz, nch);
    ND_LAUNCH_CHECK();
    ND_CHECK(exclusive_scan_i64(nch, s->split_chunk_ptr, s->n_split, tot, st));
    ND_HIP(hipMemcpyAsync(s->split_chunk_ptr + s->n_split, tot, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    ND_HIP(hipMemcpyAsync(&s->n_chunks, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
    ND_CHECK(dalloc_t(&s->chunk_owner, static_cast<size_t>(s->n_chunks)));
    hipLaunchKernelGGL(k_chunk_owner, dim3(grid_for(s->n_split * kWave, kBlock)), dim3(kBlock), 0, st,
                       s->split_chunk_ptr, s->n_split, s->chunk_owner);
    ND_LAUNCH_CHECK();
    ND_HIP(hipStreamSynchronize(st));
  }
  s->n_items = s->n_chunks + item;
  *out = s.get();
  g->sched[L] = std::move(s);
  return ND_OK;
}

}  // namespace nd
