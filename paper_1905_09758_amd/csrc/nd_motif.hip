// Twin motifs (Sec. 3.4): nodes with identical open neighbourhoods.
//
// The paper finds node copies with a random hash w = Hz and equal entries
// w_i = w_j.  Here the hash is integer and order-free,
//   h_i = sum_{j in N(i)} r_j  (mod 2^64),  r_j = SplitMix64 output j+1,
// so it is identical on any thread mapping.  Nodes are sorted by h (stable,
// ascending node id within equal keys); each run of equal h is a candidate
// class, confirmed by exact comparison of the sorted neighbour lists against
// the group leader.  Members that differ (hash collisions) are split off into
// a new group led by their smallest member and verified again, until every
// group is exact.  The resulting partition is independent of the seed.
#include <cstdlib>

#include "nd_common.h"

namespace nd {
namespace {

__global__ __launch_bounds__(kBlock) void k_twin_hash(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, int64_t n, uint64_t key,
                                                      uint64_t mask, uint64_t* __restrict__ h,
                                                      uint32_t* __restrict__ idx) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    uint64_t s = 0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += splitmix64(key, static_cast<uint64_t>(col[e]) + 1);
    h[i] = s & mask;
    idx[i] = static_cast<uint32_t>(i);
  }
}

// label[p] = first position of p's run of equal hash; run_size at the head.
__global__ __launch_bounds__(kBlock) void k_runs(const uint64_t* __restrict__ h, int64_t n,
                                                 int64_t* __restrict__ label) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (p == 0 || h[p] != h[p - 1]) {
      int64_t q = p;
      while (q + 1 < n && h[q + 1] == h[p]) ++q;
      for (int64_t t = p; t <= q; ++t) label[t] = p;
    }
  }
}

__device__ inline bool same_neighbourhood(const int64_t* row_ptr, const int32_t* col, int64_t a, int64_t b) {
  const int64_t a0 = row_ptr[a], a1 = row_ptr[a + 1], b0 = row_ptr[b], b1 = row_ptr[b + 1];
  if (a1 - a0 != b1 - b0) return false;
  for (int64_t t = 0; t < a1 - a0; ++t)
    if (col[a0 + t] != col[b0 + t]) return false;
  return true;
}

// Compare each non-leader with its group leader; mismatches propose the
// smallest mismatching position of the group as the new group's leader.
__global__ __launch_bounds__(kBlock) void k_verify(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   const uint32_t* __restrict__ node, const int64_t* __restrict__ label,
                                                   int64_t n, int32_t* __restrict__ mism,
                                                   unsigned long long* __restrict__ newlab,
                                                   unsigned long long* __restrict__ n_mism,
                                                   int32_t* __restrict__ run_split, const int64_t* __restrict__ run_of) {
  unsigned long long cnt = 0;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t l = label[p];
    mism[p] = 0;
    if (l == p) continue;
    if (!same_neighbourhood(row_ptr, col, node[p], node[l])) {
      mism[p] = 1;
      atomicMin(&newlab[l], static_cast<unsigned long long>(p));
      run_split[run_of[p]] = 1;
      cnt++;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(n_mism, cnt);
}

__global__ __launch_bounds__(kBlock) void k_relabel(int64_t n, const int32_t* __restrict__ mism,
                                                    int64_t* __restrict__ label,
                                                    const unsigned long long* __restrict__ newlab) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    if (mism[p]) label[p] = static_cast<int64_t>(newlab[label[p]]);
}

__global__ __launch_bounds__(kBlock) void k_reset_newlab(int64_t n, unsigned long long* __restrict__ newlab) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    newlab[p] = ~0ull;
}

// Run index of each position (run_of) from the initial labels.
__global__ __launch_bounds__(kBlock) void k_run_flags(const int64_t* __restrict__ label, int64_t n,
                                                      int32_t* __restrict__ flag) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    flag[p] = label[p] == p ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_run_index(const int64_t* __restrict__ excl, const int32_t* __restrict__ flag,
                                                      int64_t n, int64_t* __restrict__ run_of) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    run_of[p] = excl[p] + flag[p] - 1;
}

// Group sizes (by leader position).
__global__ __launch_bounds__(kBlock) void k_group_count(const int64_t* __restrict__ label, int64_t n,
                                                        int32_t* __restrict__ gsize) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    atomicAdd(&gsize[label[p]], 1);
}

// Mark the smallest member (the leader) of every group of size >= 2, by node id.
__global__ __launch_bounds__(kBlock) void k_leader_flags(const int64_t* __restrict__ label,
                                                         const int32_t* __restrict__ gsize,
                                                         const uint32_t* __restrict__ node, int64_t n,
                                                         int32_t* __restrict__ is_leader, int32_t* __restrict__ csize) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    if (label[p] == p && gsize[p] >= 2) {
      is_leader[node[p]] = 1;
      csize[node[p]] = gsize[p];
    }
}

// Class size indexed by class (ordered by leader node id).
__global__ __launch_bounds__(kBlock) void k_class_sizes(const int32_t* __restrict__ is_leader,
                                                        const int32_t* __restrict__ csize,
                                                        const int64_t* __restrict__ cls_of_node, int64_t n,
                                                        int64_t* __restrict__ sizes) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    if (is_leader[i]) sizes[cls_of_node[i]] = csize[i];
}

// Rank of each member inside its group, in ascending position (= node) order.
// Runs that never split hold one group in consecutive positions.
__global__ __launch_bounds__(kBlock) void k_rank_simple(const int64_t* __restrict__ label,
                                                        const int32_t* __restrict__ run_split,
                                                        const int64_t* __restrict__ run_of, int64_t n,
                                                        int64_t* __restrict__ rank) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    if (!run_split[run_of[p]]) rank[p] = p - label[p];
}

// Split runs: one thread walks the run and counts per group (by leader position).
__global__ __launch_bounds__(kBlock) void k_rank_split(const int64_t* __restrict__ label,
                                                       const int32_t* __restrict__ run_split,
                                                       const int64_t* __restrict__ run_of, int64_t n,
                                                       int32_t* __restrict__ counter, int64_t* __restrict__ rank) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (!(p == 0 || run_of[p] != run_of[p - 1])) continue;  // run heads only
    if (!run_split[run_of[p]]) continue;
    for (int64_t t = p; t < n && run_of[t] == run_of[p]; ++t) rank[t] = counter[label[t]]++;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_members(const int64_t* __restrict__ label,
                                                            const int32_t* __restrict__ gsize,
                                                            const uint32_t* __restrict__ node,
                                                            const int64_t* __restrict__ cls_of_node,
                                                            const int64_t* __restrict__ class_ptr,
                                                            const int64_t* __restrict__ rank, int64_t n,
                                                            int32_t* __restrict__ members) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t l = label[p];
    if (gsize[l] < 2) continue;
    const int64_t c = cls_of_node[node[l]];
    members[class_ptr[c] + rank[p]] = static_cast<int32_t>(node[p]);
  }
}


nd_status twins_impl(const nd_graph* g, uint64_t seed, hipStream_t st, nd_motifs* out) {
  const int64_t n = g->n;
  out->n = n;
  if (n < 2) {
    ND_CHECK(dalloc_t(&out->class_ptr, 1));
    ND_HIP(hipMemsetAsync(out->class_ptr, 0, 8, st));
    ND_HIP(hipStreamSynchronize(st));
    return ND_OK;
  }
  Tmp t;
  const int grid = grid_for(n, kBlock);
  uint64_t *h, *h2;
  uint32_t *node, *node2;
  ND_CHECK(t.get(&h, n));
  ND_CHECK(t.get(&h2, n));
  ND_CHECK(t.get(&node, n));
  ND_CHECK(t.get(&node2, n));
  uint64_t mask = ~0ull;
  if (const char* e = std::getenv("ND_TWIN_HASH_BITS")) {  // test hook: force collisions
    int b = std::atoi(e);
    if (b > 0 && b < 64) mask = (1ull << b) - 1ull;
  }
  hipLaunchKernelGGL(k_twin_hash, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, n, splitmix64(seed, 1), mask,
                     h, node);
  ND_LAUNCH_CHECK();
  ND_CHECK(radix_sort_u64(h, h2, node, node2, n, 64, st));
  int64_t *label, *run_of, *excl, *tot;
  int32_t *flag, *mism, *run_split;
  unsigned long long *newlab, *n_mism;
  ND_CHECK(t.get(&label, n));
  ND_CHECK(t.get(&run_of, n));
  ND_CHECK(t.get(&excl, n));
  ND_CHECK(t.get(&tot, 1));
  ND_CHECK(t.get(&flag, n));
  ND_CHECK(t.get(&mism, n));
  ND_CHECK(t.get(&run_split, n));
  ND_CHECK(t.get(&newlab, n));
  ND_CHECK(t.get(&n_mism, 1));
  hipLaunchKernelGGL(k_runs, dim3(grid), dim3(kBlock), 0, st, h, n, label);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_run_flags, dim3(grid), dim3(kBlock), 0, st, label, n, flag);
  ND_LAUNCH_CHECK();
  ND_CHECK(exclusive_scan_i32_i64(flag, excl, n, tot, st));
  hipLaunchKernelGGL(k_run_index, dim3(grid), dim3(kBlock), 0, st, excl, flag, n, run_of);
  ND_LAUNCH_CHECK();
  ND_HIP(hipMemsetAsync(run_split, 0, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_reset_newlab, dim3(grid), dim3(kBlock), 0, st, n, newlab);
  ND_LAUNCH_CHECK();
  // every iteration splits at least one new exact group off each mixed group,
  // so n iterations always suffice
  for (int64_t iter = 0; iter < n; ++iter) {
    ND_HIP(hipMemsetAsync(n_mism, 0, 8, st));
    hipLaunchKernelGGL(k_verify, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, node, label, n, mism, newlab,
                       n_mism, run_split, run_of);
    ND_LAUNCH_CHECK();
    unsigned long long hm = 0;
    ND_HIP(hipMemcpyAsync(&hm, n_mism, 8, hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
    if (hm == 0) break;
    hipLaunchKernelGGL(k_relabel, dim3(grid), dim3(kBlock), 0, st, n, mism, label, newlab);
    ND_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_reset_newlab, dim3(grid), dim3(kBlock), 0, st, n, newlab);
    ND_LAUNCH_CHECK();
  }
  int32_t *gsize, *is_leader, *csize;
  int64_t *cls_of_node, *sizes, *rank;
  ND_CHECK(t.get(&gsize, n));
  ND_CHECK(t.get(&is_leader, n));
  ND_CHECK(t.get(&csize, n));
  ND_CHECK(t.get(&cls_of_node, n));
  ND_CHECK(t.get(&rank, n));
  ND_HIP(hipMemsetAsync(gsize, 0, static_cast<size_t>(n) * 4, st));
  ND_HIP(hipMemsetAsync(is_leader, 0, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_group_count, dim3(grid), dim3(kBlock), 0, st, label, n, gsize);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_leader_flags, dim3(grid), dim3(kBlock), 0, st, label, gsize, node, n, is_leader, csize);
  ND_LAUNCH_CHECK();
  ND_CHECK(exclusive_scan_i32_i64(is_leader, cls_of_node, n, tot, st));
  int64_t n_cls = 0;
  ND_HIP(hipMemcpyAsync(&n_cls, tot, 8, hipMemcpyDeviceToHost, st));
  ND_HIP(hipStreamSynchronize(st));
  out->n_classes = n_cls;
  ND_CHECK(dalloc_t(&out->class_ptr, static_cast<size_t>(n_cls + 1)));
  if (n_cls == 0) {
    ND_HIP(hipMemsetAsync(out->class_ptr, 0, 8, st));
    ND_HIP(hipStreamSynchronize(st));
    return ND_OK;
  }
  ND_CHECK(t.get(&sizes, n_cls));
  hipLaunchKernelGGL(k_class_sizes, dim3(grid), dim3(kBlock), 0, st, is_leader, csize, cls_of_node, n, sizes);
  ND_LAUNCH_CHECK();
  ND_CHECK(exclusive_scan_i64(sizes, out->class_ptr, n_cls, tot, st));
  ND_HIP(hipMemcpyAsync(out->class_ptr + n_cls, tot, 8, hipMemcpyDeviceToDevice, st));
  int64_t n_mem = 0;
  ND_HIP(hipMemcpyAsync(&n_mem, tot, 8, hipMemcpyDeviceToHost, st));
  ND_HIP(hipStreamSynchronize(st));
  out->n_members = n_mem;
  out->spike_weight = static_cast<double>(n_mem - n_cls) / static_cast<double>(n);
  ND_CHECK(dalloc_t(&out->members, static_cast<size_t>(n_mem)));
  // ranks: reuse gsize-shaped counters for split runs
  int32_t* counter;
  ND_CHECK(t.get(&counter, n));
  ND_HIP(hipMemsetAsync(counter, 0, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_rank_simple, dim3(grid), dim3(kBlock), 0, st, label, run_split, run_of, n, rank);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rank_split, dim3(grid), dim3(kBlock), 0, st, label, run_split, run_of, n, counter, rank);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scatter_members, dim3(grid), dim3(kBlock), 0, st, label, gsize, node, cls_of_node,
                     out->class_ptr, rank, n, out->members);
  ND_LAUNCH_CHECK();
  ND_HIP(hipStreamSynchronize(st));
  return ND_OK;
}

}  // namespace
}  // namespace nd

nd_motifs::~nd_motifs() {
  nd::dfree(class_ptr);
  nd::dfree(members);
}

extern "C" {

nd_status nd_motif_filter(const nd_graph* g, uint64_t seed, uint32_t kinds, void* stream, nd_motifs** out) {
  nd::clear_error();
  ND_REQUIRE(out != nullptr, "nd_motif_filter: out is NULL");
  *out = nullptr;
  ND_REQUIRE(g != nullptr, "nd_motif_filter: graph is NULL");
  if (kinds != ND_TWINS_OPEN) {
    nd::set_error("nd_motif_filter: kinds=0x%x; only ND_TWINS_OPEN is implemented", kinds);
    return ND_EUNSUPPORTED;
  }
  std::unique_ptr<nd_motifs> m(new nd_motifs());
  ND_HIP(hipGetDevice(&m->device));
  ND_CHECK(nd::twins_impl(g, seed, nd::as_stream(stream), m.get()));
  *out = m.release();
  return ND_OK;
}

nd_status nd_motif_info(const nd_motifs* m, int64_t* n_classes, int64_t* n_motif_nodes, int32_t* n_spikes,
                        double* spike_lambda, double* spike_weight) {
  nd::clear_error();
  ND_REQUIRE(m != nullptr, "nd_motif_info: motifs is NULL");
  if (n_classes) *n_classes = m->n_classes;
  if (n_motif_nodes) *n_motif_nodes = m->n_members;
  const int32_t ns = m->n_classes > 0 ? 1 : 0;
  if (n_spikes) *n_spikes = ns;
  if (ns && spike_lambda) spike_lambda[0] = 0.0;
  if (ns && spike_weight) spike_weight[0] = m->spike_weight;
  return ND_OK;
}

nd_status nd_motif_export(const nd_motifs* m, int64_t* class_ptr, int32_t* members) {
  nd::clear_error();
  ND_REQUIRE(m != nullptr, "nd_motif_export: motifs is NULL");
  ND_HIP(hipDeviceSynchronize());
  if (class_ptr)
    ND_HIP(hipMemcpy(class_ptr, m->class_ptr, static_cast<size_t>(m->n_classes + 1) * 8, hipMemcpyDeviceToHost));
  if (members && m->n_members)
    ND_HIP(hipMemcpy(members, m->members, static_cast<size_t>(m->n_members) * 4, hipMemcpyDeviceToHost));
  return ND_OK;
}

void nd_motifs_free(nd_motifs* m) { delete m; }

}  // extern "C"
