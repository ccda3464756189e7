// Twin motifs (Sec. 3.4): nodes with identical open neighbourhoods
// (eigenvalue 0 on the differences inside a class) or identical closed
// neighbourhoods N(i) + {i} (adjacent nodes of equal degree d, eigenvalue
// -1/d; the paper's blade motif at -1/2 and its -1/m family).
//
// The paper finds node copies with a random hash w = Hz and equal entries
// w_i = w_j.  Here the hash is integer and order-free,
//   h_i = sum_{j in N(i)} r_j (+ r_i for closed neighbourhoods)  (mod 2^64),
// r_j = SplitMix64 output j+1, so it is identical on any thread mapping.
// Nodes are sorted by h (stable, ascending node id within equal keys); each
// run of equal h is a candidate group, confirmed by exact comparison of the
// sorted neighbour lists against the group leader.  Members that differ (hash
// collisions) are split off into a new group led by their smallest member
// and verified again, until every group is exact.  The partition is
// independent of the seed.  A node cannot have twins of both kinds, so the
// two passes give disjoint groups.
//
// Pendant twins (the motif figure's panels at +-1/sqrt(2) and +-1/2): nodes
// B of degree d >= 2 with exactly one leaf neighbour A and equal remaining
// neighbourhoods N(B) - {A}, found by the same hash-sort-verify passes on
// that remaining neighbourhood.  A group of c >= 2 gives two classes (the B's
// and the A's) whose differences carry c-1 eigenvalues at +1/sqrt(d) and c-1
// at -1/sqrt(d).  Pendant-twin nodes are never twins, so all classes stay
// disjoint.
//
// Hub paths (the figure's left panel at +-1/2): c >= 2 paths E - X - Y - F
// between the same two distinct nodes, with X, Y of degree 2 and no other
// degree-2 neighbour.  Keyed by the end pair (E, F), sorted; the nodes next
// to the smaller end form one class, the others a second, carrying c-1
// eigenvalues at +1/2 and c-1 at -1/2.
#include <cstdlib>
#include <map>
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

// The single leaf neighbour of b if b has degree >= 2 and exactly one leaf
// neighbour, else -1.
__device__ inline int64_t pendant_leaf(const int64_t* row_ptr, const int32_t* col, int64_t b) {
  if (row_ptr[b + 1] - row_ptr[b] < 2) return -1;
  int64_t leaf = -1;
  for (int64_t e = row_ptr[b]; e < row_ptr[b + 1]; ++e) {
    const int32_t u = col[e];
    if (row_ptr[u + 1] - row_ptr[u] == 1) {
      if (leaf >= 0) return -1;
      leaf = u;
    }
  }
  return leaf;
}

// Hash modes: 0 open neighbourhood, 1 closed, 2 the neighbourhood without
// the private leaf (pendant-twin candidates; other nodes get distinct keys
// with the top bit set, which the verification never groups).
//
// A wavefront takes 64 consecutive nodes: each lane hashes its own node when
// it has at most kLongRow neighbours; the longer rows of the 64 are then
// hashed by the whole wavefront in turn (lanes stride over the neighbours).
// The hash is a sum mod 2^64, so the split does not change its value.
constexpr int64_t kLongRow = 32;

__device__ inline uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(x), off, kWave);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(x >> 32), off, kWave);
    x += (static_cast<uint64_t>(hi) << 32) | lo;
  }
  return x;
}

__global__ __launch_bounds__(kBlock) void k_twin_hash(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, int64_t n, uint64_t key,
                                                      uint64_t mask, int mode, uint64_t* __restrict__ h,
                                                      uint32_t* __restrict__ idx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t n_waves = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
  for (int64_t base = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave * kWave; base < n;
       base += n_waves * kWave) {
    const int64_t i = base + lane;
    bool is_long = false;
    if (i < n) {
      idx[i] = static_cast<uint32_t>(i);
      is_long = row_ptr[i + 1] - row_ptr[i] > kLongRow;
      if (!is_long) {
        if (mode == 2) {
          const int64_t leaf = pendant_leaf(row_ptr, col, i);
          if (leaf < 0) {
            h[i] = (uint64_t(1) << 63) | static_cast<uint64_t>(i);
          } else {
            uint64_t s = 0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
              if (col[e] != leaf) s += splitmix64(key, static_cast<uint64_t>(col[e]) + 1);
            h[i] = (s & mask) & ~(uint64_t(1) << 63);
          }
        } else {
          uint64_t s = mode == 1 ? splitmix64(key, static_cast<uint64_t>(i) + 1) : 0;
          for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += splitmix64(key, static_cast<uint64_t>(col[e]) + 1);
          h[i] = s & mask;
        }
      }
    }
    uint64_t longs = __ballot(is_long);
    while (longs) {
      const int l = __ffsll(static_cast<long long>(longs)) - 1;
      longs &= longs - 1;
      const int64_t b = base + l;
      const int64_t e0 = row_ptr[b], e1 = row_ptr[b + 1];
      int64_t leaf = -1;
      bool keyed = true;
      if (mode == 2) {
        // the private leaf: the unique neighbour of degree 1, if exactly one
        // (the scan stops at the second one, like pendant_leaf)
        uint64_t cnt = 0, lsum = 0;
        for (int64_t e = e0; e < e1 && cnt < 2; e += kWave) {
          uint64_t c = 0, ls = 0;
          if (e + lane < e1) {
            const int32_t u = col[e + lane];
            if (row_ptr[u + 1] - row_ptr[u] == 1) {
              c = 1;
              ls = static_cast<uint64_t>(u) + 1;
            }
          }
          cnt += wave_sum_u64(c);
          lsum += wave_sum_u64(ls);
        }
        keyed = cnt == 1;
        leaf = keyed ? static_cast<int64_t>(lsum) - 1 : -1;
      }
      uint64_t s = 0;
      if (keyed)
        for (int64_t e = e0 + lane; e < e1; e += kWave)
          if (col[e] != leaf) s += splitmix64(key, static_cast<uint64_t>(col[e]) + 1);
      s = wave_sum_u64(s);
      if (lane == 0) {
        if (mode == 2)
          h[b] = keyed ? ((s & mask) & ~(uint64_t(1) << 63)) : ((uint64_t(1) << 63) | static_cast<uint64_t>(b));
        else
          h[b] = ((mode == 1 ? splitmix64(key, static_cast<uint64_t>(b) + 1) : 0) + s) & mask;
      }
    }
  }
}

// label[p] = first position of p's run of equal hash.
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

// Open: N(a) == N(b).  Closed: a ~ b and N(a) - {b} == N(b) - {a} (sorted
// lists compared while skipping b in a's list and a in b's list).  Pendant:
// both are candidates and N(a) - {leaf a} == N(b) - {leaf b}.
__device__ inline bool same_neighbourhood(const int64_t* row_ptr, const int32_t* col, int64_t a, int64_t b,
                                          int mode) {
  const int64_t a0 = row_ptr[a], a1 = row_ptr[a + 1], b0 = row_ptr[b], b1 = row_ptr[b + 1];
  if (a1 - a0 != b1 - b0) return false;
  if (mode == 0) {
    for (int64_t t = 0; t < a1 - a0; ++t)
      if (col[a0 + t] != col[b0 + t]) return false;
    return true;
  }
  if (mode == 2) {
    const int64_t la = pendant_leaf(row_ptr, col, a), lb = pendant_leaf(row_ptr, col, b);
    if (la < 0 || lb < 0) return false;
    int64_t i = a0, j = b0;
    while (true) {
      if (i < a1 && col[i] == la) ++i;
      if (j < b1 && col[j] == lb) ++j;
      if (i >= a1 || j >= b1) return i >= a1 && j >= b1;
      if (col[i] != col[j]) return false;
      ++i;
      ++j;
    }
  }
  bool adjacent = false;
  int64_t i = a0, j = b0;
  while (i < a1 || j < b1) {
    if (i < a1 && col[i] == b) {
      adjacent = true;
      ++i;
      continue;
    }
    if (j < b1 && col[j] == a) {
      ++j;
      continue;
    }
    if (i >= a1 || j >= b1 || col[i] != col[j]) return false;
    ++i;
    ++j;
  }
  return adjacent;
}

// Compare each non-leader with its group leader; mismatches propose the
// smallest mismatching position of the group as the new group's leader.
__global__ __launch_bounds__(kBlock) void k_verify(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   const uint32_t* __restrict__ node, const int64_t* __restrict__ label,
                                                   int64_t n, int mode, int32_t* __restrict__ mism,
                                                   unsigned long long* __restrict__ newlab,
                                                   unsigned long long* __restrict__ n_mism) {
  unsigned long long cnt = 0;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t l = label[p];
    mism[p] = 0;
    if (l == p) continue;
    if (!same_neighbourhood(row_ptr, col, node[p], node[l], mode)) {
      mism[p] = 1;
      atomicMin(&newlab[l], static_cast<unsigned long long>(p));
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

// Group sizes (by leader position).
__global__ __launch_bounds__(kBlock) void k_group_count(const int64_t* __restrict__ label, int64_t n,
                                                        int32_t* __restrict__ gsize) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock)
    atomicAdd(&gsize[label[p]], 1);
}

// Per node: the smallest node of its group (the leader position holds it:
// positions of a run are in ascending node order and split groups are led by
// their smallest position), or -1 for groups of one.
__global__ __launch_bounds__(kBlock) void k_node_labels(const int64_t* __restrict__ label,
                                                        const int32_t* __restrict__ gsize,
                                                        const uint32_t* __restrict__ node, int64_t n,
                                                        int32_t* __restrict__ lab) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t l = label[p];
    lab[node[p]] = gsize[l] >= 2 ? static_cast<int32_t>(node[l]) : -1;
  }
}

// Merge another pass's labels into lab (the kinds are disjoint), marking
// the merged nodes with `kind_id` (1 closed twins, 2 pendant twins, 3 hub
// paths).
__global__ __launch_bounds__(kBlock) void k_merge_labels(int32_t* __restrict__ lab, const int32_t* __restrict__ lab2,
                                                         int64_t n, int kind_id, int32_t* __restrict__ kind) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (lab[i] < 0 && lab2[i] >= 0) {
      lab[i] = lab2[i];
      kind[i] = kind_id;
    }
  }
}

// Pendant twins: the A-class of a B-class is led by its smallest leaf.
__global__ __launch_bounds__(kBlock) void k_pendant_min_leaf(const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ col,
                                                             const int32_t* __restrict__ lab, int64_t n,
                                                             int32_t* __restrict__ amin) {
  for (int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; b < n;
       b += static_cast<int64_t>(gridDim.x) * kBlock)
    if (lab[b] >= 0) atomicMin(&amin[lab[b]], static_cast<int32_t>(pendant_leaf(row_ptr, col, b)));
}

__global__ __launch_bounds__(kBlock) void k_pendant_leaf_labels(const int64_t* __restrict__ row_ptr,
                                                                const int32_t* __restrict__ col,
                                                                int32_t* __restrict__ lab, int64_t n,
                                                                const int32_t* __restrict__ amin) {
  for (int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; b < n;
       b += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (row_ptr[b + 1] - row_ptr[b] < 2) continue;  // leaves are never B's
    const int32_t l = lab[b];
    if (l >= 0) lab[pendant_leaf(row_ptr, col, b)] = amin[l];
  }
}

// Hub-path candidates: key = E * n + F for the end pair E < F of x's path
// (n^2 when x is not the interior of a two-node path), payload x; the side
// (0: next to E) goes to the top bit of the payload-free key order through
// a separate array.
__global__ __launch_bounds__(kBlock) void k_hubpath_keys(const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, int64_t n,
                                                         uint64_t* __restrict__ key, uint32_t* __restrict__ val,
                                                         int32_t* __restrict__ side) {
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; x < n;
       x += static_cast<int64_t>(gridDim.x) * kBlock) {
    uint64_t k = static_cast<uint64_t>(n) * static_cast<uint64_t>(n);
    int32_t sd = 0;
    auto deg = [&](int64_t v) { return row_ptr[v + 1] - row_ptr[v]; };
    if (deg(x) == 2) {
      const int32_t u = col[row_ptr[x]], v = col[row_ptr[x] + 1];
      const bool du = deg(u) == 2, dv = deg(v) == 2;
      if (du != dv) {
        const int32_t y = du ? u : v, e = du ? v : u;
        const int32_t y0 = col[row_ptr[y]], y1 = col[row_ptr[y] + 1];
        const int32_t f = y0 == x ? y1 : y0;
        if (deg(f) != 2 && e != f) {
          const uint64_t lo = static_cast<uint64_t>(e < f ? e : f), hi = static_cast<uint64_t>(e < f ? f : e);
          k = lo * static_cast<uint64_t>(n) + hi;
          sd = e < f ? 0 : 1;
        }
      }
    }
    key[x] = k;
    val[x] = static_cast<uint32_t>(x);
    side[x] = sd;
  }
}

// Runs of equal key (x ascending within a run): with >= 2 paths (>= 4
// nodes), each side forms a class led by its smallest node.  The thread at a
// run's head walks the run.
__global__ __launch_bounds__(kBlock) void k_hubpath_groups(const uint64_t* __restrict__ key,
                                                           const uint32_t* __restrict__ val,
                                                           const int32_t* __restrict__ side, int64_t n,
                                                           int32_t* __restrict__ lab) {
  const uint64_t none = static_cast<uint64_t>(n) * static_cast<uint64_t>(n);
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (key[p] == none || (p > 0 && key[p - 1] == key[p])) continue;
    int64_t e = p;
    while (e + 1 < n && key[e + 1] == key[p]) ++e;
    if (e - p + 1 < 4) continue;  // a single path
    int32_t lead[2] = {-1, -1};
    for (int64_t t = p; t <= e; ++t) {
      const int sd = side[val[t]];
      if (lead[sd] < 0) lead[sd] = static_cast<int32_t>(val[t]);
    }
    for (int64_t t = p; t <= e; ++t) lab[val[t]] = lead[side[val[t]]];
  }
}

__global__ __launch_bounds__(kBlock) void k_leaders(const int32_t* __restrict__ lab, int64_t n,
                                                    int32_t* __restrict__ is_leader, int32_t* __restrict__ cnt) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int32_t l = lab[i];
    is_leader[i] = (l == i) ? 1 : 0;
    if (l >= 0) atomicAdd(&cnt[l], 1);
  }
}

// Class c (classes ordered by leader node): size, removed eigenvalue (0 for
// open twins, -1/d for closed twins of degree d, 1/sqrt(d) for pendant-twin
// classes of degree-d B's, which hold the pair +-1/sqrt(d) with half of the
// class's dimensions each; an A-class leader is a leaf whose neighbour is a
// B; 1/2 for hub-path classes, also paired) and the pair flag.
__global__ __launch_bounds__(kBlock) void k_class_info(const int32_t* __restrict__ is_leader,
                                                       const int32_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ cls_of_node,
                                                       const int32_t* __restrict__ kind,
                                                       const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int64_t n,
                                                       int64_t* __restrict__ sizes, double* __restrict__ lam,
                                                       int32_t* __restrict__ paired) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (!is_leader[i]) continue;
    const int64_t c = cls_of_node[i];
    sizes[c] = cnt[i];
    const int k = kind[i];
    const int64_t d = row_ptr[i + 1] - row_ptr[i];
    double l = 0.0;
    if (k == 1) {
      l = -1.0 / static_cast<double>(d);
    } else if (k == 2) {
      const int64_t db = d >= 2 ? d : row_ptr[col[row_ptr[i]] + 1] - row_ptr[col[row_ptr[i]]];
      l = sqrt(1.0 / static_cast<double>(db));
    } else if (k == 3) {
      l = 0.5;
    }
    lam[c] = l;
    paired[c] = k >= 2 ? 1 : 0;
  }
}

// Sort keys: the class of each member (n_cls for nodes outside the classes),
// node ids as payload; a stable sort then lists every class's members in
// ascending order, classes in leader order.
__global__ __launch_bounds__(kBlock) void k_member_keys(const int32_t* __restrict__ lab,
                                                        const int64_t* __restrict__ cls_of_node, int64_t n,
                                                        int64_t n_cls, uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int32_t l = lab[i];
    keys[i] = static_cast<uint64_t>(l >= 0 ? cls_of_node[l] : n_cls);
    vals[i] = static_cast<uint32_t>(i);
  }
}

// One detection pass: lab[i] = leader node of i's exact group (size >= 2) or -1.
// Detection pass in hash mode `mode` (0 open, 1 closed, 2 pendant twins).
nd_status twin_pass(const nd_graph* g, uint64_t seed, int mode, hipStream_t st, Tmp& t, int32_t* lab) {
  const int64_t n = g->n;
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
                     mode, h, node);
  ND_LAUNCH_CHECK();
  ND_CHECK(radix_sort_u64(h, h2, node, node2, n, 64, st));
  int64_t* label;
  int32_t *mism, *gsize;
  unsigned long long *newlab, *n_mism;
  ND_CHECK(t.get(&label, n));
  ND_CHECK(t.get(&mism, n));
  ND_CHECK(t.get(&gsize, n));
  ND_CHECK(t.get(&newlab, n));
  ND_CHECK(t.get(&n_mism, 1));
  hipLaunchKernelGGL(k_runs, dim3(grid), dim3(kBlock), 0, st, h, n, label);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reset_newlab, dim3(grid), dim3(kBlock), 0, st, n, newlab);
  ND_LAUNCH_CHECK();
  // every iteration splits at least one new exact group off each mixed group,
  // so n iterations always suffice
  for (int64_t iter = 0; iter < n; ++iter) {
    ND_HIP(hipMemsetAsync(n_mism, 0, 8, st));
    hipLaunchKernelGGL(k_verify, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, node, label, n,
                       mode, mism, newlab, n_mism);
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
  ND_HIP(hipMemsetAsync(gsize, 0, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_group_count, dim3(grid), dim3(kBlock), 0, st, label, n, gsize);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_node_labels, dim3(grid), dim3(kBlock), 0, st, label, gsize, node, n, lab);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

// Pendant-twin pass: lab[i] = leader of i's class (the smallest B of the
// group for B's, the smallest leaf for A's) or -1.
nd_status pendant_pass(const nd_graph* g, uint64_t seed, hipStream_t st, Tmp& t, int32_t* lab) {
  const int64_t n = g->n;
  const int grid = grid_for(n, kBlock);
  ND_CHECK(twin_pass(g, seed, 2, st, t, lab));
  int32_t* amin;
  ND_CHECK(t.get(&amin, n));
  ND_HIP(hipMemsetAsync(amin, 0x7F, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_pendant_min_leaf, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, lab, n, amin);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_pendant_leaf_labels, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, lab, n, amin);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

// Hub-path pass: lab[i] = leader of i's class or -1.
nd_status hubpath_pass(const nd_graph* g, hipStream_t st, Tmp& t, int32_t* lab) {
  const int64_t n = g->n;
  const int grid = grid_for(n, kBlock);
  uint64_t *key, *key2;
  uint32_t *val, *val2;
  int32_t* side;
  ND_CHECK(t.get(&key, n));
  ND_CHECK(t.get(&key2, n));
  ND_CHECK(t.get(&val, n));
  ND_CHECK(t.get(&val2, n));
  ND_CHECK(t.get(&side, n));
  ND_HIP(hipMemsetAsync(lab, 0xFF, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_hubpath_keys, dim3(grid), dim3(kBlock), 0, st, g->row_ptr, g->col, n, key, val, side);
  ND_LAUNCH_CHECK();
  const uint64_t none = static_cast<uint64_t>(n) * static_cast<uint64_t>(n);
  int nbits = 0;
  while ((uint64_t(1) << nbits) <= none && nbits < 64) ++nbits;
  ND_CHECK(radix_sort_u64(key, key2, val, val2, n, nbits, st));
  hipLaunchKernelGGL(k_hubpath_groups, dim3(grid), dim3(kBlock), 0, st, key, val, side, n, lab);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

nd_status twins_impl(const nd_graph* g, uint64_t seed, uint32_t kinds, hipStream_t st, nd_motifs* out) {
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
  // per node: leader of its class (-1 outside the classes) and kind
  // (0 open twins, 1 closed twins, 2 pendant twins, 3 hub paths)
  int32_t *lab, *kind, *lab2;
  ND_CHECK(t.get(&lab, n));
  ND_CHECK(t.get(&kind, n));
  ND_CHECK(t.get(&lab2, n));
  ND_HIP(hipMemsetAsync(kind, 0, static_cast<size_t>(n) * 4, st));
  if (kinds & ND_TWINS_OPEN)
    ND_CHECK(twin_pass(g, seed, 0, st, t, lab));
  else
    ND_HIP(hipMemsetAsync(lab, 0xFF, static_cast<size_t>(n) * 4, st));
  if (kinds & ND_TWINS_CLOSED) {
    ND_CHECK(twin_pass(g, seed, 1, st, t, lab2));
    hipLaunchKernelGGL(k_merge_labels, dim3(grid), dim3(kBlock), 0, st, lab, lab2, n, 1, kind);
    ND_LAUNCH_CHECK();
  }
  if (kinds & ND_PENDANTS) {
    ND_CHECK(pendant_pass(g, seed, st, t, lab2));
    hipLaunchKernelGGL(k_merge_labels, dim3(grid), dim3(kBlock), 0, st, lab, lab2, n, 2, kind);
    ND_LAUNCH_CHECK();
  }
  if (kinds & ND_HUBPATHS) {
    ND_CHECK(hubpath_pass(g, st, t, lab2));
    hipLaunchKernelGGL(k_merge_labels, dim3(grid), dim3(kBlock), 0, st, lab, lab2, n, 3, kind);
    ND_LAUNCH_CHECK();
  }
  int32_t *is_leader, *cnt;
  int64_t *cls_of_node, *tot;
  ND_CHECK(t.get(&is_leader, n));
  ND_CHECK(t.get(&cnt, n));
  ND_CHECK(t.get(&cls_of_node, n));
  ND_CHECK(t.get(&tot, 1));
  ND_HIP(hipMemsetAsync(cnt, 0, static_cast<size_t>(n) * 4, st));
  hipLaunchKernelGGL(k_leaders, dim3(grid), dim3(kBlock), 0, st, lab, n, is_leader, cnt);
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
  int64_t* sizes;
  ND_CHECK(t.get(&sizes, n_cls));
  ND_CHECK(dalloc_t(&out->class_lambda, static_cast<size_t>(n_cls)));
  ND_CHECK(dalloc_t(&out->class_paired, static_cast<size_t>(n_cls)));
  hipLaunchKernelGGL(k_class_info, dim3(grid), dim3(kBlock), 0, st, is_leader, cnt, cls_of_node, kind, g->row_ptr,
                     g->col, n, sizes, out->class_lambda, out->class_paired);
  ND_LAUNCH_CHECK();
  ND_CHECK(exclusive_scan_i64(sizes, out->class_ptr, n_cls, tot, st));
  ND_HIP(hipMemcpyAsync(out->class_ptr + n_cls, tot, 8, hipMemcpyDeviceToDevice, st));
  int64_t n_mem = 0;
  ND_HIP(hipMemcpyAsync(&n_mem, tot, 8, hipMemcpyDeviceToHost, st));
  // spikes: total (|C| - 1) per distinct eigenvalue, ascending
  std::vector<int64_t> h_sizes(static_cast<size_t>(n_cls));
  std::vector<double> h_lam(static_cast<size_t>(n_cls));
  std::vector<int32_t> h_pair(static_cast<size_t>(n_cls));
  ND_HIP(hipMemcpyAsync(h_pair.data(), out->class_paired, static_cast<size_t>(n_cls) * 4, hipMemcpyDeviceToHost, st));
  ND_HIP(hipMemcpyAsync(h_sizes.data(), sizes, static_cast<size_t>(n_cls) * 8, hipMemcpyDeviceToHost, st));
  ND_HIP(hipMemcpyAsync(h_lam.data(), out->class_lambda, static_cast<size_t>(n_cls) * 8, hipMemcpyDeviceToHost, st));
  ND_HIP(hipStreamSynchronize(st));
  out->n_members = n_mem;
  // removed dimensions per distinct eigenvalue (multiples of 1/2: exact in
  // any order); a pendant-twin class holds half of its dimensions at each of +-h
  std::map<double, double> acc;
  for (int64_t c = 0; c < n_cls; ++c) {
    const double dims = static_cast<double>(h_sizes[c] - 1);
    if (h_pair[c]) {
      acc[h_lam[c]] += 0.5 * dims;
      acc[-h_lam[c]] += 0.5 * dims;
    } else {
      acc[h_lam[c]] += dims;
    }
  }
  for (const auto& kv : acc) {
    out->spike_lambda.push_back(kv.first);
    out->spike_weight.push_back(kv.second / static_cast<double>(n));
  }
  const size_t ns = out->spike_lambda.size();
  ND_CHECK(dalloc_t(&out->spikes_d, 2 * ns));
  ND_HIP(hipMemcpyAsync(out->spikes_d, out->spike_lambda.data(), ns * 8, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(out->spikes_d + ns, out->spike_weight.data(), ns * 8, hipMemcpyHostToDevice, st));
  // members: stable sort of the nodes by class
  uint64_t *keys, *keys2;
  uint32_t *vals, *vals2;
  ND_CHECK(t.get(&keys, n));
  ND_CHECK(t.get(&keys2, n));
  ND_CHECK(t.get(&vals, n));
  ND_CHECK(t.get(&vals2, n));
  hipLaunchKernelGGL(k_member_keys, dim3(grid), dim3(kBlock), 0, st, lab, cls_of_node, n, n_cls, keys, vals);
  ND_LAUNCH_CHECK();
  int nbits = 0;
  while ((uint64_t(1) << nbits) <= static_cast<uint64_t>(n_cls)) ++nbits;
  ND_CHECK(radix_sort_u64(keys, keys2, vals, vals2, n, nbits, st));
  ND_CHECK(dalloc_t(&out->members, static_cast<size_t>(n_mem)));
  ND_HIP(hipMemcpyAsync(out->members, vals, static_cast<size_t>(n_mem) * 4, hipMemcpyDeviceToDevice, st));
  ND_HIP(hipStreamSynchronize(st));
  return ND_OK;
}

}  // namespace
}  // namespace nd

nd_motifs::~nd_motifs() {
  nd::dfree(class_ptr);
  nd::dfree(members);
  nd::dfree(class_lambda);
  nd::dfree(class_paired);
  nd::dfree(spikes_d);
}

extern "C" {

nd_status nd_motif_filter(const nd_graph* g, uint64_t seed, uint32_t kinds, void* stream, nd_motifs** out) {
  nd::clear_error();
  ND_REQUIRE(out != nullptr, "nd_motif_filter: out is NULL");
  *out = nullptr;
  ND_REQUIRE(g != nullptr, "nd_motif_filter: graph is NULL");
  if (kinds == 0 || (kinds & ~(ND_TWINS_OPEN | ND_TWINS_CLOSED | ND_PENDANTS | ND_HUBPATHS)) != 0) {
    nd::set_error("nd_motif_filter: kinds=0x%x; implemented: ND_TWINS_OPEN, ND_TWINS_CLOSED, ND_PENDANTS, "
                  "ND_HUBPATHS", kinds);
    return ND_EUNSUPPORTED;
  }
  std::unique_ptr<nd_motifs> m(new nd_motifs());
  ND_HIP(hipGetDevice(&m->device));
  ND_CHECK(nd::twins_impl(g, seed, kinds, nd::as_stream(stream), m.get()));
  *out = m.release();
  return ND_OK;
}

nd_status nd_motif_info(const nd_motifs* m, int64_t* n_classes, int64_t* n_motif_nodes, int32_t* n_spikes,
                        double* spike_lambda, double* spike_weight) {
  nd::clear_error();
  ND_REQUIRE(m != nullptr, "nd_motif_info: motifs is NULL");
  if (n_classes) *n_classes = m->n_classes;
  if (n_motif_nodes) *n_motif_nodes = m->n_members;
  const size_t ns = m->spike_lambda.size();
  if (n_spikes) *n_spikes = static_cast<int32_t>(ns);
  for (size_t s = 0; s < ns; ++s) {
    if (spike_lambda) spike_lambda[s] = m->spike_lambda[s];
    if (spike_weight) spike_weight[s] = m->spike_weight[s];
  }
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

nd_status nd_motif_export_lambda(const nd_motifs* m, double* class_lambda, int32_t* class_paired) {
  nd::clear_error();
  ND_REQUIRE(m != nullptr, "nd_motif_export_lambda: motifs is NULL");
  ND_HIP(hipDeviceSynchronize());
  if (m->n_classes && class_lambda)
    ND_HIP(hipMemcpy(class_lambda, m->class_lambda, static_cast<size_t>(m->n_classes) * 8, hipMemcpyDeviceToHost));
  if (m->n_classes && class_paired)
    ND_HIP(hipMemcpy(class_paired, m->class_paired, static_cast<size_t>(m->n_classes) * 4, hipMemcpyDeviceToHost));
  return ND_OK;
}

void nd_motifs_free(nd_motifs* m) { delete m; }

}  // extern "C"
