// Nested dissection for the PDOS (Sec. 3.3, Algorithm 1): exact PDOS moments
// of every node from block recurrences on a nested-dissection tree.
//
// Tree: every tree node t owns a partition I_p (its nodes and all below it)
// and a separator I_s (leaves: I_s = I_p).  Removing I_s splits I_p into the
// children's partitions, which share no edge.  For the columns of T_m(H) at
// the separator nodes, restricted to the partition, eqn ndchebsep gives
//   T_{m+1}(I_p, I_s) = 2 H(I_p, I_p) T_m(I_p, I_s) - T_{m-1}(I_p, I_s)
//                      + 2 sum_{t' ancestor of t} H(I_p, I_s') T_m(I_s', I_s),
// where T_m(I_s', I_s) = T_m(I_s, I_s')^T is a block of the ancestor's own
// columns (rows I_s lie in the ancestor's partition).  Every node is in
// exactly one separator (or leaf), so the diagonals of these blocks are the
// PDOS moments T_m(H)_vv of all nodes.
//
// The partition is built on the host by recursive bisection on BFS level
// structures (a separator is the part of one BFS level, from a
// pseudo-peripheral node of the partition, that touches the next level,
// chosen small among the levels near the middle; components split with an
// empty separator).  This is a simple stand-in for the
// multilevel partitioner the paper uses; it finds small separators on
// graphs with low-dimensional structure (lattices, trees, rings, road-like
// graphs) and fails cleanly (ND_EUNSUPPORTED) when the dense blocks would
// exceed the requested size.  The recurrences run on the GPU in fp64: one
// thread per block entry, all blocks of a moment in one launch.
#include <algorithm>
#include <cmath>
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

struct TreeNode {
  std::vector<int32_t> part, sep;  // sorted node lists
  int depth = 0;
};

// BFS inside the nodes with mark == id, from src: dist (global array, -1 for
// unreached) and the visit order.
void bfs(const std::vector<int64_t>& rp, const std::vector<int32_t>& col, const std::vector<int32_t>& mark, int id,
         int32_t src, std::vector<int32_t>& dist, std::vector<int32_t>& order) {
  order.clear();
  order.push_back(src);
  dist[src] = 0;
  for (size_t h = 0; h < order.size(); ++h) {
    const int32_t v = order[h];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int32_t u = col[e];
      if (mark[u] == id && dist[u] < 0) {
        dist[u] = dist[v] + 1;
        order.push_back(u);
      }
    }
  }
}

// Builds the tree.  Returns false (message set) when a partition that cannot
// be split stays larger than max_leaf.
bool build_tree(const std::vector<int64_t>& rp, const std::vector<int32_t>& col, int64_t n, int leaf_size,
                int max_leaf, std::vector<TreeNode>& tree) {
  std::vector<int32_t> mark(static_cast<size_t>(n), -1), dist(static_cast<size_t>(n), -1), order;
  struct Job {
    std::vector<int32_t> nodes;
    int depth;
  };
  std::vector<Job> stack;
  {
    Job root;
    root.nodes.resize(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) root.nodes[static_cast<size_t>(i)] = static_cast<int32_t>(i);
    root.depth = 0;
    stack.push_back(std::move(root));
  }
  while (!stack.empty()) {
    Job job = std::move(stack.back());
    stack.pop_back();
    std::sort(job.nodes.begin(), job.nodes.end());
    const int id = static_cast<int>(tree.size());
    tree.emplace_back();
    tree[id].part = job.nodes;
    tree[id].depth = job.depth;
    const auto& P = tree[id].part;
    const size_t np = P.size();
    if (static_cast<int64_t>(np) <= leaf_size) {
      tree[id].sep = P;
      continue;
    }
    for (int32_t v : P) {
      mark[v] = id;
      dist[v] = -1;
    }
    bfs(rp, col, mark, id, P[0], dist, order);
    if (order.size() < np) {
      // disconnected: empty separator, one child per component
      std::vector<Job> comps;
      comps.push_back({order, job.depth + 1});
      for (int32_t v : P) {
        if (dist[v] >= 0) continue;
        bfs(rp, col, mark, id, v, dist, order);
        comps.push_back({order, job.depth + 1});
      }
      for (auto& c : comps) stack.push_back(std::move(c));
      continue;
    }
    // pseudo-peripheral start: BFS again from the last node reached
    const int32_t far = order.back();
    for (int32_t v : P) dist[v] = -1;
    bfs(rp, col, mark, id, far, dist, order);
    const int n_levels = dist[order.back()] + 1;
    if (n_levels < 3) {
      if (static_cast<int64_t>(np) > max_leaf) {
        set_error("nd_pdos_nested: a partition of %zu nodes has no separator (diameter %d); the graph has no "
                  "small separators", np, n_levels - 1);
        return false;
      }
      tree[id].sep = P;
      continue;
    }
    // a level's separator is only its nodes with a neighbour one level
    // further out; the others join the inner side (they touch no outer node)
    auto reaches_out = [&](int32_t v) {
      for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
        if (mark[col[e]] == id && dist[col[e]] == dist[v] + 1) return true;
      return false;
    };
    std::vector<int64_t> cnt(static_cast<size_t>(n_levels), 0), cut(static_cast<size_t>(n_levels), 0);
    for (int32_t v : P) {
      cnt[static_cast<size_t>(dist[v])]++;
      if (reaches_out(v)) cut[static_cast<size_t>(dist[v])]++;
    }
    // the smallest cut among the levels that leave >= 1/4 of the nodes on
    // each side; else the level where the cumulative count crosses the middle
    int best = -1;
    int64_t below = cnt[0];
    for (int l = 1; l < n_levels - 1; ++l) {
      const int64_t above = static_cast<int64_t>(np) - below - cnt[static_cast<size_t>(l)];
      if (4 * below >= static_cast<int64_t>(np) && 4 * above >= static_cast<int64_t>(np) &&
          (best < 0 || cut[static_cast<size_t>(l)] < cut[static_cast<size_t>(best)]))
        best = l;
      below += cnt[static_cast<size_t>(l)];
    }
    if (best < 0) {
      int64_t c = 0;
      best = n_levels - 2;
      for (int l = 0; l < n_levels - 1; ++l) {
        c += cnt[static_cast<size_t>(l)];
        if (2 * c >= static_cast<int64_t>(np)) {
          best = l < 1 ? 1 : l;
          break;
        }
      }
    }
    Job left{{}, job.depth + 1}, right{{}, job.depth + 1};
    for (int32_t v : P) {
      const int l = dist[v];
      if (l == best && reaches_out(v))
        tree[id].sep.push_back(v);
      else if (l <= best)
        left.nodes.push_back(v);
      else
        right.nodes.push_back(v);
    }
    std::sort(tree[id].sep.begin(), tree[id].sep.end());
    stack.push_back(std::move(left));
    stack.push_back(std::move(right));
  }
  return true;
}

// Block entry e -> (tree node, local row, local column).
__device__ inline int64_t find_block(const int64_t* __restrict__ off, int64_t T, int64_t e) {
  int64_t lo = 0, hi = T;  // off[lo] <= e < off[lo+1]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

struct NestedArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  int64_t n, T, E;
  const int64_t* off;       // [T+1] first block entry of each tree node
  const int64_t* part_ptr;  // [T+1] into part
  const int32_t* part;
  const int64_t* sep_ptr;   // [T+1] into sep
  const int32_t* sep;
  const int32_t* depth;     // [T]
  const int32_t* loc;       // [(max_depth+1) * n]: row of v in its partition at that depth, or -1
  const int32_t* owner;     // [n] tree node whose separator holds v
  const int32_t* sidx;      // [n] index of v in that separator
};

// B0 = T_0(H) = I on the blocks.
__global__ __launch_bounds__(kBlock) void k_nd_init(NestedArgs a, double* __restrict__ B) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < a.E;
       e += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t t = find_block(a.off, a.T, e);
    const int64_t S = a.sep_ptr[t + 1] - a.sep_ptr[t];
    const int64_t r = (e - a.off[t]) / S, c = (e - a.off[t]) % S;
    B[e] = a.part[a.part_ptr[t] + r] == a.sep[a.sep_ptr[t] + c] ? 1.0 : 0.0;
  }
}

// One moment: Bio (T_{m-1} in, T_{m+1} out, entrywise in place) from Bcur.
__global__ __launch_bounds__(kBlock) void k_nd_step(NestedArgs a, const double* __restrict__ Bcur,
                                                    double* __restrict__ Bio, int first) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < a.E;
       e += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t t = find_block(a.off, a.T, e);
    const int64_t S = a.sep_ptr[t + 1] - a.sep_ptr[t];
    const int64_t r = (e - a.off[t]) / S, c = (e - a.off[t]) % S;
    const int32_t v = a.part[a.part_ptr[t] + r];
    const int32_t sc = a.sep[a.sep_ptr[t] + c];
    const int dt = a.depth[t];
    const double hv = 1.0 / sqrt(static_cast<double>(a.row_ptr[v + 1] - a.row_ptr[v]));
    double acc = 0.0;
    for (int64_t q = a.row_ptr[v]; q < a.row_ptr[v + 1]; ++q) {
      const int32_t k = a.col[q];
      const double hk = hv / sqrt(static_cast<double>(a.row_ptr[k + 1] - a.row_ptr[k]));
      const int32_t lk = a.loc[static_cast<int64_t>(dt) * a.n + k];
      double tk;
      if (lk >= 0) {
        tk = Bcur[a.off[t] + static_cast<int64_t>(lk) * S + c];  // T_m(k, sc), own block
      } else {
        // k lies in an ancestor's separator: T_m(k, sc) = T_m(sc, k) from its block
        const int32_t tp = a.owner[k];
        const int64_t Sp = a.sep_ptr[tp + 1] - a.sep_ptr[tp];
        const int32_t lsc = a.loc[static_cast<int64_t>(a.depth[tp]) * a.n + sc];
        tk = Bcur[a.off[tp] + static_cast<int64_t>(lsc) * Sp + a.sidx[k]];
      }
      acc += hk * tk;
    }
    Bio[e] = first ? acc : 2.0 * acc - Bio[e];
  }
}

// pdos[v][m] = T_m(H)_vv from the block of v's separator.
__global__ __launch_bounds__(kBlock) void k_nd_diag(NestedArgs a, const double* __restrict__ B, int M, int m,
                                                    double* __restrict__ pdos) {
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; v < a.n;
       v += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int32_t t = a.owner[v];
    const int64_t S = a.sep_ptr[t + 1] - a.sep_ptr[t];
    const int32_t lv = a.loc[static_cast<int64_t>(a.depth[t]) * a.n + v];
    pdos[v * M + m] = B[a.off[t] + static_cast<int64_t>(lv) * S + a.sidx[v]];
  }
}

}  // namespace
}  // namespace nd

extern "C" nd_status nd_pdos_nested(const nd_graph* g, int32_t n_moments, int32_t leaf_size, int64_t max_entries,
                                    uint32_t flags, double* pdos, int64_t* stats, void* stream) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(g != nullptr && g->n > 0, "nd_pdos_nested: empty graph");
  ND_REQUIRE(n_moments >= 1, "nd_pdos_nested: n_moments=%d", n_moments);
  ND_REQUIRE(leaf_size >= 1 && leaf_size <= 4096, "nd_pdos_nested: leaf_size=%d not in [1, 4096]", leaf_size);
  ND_REQUIRE(max_entries >= 1, "nd_pdos_nested: max_entries=%lld", (long long)max_entries);
  ND_REQUIRE((flags & ~ND_TIME_STEPS) == 0, "nd_pdos_nested: flags 0x%x (only ND_TIME_STEPS applies)", flags);
  ND_REQUIRE(pdos != nullptr, "nd_pdos_nested: pdos is NULL");
  int dev = -1;
  ND_HIP(hipGetDevice(&dev));
  ND_REQUIRE(dev == g->device, "nd_pdos_nested: graph lives on device %d, current device is %d", g->device, dev);
  hipStream_t st = as_stream(stream);
  const int64_t n = g->n;
  // host copy of the pattern for the partitioner
  std::vector<int64_t> rp(static_cast<size_t>(n + 1));
  std::vector<int32_t> col(static_cast<size_t>(g->nnz));
  ND_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, st));
  ND_HIP(hipMemcpyAsync(col.data(), g->col, col.size() * 4, hipMemcpyDeviceToHost, st));
  ND_HIP(hipStreamSynchronize(st));
  std::vector<TreeNode> tree;
  // a partition that cannot be split may stay dense up to this size
  const int max_leaf = 4096;
  if (!build_tree(rp, col, n, leaf_size, max_leaf, tree)) return ND_EUNSUPPORTED;
  const int64_t T = static_cast<int64_t>(tree.size());
  int max_depth = 0;
  int64_t E = 0, sep_total = 0;
  std::vector<int64_t> off(static_cast<size_t>(T + 1)), part_ptr(static_cast<size_t>(T + 1)),
      sep_ptr(static_cast<size_t>(T + 1));
  for (int64_t t = 0; t < T; ++t) {
    const auto& tn = tree[static_cast<size_t>(t)];
    max_depth = std::max(max_depth, tn.depth);
    off[static_cast<size_t>(t)] = E;
    E += static_cast<int64_t>(tn.part.size()) * static_cast<int64_t>(tn.sep.size());
    part_ptr[static_cast<size_t>(t + 1)] = part_ptr[static_cast<size_t>(t)] + static_cast<int64_t>(tn.part.size());
    sep_ptr[static_cast<size_t>(t + 1)] = sep_ptr[static_cast<size_t>(t)] + static_cast<int64_t>(tn.sep.size());
    if (tn.sep.size() != tn.part.size()) sep_total += static_cast<int64_t>(tn.sep.size());
  }
  off[static_cast<size_t>(T)] = E;
  if (stats) {
    stats[0] = T;
    stats[1] = max_depth;
    stats[2] = sep_total;
    stats[3] = E;
  }
  if (E > max_entries) {
    set_error("nd_pdos_nested: the blocks need %lld entries, more than max_entries=%lld", (long long)E,
              (long long)max_entries);
    return ND_EUNSUPPORTED;
  }
  // node -> separator owner and index; per-depth local rows
  std::vector<int32_t> part(static_cast<size_t>(part_ptr[static_cast<size_t>(T)])),
      sep(static_cast<size_t>(sep_ptr[static_cast<size_t>(T)])), depth(static_cast<size_t>(T)),
      owner(static_cast<size_t>(n), -1), sidx(static_cast<size_t>(n), -1),
      loc(static_cast<size_t>(max_depth + 1) * static_cast<size_t>(n), -1);
  for (int64_t t = 0; t < T; ++t) {
    const auto& tn = tree[static_cast<size_t>(t)];
    depth[static_cast<size_t>(t)] = tn.depth;
    std::copy(tn.part.begin(), tn.part.end(), part.begin() + part_ptr[static_cast<size_t>(t)]);
    std::copy(tn.sep.begin(), tn.sep.end(), sep.begin() + sep_ptr[static_cast<size_t>(t)]);
    for (size_t r = 0; r < tn.part.size(); ++r)
      loc[static_cast<size_t>(tn.depth) * static_cast<size_t>(n) + static_cast<size_t>(tn.part[r])] =
          static_cast<int32_t>(r);
    for (size_t c = 0; c < tn.sep.size(); ++c) {
      owner[static_cast<size_t>(tn.sep[c])] = static_cast<int32_t>(t);
      sidx[static_cast<size_t>(tn.sep[c])] = static_cast<int32_t>(c);
    }
  }
  for (int64_t v = 0; v < n; ++v)
    ND_REQUIRE(owner[static_cast<size_t>(v)] >= 0, "internal: node %lld in no separator", (long long)v);
  Tmp t;
  int64_t *d_off, *d_pp, *d_sp;
  int32_t *d_part, *d_sep, *d_depth, *d_loc, *d_owner, *d_sidx;
  double *Ba, *Bb;
  ND_CHECK(t.get(&d_off, off.size()));
  ND_CHECK(t.get(&d_pp, part_ptr.size()));
  ND_CHECK(t.get(&d_sp, sep_ptr.size()));
  ND_CHECK(t.get(&d_part, std::max<size_t>(part.size(), 1)));
  ND_CHECK(t.get(&d_sep, std::max<size_t>(sep.size(), 1)));
  ND_CHECK(t.get(&d_depth, depth.size()));
  ND_CHECK(t.get(&d_loc, loc.size()));
  ND_CHECK(t.get(&d_owner, owner.size()));
  ND_CHECK(t.get(&d_sidx, sidx.size()));
  ND_CHECK(t.get(&Ba, static_cast<size_t>(E)));
  ND_CHECK(t.get(&Bb, static_cast<size_t>(E)));
  ND_HIP(hipMemcpyAsync(d_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_pp, part_ptr.data(), part_ptr.size() * 8, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_sp, sep_ptr.data(), sep_ptr.size() * 8, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_part, part.data(), part.size() * 4, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_sep, sep.data(), sep.size() * 4, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_depth, depth.data(), depth.size() * 4, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_loc, loc.data(), loc.size() * 4, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_owner, owner.data(), owner.size() * 4, hipMemcpyHostToDevice, st));
  ND_HIP(hipMemcpyAsync(d_sidx, sidx.data(), sidx.size() * 4, hipMemcpyHostToDevice, st));
  NestedArgs a{g->row_ptr, g->col, n, T, E, d_off, d_pp, d_part, d_sp, d_sep, d_depth, d_loc, d_owner, d_sidx};
  const int ge = grid_for(E, kBlock), gn = grid_for(n, kBlock);
  // Ba holds T_m, Bb T_{m-1} (then T_{m+1}); swap after each step
  hipLaunchKernelGGL(k_nd_init, dim3(ge), dim3(kBlock), 0, st, a, Ba);
  ND_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nd_diag, dim3(gn), dim3(kBlock), 0, st, a, Ba, n_moments, 0, pdos);
  ND_LAUNCH_CHECK();
  std::vector<hipEvent_t> evs;
  struct EvFree {
    std::vector<hipEvent_t>& e;
    ~EvFree() {
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
  } ev_free{evs};
  nd_graph* gm = const_cast<nd_graph*>(g);
  const bool timed = (flags & ND_TIME_STEPS) != 0;
  double *cur = Ba, *io = Bb;
  for (int m = 1; m < n_moments; ++m) {
    if (timed) {
      hipEvent_t e0, e1;
      ND_HIP(hipEventCreate(&e0));
      evs.push_back(e0);
      ND_HIP(hipEventCreate(&e1));
      evs.push_back(e1);
      ND_HIP(hipEventRecord(e0, st));
    }
    hipLaunchKernelGGL(k_nd_step, dim3(ge), dim3(kBlock), 0, st, a, cur, io, m == 1 ? 1 : 0);
    ND_LAUNCH_CHECK();
    if (timed) ND_HIP(hipEventRecord(evs.back(), st));
    std::swap(cur, io);
    hipLaunchKernelGGL(k_nd_diag, dim3(gn), dim3(kBlock), 0, st, a, cur, n_moments, m, pdos);
    ND_LAUNCH_CHECK();
  }
  ND_HIP(hipStreamSynchronize(st));
  if (timed) {
    gm->step_ms = 0.0;
    gm->step_launches = 0;
    for (size_t i = 0; i + 1 < evs.size(); i += 2) {
      float ms = 0.f;
      ND_HIP(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      gm->step_ms += ms;
      gm->step_launches++;
    }
  }
  return ND_OK;
}
