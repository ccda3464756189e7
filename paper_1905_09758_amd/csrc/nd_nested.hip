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
// The partition is built on the host (graph preprocessing, as the paper's
// partitioner call is) by recursive bisection.  Components split with an
// empty separator.  A connected partition gets two candidate separators and
// keeps the smaller one:
//  * a BFS level structure from a pseudo-peripheral node: the part of one
//    level that touches the next, chosen small among the levels that leave a
//    quarter of the nodes on each side (good on lattices, trees, rings);
//  * a multilevel edge bisection -- heavy-edge matching down to ~100
//    vertices, greedy growing from several seeds, Fiduccia-Mattheyses
//    refinement on the way back up -- turned into a vertex separator by a
//    minimum vertex cover of the cut edges (Konig's theorem, from a maximum
//    bipartite matching), which works without any BFS-level structure.
// A partition that neither splits stays a dense leaf up to 4096 nodes; the
// call fails cleanly (ND_EUNSUPPORTED) beyond that, or when the dense blocks
// would exceed the requested size.  The recurrences run on the GPU in fp64:
// one thread per block entry, all blocks of a moment in one launch.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <queue>
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

struct TreeNode {
  std::vector<int32_t> part, sep;  // sorted node lists
  int depth = 0;
  int parent = -1;
};

// ------------------------------------------------------------ multilevel bisection
// A weighted graph in CSR form (vertex weights: merged vertices; edge
// weights: merged edges).
struct WGraph {
  int32_t n = 0;
  std::vector<int32_t> xadj, adj, adjw, vw;
  int64_t total_w = 0;
};

struct Rng {  // xorshift64*: fixed-seed choices, reproducible partitions
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed ? seed : 0x9e3779b97f4a7c15ull) {}
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 0x2545f4914f6cdd1dull;
  }
  int32_t below(int32_t n) { return static_cast<int32_t>(next() % static_cast<uint64_t>(n)); }
};

// Heavy-edge matching: vertices in a random order, each unmatched one with
// its unmatched neighbour of largest edge weight (or alone).  Returns the
// coarse graph and cmap (fine -> coarse).
WGraph coarsen(const WGraph& g, Rng& rng, std::vector<int32_t>& cmap) {
  const int32_t n = g.n;
  std::vector<int32_t> order(static_cast<size_t>(n)), match(static_cast<size_t>(n), -1);
  for (int32_t i = 0; i < n; ++i) order[static_cast<size_t>(i)] = i;
  for (int32_t i = n - 1; i > 0; --i) std::swap(order[static_cast<size_t>(i)], order[static_cast<size_t>(rng.below(i + 1))]);
  cmap.assign(static_cast<size_t>(n), -1);
  int32_t nc = 0;
  for (int32_t u : order) {
    if (match[static_cast<size_t>(u)] >= 0) continue;
    int32_t best = u, bw = -1;
    for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e) {
      const int32_t v = g.adj[static_cast<size_t>(e)];
      if (match[static_cast<size_t>(v)] < 0 && v != u && g.adjw[static_cast<size_t>(e)] > bw) {
        bw = g.adjw[static_cast<size_t>(e)];
        best = v;
      }
    }
    match[static_cast<size_t>(u)] = best;
    match[static_cast<size_t>(best)] = u;
    cmap[static_cast<size_t>(u)] = cmap[static_cast<size_t>(best)] = nc++;
  }
  WGraph c;
  c.n = nc;
  c.vw.assign(static_cast<size_t>(nc), 0);
  c.xadj.assign(static_cast<size_t>(nc) + 1, 0);
  c.total_w = g.total_w;
  std::vector<int32_t> members(static_cast<size_t>(nc) * 2, -1);
  for (int32_t u = 0; u < n; ++u) {
    const int32_t cu = cmap[static_cast<size_t>(u)];
    c.vw[static_cast<size_t>(cu)] += g.vw[static_cast<size_t>(u)];
    members[static_cast<size_t>(cu) * 2 + (members[static_cast<size_t>(cu) * 2] < 0 ? 0 : 1)] = u;
  }
  std::vector<int32_t> slot(static_cast<size_t>(nc), -1);
  for (int32_t cu = 0; cu < nc; ++cu) {
    const size_t start = c.adj.size();
    for (int k = 0; k < 2; ++k) {
      const int32_t u = members[static_cast<size_t>(cu) * 2 + k];
      if (u < 0) continue;
      for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e) {
        const int32_t cv = cmap[static_cast<size_t>(g.adj[static_cast<size_t>(e)])];
        if (cv == cu) continue;
        if (slot[static_cast<size_t>(cv)] < 0) {
          slot[static_cast<size_t>(cv)] = static_cast<int32_t>(c.adj.size());
          c.adj.push_back(cv);
          c.adjw.push_back(0);
        }
        c.adjw[static_cast<size_t>(slot[static_cast<size_t>(cv)])] += g.adjw[static_cast<size_t>(e)];
      }
    }
    for (size_t e = start; e < c.adj.size(); ++e) slot[static_cast<size_t>(c.adj[e])] = -1;
    c.xadj[static_cast<size_t>(cu) + 1] = static_cast<int32_t>(c.adj.size());
  }
  return c;
}

int64_t cut_of(const WGraph& g, const std::vector<uint8_t>& side) {
  int64_t cut = 0;
  for (int32_t u = 0; u < g.n; ++u)
    for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e)
      if (side[static_cast<size_t>(u)] != side[static_cast<size_t>(g.adj[static_cast<size_t>(e)])])
        cut += g.adjw[static_cast<size_t>(e)];
  return cut / 2;
}

// Fiduccia-Mattheyses passes: every vertex may move once per pass; each
// move takes the highest-gain vertex among the tops of the two sides' heaps
// whose move keeps both sides' weights within [lo, hi]; the pass is rolled
// back to its best prefix.  Returns the cut.
int64_t fm_refine(const WGraph& g, std::vector<uint8_t>& side, int64_t lo, int64_t hi, int passes) {
  const int32_t n = g.n;
  std::vector<int64_t> gain(static_cast<size_t>(n));
  int64_t w[2] = {0, 0};
  for (int32_t u = 0; u < n; ++u) w[side[static_cast<size_t>(u)]] += g.vw[static_cast<size_t>(u)];
  int64_t cut = cut_of(g, side);
  std::vector<uint8_t> locked(static_cast<size_t>(n));
  std::vector<int32_t> moved;
  using Heap = std::priority_queue<std::pair<int64_t, int32_t>>;  // (gain, -vertex), lazy invalidation
  for (int pass = 0; pass < passes; ++pass) {
    Heap heap[2];
    for (int32_t u = 0; u < n; ++u) {
      int64_t gn = 0;
      for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e)
        gn += (side[static_cast<size_t>(g.adj[static_cast<size_t>(e)])] != side[static_cast<size_t>(u)])
                  ? g.adjw[static_cast<size_t>(e)] : -g.adjw[static_cast<size_t>(e)];
      gain[static_cast<size_t>(u)] = gn;
      heap[side[static_cast<size_t>(u)]].push({gn, -u});
    }
    std::fill(locked.begin(), locked.end(), 0);
    moved.clear();
    int64_t cur = cut, best = cut;
    size_t best_len = 0;
    for (;;) {
      int32_t cand[2] = {-1, -1};
      for (int sd = 0; sd < 2; ++sd) {
        while (!heap[sd].empty()) {
          const auto [gn, mu] = heap[sd].top();
          const int32_t u = -mu;
          if (locked[static_cast<size_t>(u)] || side[static_cast<size_t>(u)] != sd ||
              gn != gain[static_cast<size_t>(u)]) {
            heap[sd].pop();
            continue;
          }
          const int64_t wu = g.vw[static_cast<size_t>(u)];
          if (w[1 - sd] + wu <= hi && w[sd] - wu >= lo) cand[sd] = u;
          break;
        }
      }
      int sd = -1;
      if (cand[0] >= 0 && (cand[1] < 0 || gain[static_cast<size_t>(cand[0])] >= gain[static_cast<size_t>(cand[1])]))
        sd = 0;
      else if (cand[1] >= 0)
        sd = 1;
      if (sd < 0) break;
      const int32_t u = cand[sd];
      heap[sd].pop();
      const int64_t gn = gain[static_cast<size_t>(u)], wu = g.vw[static_cast<size_t>(u)];
      locked[static_cast<size_t>(u)] = 1;
      side[static_cast<size_t>(u)] = static_cast<uint8_t>(1 - sd);
      w[sd] -= wu;
      w[1 - sd] += wu;
      cur -= gn;
      moved.push_back(u);
      for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e) {
        const int32_t v = g.adj[static_cast<size_t>(e)];
        if (locked[static_cast<size_t>(v)]) continue;
        const int64_t ew = g.adjw[static_cast<size_t>(e)];
        // u left v's side (gain +2w) or joined it (gain -2w)
        gain[static_cast<size_t>(v)] += (side[static_cast<size_t>(v)] == sd) ? 2 * ew : -2 * ew;
        heap[side[static_cast<size_t>(v)]].push({gain[static_cast<size_t>(v)], -v});
      }
      if (cur < best) {
        best = cur;
        best_len = moved.size();
      }
      if (moved.size() > best_len + 64 + static_cast<size_t>(n) / 20) break;  // no recent improvement
    }
    for (size_t k = moved.size(); k > best_len; --k) {  // roll back past the best prefix
      const int32_t u = moved[k - 1];
      const int sd = side[static_cast<size_t>(u)];
      side[static_cast<size_t>(u)] = static_cast<uint8_t>(1 - sd);
      w[sd] -= g.vw[static_cast<size_t>(u)];
      w[1 - sd] += g.vw[static_cast<size_t>(u)];
    }
    if (best >= cut) break;
    cut = best;
  }
  return cut;
}

// Greedy growing from `seed`: side 1 takes vertices in BFS order until it
// holds half the weight.
void grow(const WGraph& g, int32_t seed, std::vector<uint8_t>& side) {
  side.assign(static_cast<size_t>(g.n), 0);
  std::vector<int32_t> q{seed};
  std::vector<uint8_t> seen(static_cast<size_t>(g.n), 0);
  seen[static_cast<size_t>(seed)] = 1;
  int64_t w = 0;
  for (size_t h = 0; h < q.size() && 2 * w < g.total_w; ++h) {
    const int32_t u = q[h];
    side[static_cast<size_t>(u)] = 1;
    w += g.vw[static_cast<size_t>(u)];
    for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e) {
      const int32_t v = g.adj[static_cast<size_t>(e)];
      if (!seen[static_cast<size_t>(v)]) {
        seen[static_cast<size_t>(v)] = 1;
        q.push_back(v);
      }
    }
  }
}

// Edge bisection of a connected graph (unit weights) into side 0 / 1 with
// each side's weight within 45%..55%.
std::vector<uint8_t> multilevel_bisect(const WGraph& g0, uint64_t seed) {
  Rng rng(seed);
  std::vector<WGraph> levels;
  std::vector<std::vector<int32_t>> maps;
  levels.push_back(g0);
  while (levels.back().n > 100 && levels.size() < 40) {
    std::vector<int32_t> cmap;
    WGraph c = coarsen(levels.back(), rng, cmap);
    if (c.n > levels.back().n * 9 / 10) break;
    maps.push_back(std::move(cmap));
    levels.push_back(std::move(c));
  }
  const int64_t W = g0.total_w;
  auto bounds = [&](const WGraph& g, int64_t& lo, int64_t& hi) {
    int64_t maxv = 0;
    for (int32_t u = 0; u < g.n; ++u) maxv = std::max<int64_t>(maxv, g.vw[static_cast<size_t>(u)]);
    const int64_t slack = std::max<int64_t>(W / 20, maxv);
    lo = W / 2 - slack;
    hi = W - lo;
  };
  const WGraph& gc = levels.back();
  int64_t lo, hi;
  bounds(gc, lo, hi);
  std::vector<uint8_t> side, best;
  int64_t best_cut = -1;
  for (int trial = 0; trial < 8; ++trial) {
    grow(gc, rng.below(gc.n), side);
    const int64_t c = fm_refine(gc, side, lo, hi, 8);
    int64_t w1 = 0;
    for (int32_t u = 0; u < gc.n; ++u) w1 += side[static_cast<size_t>(u)] ? gc.vw[static_cast<size_t>(u)] : 0;
    if (w1 < lo || w1 > hi) continue;
    if (best_cut < 0 || c < best_cut) {
      best_cut = c;
      best = side;
    }
  }
  if (best_cut < 0) return {};
  for (size_t l = levels.size() - 1; l > 0; --l) {  // project and refine
    const WGraph& fine = levels[l - 1];
    const std::vector<int32_t>& cmap = maps[l - 1];
    std::vector<uint8_t> fs(static_cast<size_t>(fine.n));
    for (int32_t u = 0; u < fine.n; ++u) fs[static_cast<size_t>(u)] = best[static_cast<size_t>(cmap[static_cast<size_t>(u)])];
    bounds(fine, lo, hi);
    fm_refine(fine, fs, lo, hi, 4);
    best = std::move(fs);
  }
  return best;
}

// Minimum vertex cover of the cut edges between side 0 and side 1 (Konig:
// from a maximum matching of the bipartite cut graph, the side-0 boundary
// vertices not reachable by alternating paths from unmatched side-0 ones,
// plus the side-1 ones that are).  Returns a flag per vertex.
std::vector<uint8_t> cut_cover(const WGraph& g, const std::vector<uint8_t>& side) {
  const int32_t n = g.n;
  std::vector<int32_t> mate(static_cast<size_t>(n), -1), left;
  for (int32_t u = 0; u < n; ++u) {
    if (side[static_cast<size_t>(u)] != 0) continue;
    for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e)
      if (side[static_cast<size_t>(g.adj[static_cast<size_t>(e)])] == 1) {
        left.push_back(u);
        break;
      }
  }
  // augmenting paths by iterative DFS (Kuhn), visit stamps per phase
  std::vector<int32_t> stamp(static_cast<size_t>(n), -1);
  int32_t phase = 0;
  for (int32_t root : left) {
    ++phase;
    // stack of (left vertex, next edge index); parent links through right vertices
    std::vector<std::pair<int32_t, int32_t>> st{{root, g.xadj[static_cast<size_t>(root)]}};
    std::vector<int32_t> via;  // right vertex taken at each level
    bool found = false;
    while (!st.empty() && !found) {
      auto& [u, e] = st.back();
      if (e >= g.xadj[static_cast<size_t>(u) + 1]) {
        st.pop_back();
        if (!via.empty()) via.pop_back();
        continue;
      }
      const int32_t v = g.adj[static_cast<size_t>(e++)];
      if (side[static_cast<size_t>(v)] != 1 || stamp[static_cast<size_t>(v)] == phase) continue;
      stamp[static_cast<size_t>(v)] = phase;
      via.push_back(v);
      if (mate[static_cast<size_t>(v)] < 0) {
        found = true;
      } else {
        const int32_t w = mate[static_cast<size_t>(v)];
        st.push_back({w, g.xadj[static_cast<size_t>(w)]});
      }
    }
    if (found)  // flip the path: st[k].first is matched to via[k]
      for (size_t k = 0; k < via.size(); ++k) {
        mate[static_cast<size_t>(st[k].first)] = via[k];
        mate[static_cast<size_t>(via[k])] = st[k].first;
      }
  }
  // Z: reachable from unmatched left vertices by alternating paths
  std::vector<uint8_t> inZ(static_cast<size_t>(n), 0);
  std::vector<int32_t> q;
  for (int32_t u : left)
    if (mate[static_cast<size_t>(u)] < 0) {
      inZ[static_cast<size_t>(u)] = 1;
      q.push_back(u);
    }
  for (size_t h = 0; h < q.size(); ++h) {
    const int32_t u = q[h];  // a left vertex
    for (int32_t e = g.xadj[static_cast<size_t>(u)]; e < g.xadj[static_cast<size_t>(u) + 1]; ++e) {
      const int32_t v = g.adj[static_cast<size_t>(e)];
      if (side[static_cast<size_t>(v)] != 1 || inZ[static_cast<size_t>(v)]) continue;
      inZ[static_cast<size_t>(v)] = 1;
      const int32_t w = mate[static_cast<size_t>(v)];
      if (w >= 0 && !inZ[static_cast<size_t>(w)]) {
        inZ[static_cast<size_t>(w)] = 1;
        q.push_back(w);
      }
    }
  }
  std::vector<uint8_t> cover(static_cast<size_t>(n), 0);
  for (int32_t u : left)
    if (!inZ[static_cast<size_t>(u)]) cover[static_cast<size_t>(u)] = 1;
  for (int32_t v = 0; v < n; ++v)
    if (side[static_cast<size_t>(v)] == 1 && inZ[static_cast<size_t>(v)]) cover[static_cast<size_t>(v)] = 1;
  return cover;
}

// Vertex separator of the connected partition P (sorted global ids, mark[v]
// == id) from the multilevel edge bisection: sep, left, right (global ids).
// Returns false when a side would be empty.
bool multilevel_separator(const std::vector<int64_t>& rp, const std::vector<int32_t>& col,
                          const std::vector<int32_t>& mark, int id, const std::vector<int32_t>& P,
                          std::vector<int32_t>& lid, std::vector<int32_t>& sep, std::vector<int32_t>& left,
                          std::vector<int32_t>& right) {
  WGraph g;
  g.n = static_cast<int32_t>(P.size());
  for (size_t i = 0; i < P.size(); ++i) lid[static_cast<size_t>(P[i])] = static_cast<int32_t>(i);
  g.xadj.push_back(0);
  for (int32_t v : P) {
    for (int64_t e = rp[static_cast<size_t>(v)]; e < rp[static_cast<size_t>(v) + 1]; ++e) {
      const int32_t u = col[static_cast<size_t>(e)];
      if (mark[static_cast<size_t>(u)] == id) {
        g.adj.push_back(lid[static_cast<size_t>(u)]);
        g.adjw.push_back(1);
      }
    }
    g.xadj.push_back(static_cast<int32_t>(g.adj.size()));
  }
  g.vw.assign(static_cast<size_t>(g.n), 1);
  g.total_w = g.n;
  // four seeds; the smallest separator wins
  std::vector<uint8_t> side, cover;
  size_t best = std::numeric_limits<size_t>::max();
  for (int trial = 0; trial < 4; ++trial) {
    std::vector<uint8_t> sd = multilevel_bisect(g, 0x5eedull + static_cast<uint64_t>(P.size()) * 7919u + P[0] + 104729u * trial);
    if (sd.empty()) continue;
    std::vector<uint8_t> cv = cut_cover(g, sd);
    size_t c = 0;
    for (uint8_t x : cv) c += x;
    if (c < best) { best = c; side = std::move(sd); cover = std::move(cv); }
  }
  for (int32_t v : P) lid[static_cast<size_t>(v)] = -1;
  if (side.empty()) return false;
  sep.clear();
  left.clear();
  right.clear();
  for (size_t i = 0; i < P.size(); ++i) {
    if (cover[i]) sep.push_back(P[i]);
    else if (side[i] == 0) left.push_back(P[i]);
    else right.push_back(P[i]);
  }
  return !left.empty() && !right.empty();
}

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

// BFS-level separator of the connected partition P (mark[v] == id): from a
// pseudo-peripheral node, the part of one level that touches the next,
// chosen smallest among the levels that leave >= 1/4 of the nodes on each
// side.  Returns false when the partition has fewer than three levels.
bool bfs_separator(const std::vector<int64_t>& rp, const std::vector<int32_t>& col, const std::vector<int32_t>& mark,
                   int id, const std::vector<int32_t>& P, std::vector<int32_t>& dist, std::vector<int32_t>& order,
                   std::vector<int32_t>& sep, std::vector<int32_t>& left, std::vector<int32_t>& right) {
  const size_t np = P.size();
  for (int32_t v : P) dist[static_cast<size_t>(v)] = -1;
  bfs(rp, col, mark, id, P[0], dist, order);
  const int32_t far = order.back();
  for (int32_t v : P) dist[static_cast<size_t>(v)] = -1;
  bfs(rp, col, mark, id, far, dist, order);
  const int n_levels = dist[static_cast<size_t>(order.back())] + 1;
  if (n_levels < 3) return false;
  // a level's separator is only its nodes with a neighbour one level
  // further out; the others join the inner side (they touch no outer node)
  auto reaches_out = [&](int32_t v) {
    for (int64_t e = rp[static_cast<size_t>(v)]; e < rp[static_cast<size_t>(v) + 1]; ++e)
      if (mark[static_cast<size_t>(col[static_cast<size_t>(e)])] == id &&
          dist[static_cast<size_t>(col[static_cast<size_t>(e)])] == dist[static_cast<size_t>(v)] + 1)
        return true;
    return false;
  };
  std::vector<int64_t> cnt(static_cast<size_t>(n_levels), 0), cut(static_cast<size_t>(n_levels), 0);
  for (int32_t v : P) {
    cnt[static_cast<size_t>(dist[static_cast<size_t>(v)])]++;
    if (reaches_out(v)) cut[static_cast<size_t>(dist[static_cast<size_t>(v)])]++;
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
  sep.clear();
  left.clear();
  right.clear();
  for (int32_t v : P) {
    const int l = dist[static_cast<size_t>(v)];
    if (l == best && reaches_out(v))
      sep.push_back(v);
    else if (l <= best)
      left.push_back(v);
    else
      right.push_back(v);
  }
  return !left.empty() && !right.empty();
}

// Partitions larger than this are split by BFS levels only (the multilevel
// bisection's coarsening copies the partition's subgraph several times).
constexpr size_t kMaxMultilevel = size_t(1) << 22;

// Builds the tree.  Returns false (message set) when a partition that cannot
// be split stays larger than max_leaf, or as soon as the blocks exceed
// max_entries entries.
bool build_tree(const std::vector<int64_t>& rp, const std::vector<int32_t>& col, int64_t n, int leaf_size,
                int max_leaf, int64_t max_entries, std::vector<TreeNode>& tree) {
  int64_t entries = 0;
  auto add_entries = [&](size_t part, size_t sep) {
    entries += static_cast<int64_t>(part) * static_cast<int64_t>(sep);
    if (entries > max_entries) {
      set_error("nd_pdos_nested: the blocks need more than max_entries=%lld entries", (long long)max_entries);
      return false;
    }
    return true;
  };
  std::vector<int32_t> mark(static_cast<size_t>(n), -1), dist(static_cast<size_t>(n), -1), order;
  std::vector<int32_t> lid(static_cast<size_t>(n), -1);
  struct Job {
    std::vector<int32_t> nodes;
    int depth;
    int parent;
  };
  std::vector<Job> stack;
  {
    Job root;
    root.nodes.resize(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) root.nodes[static_cast<size_t>(i)] = static_cast<int32_t>(i);
    root.depth = 0;
    root.parent = -1;
    stack.push_back(std::move(root));
  }
  std::vector<int32_t> sa, la, ra, sb, lb, rb;
  while (!stack.empty()) {
    Job job = std::move(stack.back());
    stack.pop_back();
    std::sort(job.nodes.begin(), job.nodes.end());
    const int id = static_cast<int>(tree.size());
    tree.emplace_back();
    tree[id].part = job.nodes;
    tree[id].depth = job.depth;
    tree[id].parent = job.parent;
    const auto& P = tree[id].part;
    const size_t np = P.size();
    if (static_cast<int64_t>(np) <= leaf_size) {
      tree[id].sep = P;
      if (!add_entries(np, np)) return false;
      continue;
    }
    for (int32_t v : P) {
      mark[static_cast<size_t>(v)] = id;
      dist[static_cast<size_t>(v)] = -1;
    }
    bfs(rp, col, mark, id, P[0], dist, order);
    if (order.size() < np) {
      // disconnected: empty separator, one child per component
      std::vector<Job> comps;
      comps.push_back({order, job.depth + 1, id});
      for (int32_t v : P) {
        if (dist[static_cast<size_t>(v)] >= 0) continue;
        bfs(rp, col, mark, id, v, dist, order);
        comps.push_back({order, job.depth + 1, id});
      }
      for (auto& c : comps) stack.push_back(std::move(c));
      continue;
    }
    // two candidate separators; keep the smaller.  A BFS-level separator
    // within 2 sqrt(|P|) (the size planar-like graphs admit) is taken as is.
    const bool ok_a = bfs_separator(rp, col, mark, id, P, dist, order, sa, la, ra);
    const bool small_a = ok_a && static_cast<double>(sa.size()) <= 2.0 * std::sqrt(static_cast<double>(np));
    const bool ok_b = !small_a && np <= kMaxMultilevel && multilevel_separator(rp, col, mark, id, P, lid, sb, lb, rb);
    if (!ok_a && !ok_b) {
      if (static_cast<int64_t>(np) > max_leaf) {
        set_error("nd_pdos_nested: a partition of %zu nodes has no separator that splits it; the graph has no "
                  "small separators", np);
        return false;
      }
      tree[id].sep = P;
      if (!add_entries(np, np)) return false;
      continue;
    }
    const bool use_b = ok_b && (!ok_a || sb.size() < sa.size());
    std::vector<int32_t>& sep = use_b ? sb : sa;
    std::vector<int32_t>& left = use_b ? lb : la;
    std::vector<int32_t>& right = use_b ? rb : ra;
    tree[id].sep = sep;
    std::sort(tree[id].sep.begin(), tree[id].sep.end());
    if (!add_entries(np, sep.size())) return false;
    stack.push_back({left, job.depth + 1, id});
    stack.push_back({right, job.depth + 1, id});
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
  if (!build_tree(rp, col, n, leaf_size, max_leaf, max_entries, tree)) return ND_EUNSUPPORTED;
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

extern "C" nd_status nd_nested_tree(const int64_t* row_ptr, const int32_t* col, int64_t n, int32_t leaf_size,
                                    int32_t* owner, int32_t* parent, int64_t* stats) {
  using namespace nd;
  clear_error();
  ND_REQUIRE(row_ptr != nullptr && n >= 1, "nd_nested_tree: empty graph");
  ND_REQUIRE(leaf_size >= 1 && leaf_size <= 4096, "nd_nested_tree: leaf_size=%d not in [1, 4096]", leaf_size);
  ND_REQUIRE(row_ptr[0] == 0, "nd_nested_tree: row_ptr[0] = %lld, expected 0", (long long)row_ptr[0]);
  for (int64_t v = 0; v < n; ++v)
    ND_REQUIRE(row_ptr[v + 1] >= row_ptr[v], "nd_nested_tree: row_ptr decreases at row %lld", (long long)v);
  const int64_t nnz = row_ptr[n];
  ND_REQUIRE(nnz == 0 || col != nullptr, "nd_nested_tree: col is NULL");
  for (int64_t e = 0; e < nnz; ++e)
    ND_REQUIRE(col[e] >= 0 && col[e] < n, "nd_nested_tree: column %d out of range", col[e]);
  std::vector<int64_t> rp(row_ptr, row_ptr + n + 1);
  std::vector<int32_t> cl(col, col + nnz);
  std::vector<TreeNode> tree;
  if (!build_tree(rp, cl, n, leaf_size, 4096, std::numeric_limits<int64_t>::max(), tree)) return ND_EUNSUPPORTED;
  int max_depth = 0;
  int64_t E = 0, sep_total = 0;
  for (size_t t = 0; t < tree.size(); ++t) {
    const auto& tn = tree[t];
    max_depth = std::max(max_depth, tn.depth);
    E += static_cast<int64_t>(tn.part.size()) * static_cast<int64_t>(tn.sep.size());
    if (tn.sep.size() != tn.part.size()) sep_total += static_cast<int64_t>(tn.sep.size());
    if (parent) parent[t] = tn.parent;
    if (owner)
      for (int32_t v : tn.sep) owner[v] = static_cast<int32_t>(t);
  }
  if (stats) {
    stats[0] = static_cast<int64_t>(tree.size());
    stats[1] = max_depth;
    stats[2] = sep_total;
    stats[3] = E;
  }
  return ND_OK;
}
