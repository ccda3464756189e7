/*
 * Seeded synthetic graph generators (edge lists only).
 *
 * This module produces the input edge lists that both the GPU library and the
 * CPU oracle consume.  It holds none of the density-of-states arithmetic: no
 * operator, no probes, no moments.  Every generator is deterministic for a
 * given seed, independent of the number of threads.
 *
 * Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: output n (n >= 1) of the stream seeded with s is mix(s + n*gamma).
 *
 * Models:
 *   - Erdos-Renyi G(n, p) by geometric skipping (Batagelj & Brandes, "Efficient
 *     generation of large random networks", Phys. Rev. E 71, 2005).
 *   - Stochastic block model with equal blocks, same skipping per block pair.
 *   - Barabasi-Albert preferential attachment from an (m+1)-clique, each new
 *     node attaching m distinct edges with probability proportional to degree,
 *     plus optional planted pairs of degree-1 leaves sharing a random hub.
 *   - R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004) with quadrant
 *     probabilities (a, b, c, d), optional endpoint reduction modulo n.
 *
 * Ownership: callers pass output buffers and their capacity; each function
 * returns the number of edges it generated (it writes at most `cap` of them),
 * so a caller whose buffer was too small can retry with the returned size.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#define SG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Output n (1-based) of the SplitMix64 stream seeded with s. */
static inline uint64_t sg_out(uint64_t s, uint64_t n) { return sg_mix(s + n * SG_GAMMA); }

typedef struct {
  uint64_t key;
  uint64_t n;
} sg_stream;

static inline sg_stream sg_stream_new(uint64_t seed, uint64_t tag) {
  sg_stream st;
  st.key = sg_out(seed, tag + 1);
  st.n = 0;
  return st;
}
static inline uint64_t sg_next(sg_stream* st) { return sg_out(st->key, ++st->n); }
/* uniform double in [0, 1) from the top 53 bits */
static inline double sg_unit(uint64_t b) { return (double)(b >> 11) * 0x1.0p-53; }
/* uniform integer in [0, n) (multiply-shift; bias below 2^-64 * n) */
static inline uint64_t sg_below(uint64_t b, uint64_t n) {
  return (uint64_t)(((unsigned __int128)b * n) >> 64);
}

static inline void sg_emit(int64_t* m, int64_t cap, int32_t* src, int32_t* dst, int64_t u,
                           int64_t v) {
  if (*m < cap) {
    src[*m] = (int32_t)u;
    dst[*m] = (int32_t)v;
  }
  (*m)++;
}

/* Skip length for a Bernoulli(p) sequence: number of failures before the next
   success, drawn as floor(log(1-r)/log(1-p)). */
static inline int64_t sg_skip(sg_stream* st, double log1mp) {
  double r = sg_unit(sg_next(st));
  return (int64_t)floor(log(1.0 - r) / log1mp);
}

/* All pairs w < v < n of [0, n), each kept with probability p, offset by `off`. */
static void sg_er_block(int64_t n, double p, sg_stream* st, int64_t off, int64_t* m, int64_t cap,
                        int32_t* src, int32_t* dst) {
  if (n < 2 || p <= 0.0) return;
  if (p >= 1.0) {
    for (int64_t v = 1; v < n; ++v)
      for (int64_t w = 0; w < v; ++w) sg_emit(m, cap, src, dst, off + v, off + w);
    return;
  }
  const double lp = log(1.0 - p);
  int64_t v = 1, w = -1;
  while (v < n) {
    w += 1 + sg_skip(st, lp);
    while (w >= v && v < n) {
      w -= v;
      v++;
    }
    if (v < n) sg_emit(m, cap, src, dst, off + v, off + w);
  }
}

/* All pairs (i, j) in [0, na) x [0, nb), kept with probability p. */
static void sg_bip_block(int64_t na, int64_t nb, double p, sg_stream* st, int64_t offa,
                         int64_t offb, int64_t* m, int64_t cap, int32_t* src, int32_t* dst) {
  if (na < 1 || nb < 1 || p <= 0.0) return;
  const int64_t total = na * nb;
  if (p >= 1.0) {
    for (int64_t t = 0; t < total; ++t) sg_emit(m, cap, src, dst, offa + t / nb, offb + t % nb);
    return;
  }
  const double lp = log(1.0 - p);
  int64_t t = -1;
  for (;;) {
    t += 1 + sg_skip(st, lp);
    if (t >= total || t < 0) break;
    sg_emit(m, cap, src, dst, offa + t / nb, offb + t % nb);
  }
}

int64_t sg_er(int64_t n, double p, uint64_t seed, int64_t cap, int32_t* src, int32_t* dst) {
  int64_t m = 0;
  sg_stream st = sg_stream_new(seed, 0x45520000ULL);
  sg_er_block(n, p, &st, 0, &m, cap, src, dst);
  return m;
}

/* Equal-size blocks (the first n % nblocks blocks get one extra node). */
int64_t sg_sbm(int64_t n, int32_t nblocks, double p_in, double p_out, uint64_t seed, int64_t cap,
               int32_t* src, int32_t* dst) {
  if (nblocks < 1) return 0;
  int64_t m = 0;
  int64_t base = n / nblocks, extra = n % nblocks;
  for (int32_t a = 0; a < nblocks; ++a) {
    int64_t na = base + (a < extra), offa = a * base + (a < extra ? a : extra);
    for (int32_t b = a; b < nblocks; ++b) {
      int64_t nb = base + (b < extra), offb = b * base + (b < extra ? b : extra);
      sg_stream st = sg_stream_new(seed, 0x53420000ULL + (uint64_t)a * 4096u + (uint64_t)b);
      if (a == b)
        sg_er_block(na, p_in, &st, offa, &m, cap, src, dst);
      else
        sg_bip_block(na, nb, p_out, &st, offa, offb, &m, cap, src, dst);
    }
  }
  return m;
}

/* Barabasi-Albert: nodes 0..m form a clique; node v > m attaches m distinct
   edges to existing nodes chosen proportionally to degree (uniform pick from
   the list of edge endpoints, repeats rejected).  Then `n_pairs` pairs of new
   leaves (nodes n + 2q, n + 2q + 1) each attach to one hub drawn uniformly from
   [0, n).  The edge count is known in advance:
   m(m+1)/2 + (n-m-1)m + 2 n_pairs.  Returns -1 on bad arguments or when the
   buffers are too small (cap below that count) or allocation fails. */
int64_t sg_ba(int64_t n, int32_t m, int64_t n_pairs, uint64_t seed, int64_t cap, int32_t* src,
              int32_t* dst) {
  if (m < 1 || n < m + 1 || n_pairs < 0) return -1;
  const int64_t n_edges = (int64_t)m * (m + 1) / 2 + (n - m - 1) * (int64_t)m + 2 * n_pairs;
  if (cap < n_edges) return -1;
  int32_t* pool = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n_edges);
  if (!pool) return -1;
  int64_t e = 0, plen = 0;
  for (int32_t u = 0; u <= m; ++u)
    for (int32_t v = 0; v < u; ++v) {
      src[e] = u;
      dst[e] = v;
      e++;
      pool[plen++] = u;
      pool[plen++] = v;
    }
  sg_stream st = sg_stream_new(seed, 0x42410000ULL);
  int32_t chosen[64];
  int32_t* big = NULL;
  int32_t* ch = chosen;
  if (m > 64) {
    big = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    if (!big) {
      free(pool);
      return -1;
    }
    ch = big;
  }
  for (int64_t v = m + 1; v < n; ++v) {
    int32_t got = 0;
    const int64_t plen0 = plen; /* targets drawn from the graph before v joins */
    while (got < m) {
      int32_t t = pool[sg_below(sg_next(&st), (uint64_t)plen0)];
      int dup = 0;
      for (int32_t q = 0; q < got; ++q)
        if (ch[q] == t) {
          dup = 1;
          break;
        }
      if (!dup) ch[got++] = t;
    }
    for (int32_t q = 0; q < m; ++q) {
      src[e] = (int32_t)v;
      dst[e] = ch[q];
      e++;
      pool[plen++] = (int32_t)v;
      pool[plen++] = ch[q];
    }
  }
  sg_stream sp = sg_stream_new(seed, 0x54570000ULL);
  for (int64_t q = 0; q < n_pairs; ++q) {
    int32_t hub = (int32_t)sg_below(sg_next(&sp), (uint64_t)n);
    src[e] = (int32_t)(n + 2 * q);
    dst[e] = hub;
    e++;
    src[e] = (int32_t)(n + 2 * q + 1);
    dst[e] = hub;
    e++;
  }
  free(big);
  free(pool);
  return e;
}

/* R-MAT: n_edges samples over a 2^scale x 2^scale grid.  Each level picks a
   quadrant with probabilities (a, b, c, 1-a-b-c) using 32-bit thresholds; the
   row bit is set for quadrants c and d, the column bit for b and d.  Edge e
   draws its levels from outputs e*T+1 .. e*T+T of one stream (two levels per
   64-bit output), so the result does not depend on the thread count.  With
   n_mod > 0 both endpoints are reduced modulo n_mod. */
void sg_rmat(int32_t scale, int64_t n_edges, double a, double b, double c, uint64_t seed,
             int64_t n_mod, int32_t* src, int32_t* dst) {
  const double two32 = 4294967296.0;
  double fa = a * two32, fab = (a + b) * two32, fabc = (a + b + c) * two32;
  const uint64_t ta = fa >= two32 ? 0xFFFFFFFFull : (uint64_t)fa;
  const uint64_t tab = fab >= two32 ? 0xFFFFFFFFull : (uint64_t)fab;
  const uint64_t tabc = fabc >= two32 ? 0xFFFFFFFFull : (uint64_t)fabc;
  const uint64_t key = sg_out(seed, 0x524D0000ULL + 1);
  const uint64_t T = (uint64_t)(scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n_edges; ++e) {
    uint64_t u = 0, v = 0, bits = 0;
    for (int32_t lvl = 0; lvl < scale; ++lvl) {
      uint64_t r;
      if ((lvl & 1) == 0) {
        bits = sg_out(key, (uint64_t)e * T + (uint64_t)(lvl >> 1) + 1);
        r = bits >> 32;
      } else {
        r = bits & 0xFFFFFFFFull;
      }
      int q = r < ta ? 0 : (r < tab ? 1 : (r < tabc ? 2 : 3));
      u = (u << 1) | (uint64_t)(q >> 1);
      v = (v << 1) | (uint64_t)(q & 1);
    }
    if (n_mod > 0) {
      u %= (uint64_t)n_mod;
      v %= (uint64_t)n_mod;
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
}

/* Watts-Strogatz small world: ring lattice on n nodes where each node links to
   its k/2 nearest neighbours on each side; each lattice edge (u, u+s) is
   rewired with probability p to (u, w) with w uniform over [0, n).  Rewired
   edges may duplicate or self-loop; the graph builder collapses them.
   Returns n * (k/2). */
int64_t sg_ws(int64_t n, int32_t k, double p, uint64_t seed, int64_t cap, int32_t* src,
              int32_t* dst) {
  const int32_t h = k / 2;
  int64_t m = 0;
  sg_stream st = sg_stream_new(seed, 0x57530000ULL);
  for (int32_t s = 1; s <= h; ++s)
    for (int64_t u = 0; u < n; ++u) {
      int64_t v = (u + s) % n;
      if (sg_unit(sg_next(&st)) < p) v = (int64_t)sg_below(sg_next(&st), (uint64_t)n);
      sg_emit(&m, cap, src, dst, u, v);
    }
  return m;
}
