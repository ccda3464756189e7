/*
 * CPU oracle, large-graph leg.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path links or calls this file; the test suite, the scripts that
 * write stored expected values and the benchmark's CPU-baseline leg do.  It
 * shares no code with the GPU library.
 *
 * The numpy/scipy oracle (graph.py, kpm.py) states the same definitions; this
 * plain C version exists because a graph with two billion stored entries does
 * not fit that one's intermediate arrays.  Everything is fp64, computed the
 * obvious way, with OpenMP only over independent rows:
 *
 *  - graph (Sec. 2.1): the input edge list is symmetrised and taken as a set
 *    (duplicates collapse, self-loops dropped); nodes without an edge are
 *    dropped and the survivors relabelled 0..N-1 by ascending original id;
 *    every row lists its columns in ascending order.  Built by a counting
 *    sort on the first endpoint, then a sort and de-duplication of each row.
 *  - operator (Sec. 2.1): H_ij = 1/sqrt(d_i) * 1/sqrt(d_j) on the edges.
 *  - probes (Sec. 3.1): Rademacher entries from SplitMix64 (Steele, Lea and
 *    Flood, OOPSLA 2014) used counter-based: output n >= 1 of the stream
 *    seeded with s is mix(s + n * 0x9E3779B97F4A7C15); probe j's stream is
 *    seeded with output j+1 of the stream seeded with `seed`; entry (j, i) is
 *    -1 when the top bit of output i+1 of probe j's stream is set, else +1.
 *    Or unit probes (column j is e_{node_j}).
 *  - moments (Sec. 3.1, eq. cheb_3term, eqn doscoeff, eqn pdoscoeff,
 *    eq. probe_trace, eq. probe_diag): Y_0 = Z, Y_1 = H Z,
 *    Y_{m+1} = 2 H Y_m - Y_{m-1};  mu_pp[j][m] = (1/N) z_j . y_{m,j} (or
 *    z_j . y_{m,j} for unit probes) and, for the listed rows r,
 *    C[r][m] = (1/k) sum_j z_rj y_{m,rj}.  "M moments" are T_0 .. T_{M-1}.
 *    Sums over nodes are Neumaier-compensated over fixed chunks of rows and
 *    the chunks added in order, so the result does not depend on the thread
 *    count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OCK_GAMMA 0x9E3779B97F4A7C15ULL

typedef struct {
  int64_t n;        /* nodes after dropping isolated ones */
  int64_t nnz;      /* stored entries = 2 |E| */
  int64_t* row_ptr; /* [n+1] */
  int32_t* col;     /* [nnz], ascending within a row */
  int32_t* old_id;  /* [n], original id of each kept node, ascending */
} ock_graph;

static uint64_t ock_splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * OCK_GAMMA;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static double ock_rademacher(uint64_t seed, int64_t j, int64_t i) {
  const uint64_t key = ock_splitmix64(seed, (uint64_t)j + 1);
  return (ock_splitmix64(key, (uint64_t)i + 1) >> 63) ? -1.0 : 1.0;
}

static int cmp_i32(const void* a, const void* b) {
  const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

void ock_free(ock_graph* g) {
  free(g->row_ptr);
  free(g->col);
  free(g->old_id);
  memset(g, 0, sizeof(*g));
}

/* Returns 0 on success, -1 on bad input, -2 when memory runs out. */
int ock_build_csr(int64_t n_nodes, int64_t n_edges, const int32_t* src, const int32_t* dst, ock_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n_nodes < 0 || n_edges < 0) return -1;
  for (int64_t e = 0; e < n_edges; ++e)
    if (src[e] < 0 || dst[e] < 0 || src[e] >= n_nodes || dst[e] >= n_nodes) return -1;
  /* counting sort of both orientations of every non-loop edge by first endpoint */
  int64_t* ptr = calloc((size_t)n_nodes + 1, sizeof(int64_t));
  if (!ptr) return -2;
  for (int64_t e = 0; e < n_edges; ++e)
    if (src[e] != dst[e]) {
      ptr[src[e] + 1]++;
      ptr[dst[e] + 1]++;
    }
  for (int64_t v = 0; v < n_nodes; ++v) ptr[v + 1] += ptr[v];
  const int64_t total = ptr[n_nodes];
  int32_t* adj = malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int64_t* fill = malloc((size_t)(n_nodes > 0 ? n_nodes : 1) * sizeof(int64_t));
  if (!adj || !fill) {
    free(ptr);
    free(adj);
    free(fill);
    return -2;
  }
  memcpy(fill, ptr, (size_t)n_nodes * sizeof(int64_t));
  for (int64_t e = 0; e < n_edges; ++e)
    if (src[e] != dst[e]) {
      adj[fill[src[e]]++] = dst[e];
      adj[fill[dst[e]]++] = src[e];
    }
  /* sort and de-duplicate every row; fill[v] becomes the row's distinct count */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n_nodes; ++v) {
    int32_t* r = adj + ptr[v];
    const int64_t len = ptr[v + 1] - ptr[v];
    qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t w = 0;
    for (int64_t t = 0; t < len; ++t)
      if (w == 0 || r[t] != r[w - 1]) r[w++] = r[t];
    fill[v] = w;
  }
  /* drop isolated nodes, relabel by ascending original id */
  int64_t n = 0;
  for (int64_t v = 0; v < n_nodes; ++v) n += fill[v] > 0;
  int64_t* new_of_old = malloc((size_t)(n_nodes > 0 ? n_nodes : 1) * sizeof(int64_t));
  int32_t* old_id = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t* row_ptr = malloc((size_t)(n + 1) * sizeof(int64_t));
  if (!new_of_old || !old_id || !row_ptr) {
    free(ptr); free(adj); free(fill); free(new_of_old); free(old_id); free(row_ptr);
    return -2;
  }
  int64_t i = 0;
  row_ptr[0] = 0;
  for (int64_t v = 0; v < n_nodes; ++v) {
    new_of_old[v] = -1;
    if (fill[v] > 0) {
      new_of_old[v] = i;
      old_id[i] = (int32_t)v;
      row_ptr[i + 1] = row_ptr[i] + fill[v];
      ++i;
    }
  }
  const int64_t nnz = row_ptr[n];
  /* compact the rows in place (each row moves toward the front) */
  for (int64_t v = 0, at = 0; v < n_nodes; ++v) {
    const int64_t len = fill[v];
    if (len == 0) continue;
    memmove(adj + at, adj + ptr[v], (size_t)len * sizeof(int32_t));
    at += len;
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nnz; ++e) adj[e] = (int32_t)new_of_old[adj[e]];
  int32_t* col = nnz > 0 ? realloc(adj, (size_t)nnz * sizeof(int32_t)) : adj;
  free(ptr);
  free(fill);
  free(new_of_old);
  g->n = n;
  g->nnz = nnz;
  g->row_ptr = row_ptr;
  g->col = col ? col : adj;
  g->old_id = old_id;
  return 0;
}

/* s += x with Neumaier compensation in c */
static void neumaier(double* s, double* c, double x) {
  const double t = *s + x;
  *c += (fabs(*s) >= fabs(x)) ? ((*s - t) + x) : ((x - t) + *s);
  *s = t;
}

#define OCK_CHUNK 65536

/*
 * Stochastic (or unit-probe) Chebyshev moments of g, see the file comment.
 * k probes (1..64); unit_nodes NULL for Rademacher probes from `seed`, else k node
 * ids (column j = e_{unit_nodes[j]}).  mu_pp: [k][M]; rows/ldos: n_rows node
 * ids and their [n_rows][M] per-node moments (ldos may be NULL).
 * Returns 0, -1 on bad input, -2 when memory runs out.
 */
int ock_moments(const ock_graph* g, int32_t k, uint64_t seed, const int64_t* unit_nodes, int32_t M,
                double* mu_pp, int64_t n_rows, const int64_t* rows, double* ldos) {
  const int64_t n = g->n;
  if (n <= 0 || k <= 0 || k > 64 || M <= 0) return -1;
  for (int64_t t = 0; t < n_rows; ++t)
    if (rows[t] < 0 || rows[t] >= n) return -1;
  if (unit_nodes)
    for (int32_t j = 0; j < k; ++j)
      if (unit_nodes[j] < 0 || unit_nodes[j] >= n) return -1;
  const size_t blk = (size_t)n * (size_t)k;
  double* dinv = malloc((size_t)n * sizeof(double));
  double* Z = malloc(blk * sizeof(double));
  double* Yp = malloc(blk * sizeof(double));
  double* Yc = malloc(blk * sizeof(double));
  const int64_t n_chunks = (n + OCK_CHUNK - 1) / OCK_CHUNK;
  double* part = malloc((size_t)n_chunks * (size_t)k * sizeof(double));
  if (!dinv || !Z || !Yp || !Yc || !part) {
    free(dinv); free(Z); free(Yp); free(Yc); free(part);
    return -2;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    dinv[i] = 1.0 / sqrt((double)(g->row_ptr[i + 1] - g->row_ptr[i]));
    for (int32_t j = 0; j < k; ++j) Z[(size_t)i * k + j] = unit_nodes ? 0.0 : ock_rademacher(seed, j, i);
  }
  if (unit_nodes)
    for (int32_t j = 0; j < k; ++j) Z[(size_t)unit_nodes[j] * k + j] = 1.0;
  const double scale = unit_nodes ? 1.0 : 1.0 / (double)n;
  for (int32_t m = 0; m < M; ++m) {
    /* Y_m: Z at m = 0; Yc = H Z at m = 1 (Yp = Z); afterwards
       Yp <- 2 H Yc - Yp, then Yp and Yc swap, so Yc holds Y_m */
    const double* Y = Z;
    if (m >= 1) {
      const double* X = (m == 1) ? Z : Yc;
      double* out = (m == 1) ? Yc : Yp;
#pragma omp parallel for schedule(dynamic, 1024)
      for (int64_t i = 0; i < n; ++i) {
        double acc[64];
        for (int32_t j = 0; j < k; ++j) acc[j] = 0.0;
        for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
          const int64_t c = g->col[e];
          const double h = dinv[i] * dinv[c];
          for (int32_t j = 0; j < k; ++j) acc[j] += h * X[(size_t)c * k + j];
        }
        for (int32_t j = 0; j < k; ++j) {
          const size_t t = (size_t)i * k + j;
          out[t] = (m == 1) ? acc[j] : 2.0 * acc[j] - out[t];
        }
      }
      if (m == 1) {
        memcpy(Yp, Z, blk * sizeof(double));
      } else {
        double* t = Yc;
        Yc = Yp;
        Yp = t;
      }
      Y = Yc;
    }
    /* per-probe sums z_j . y_{m,j}: compensated within fixed chunks, chunks in order */
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
      const int64_t i0 = ch * OCK_CHUNK, i1 = (i0 + OCK_CHUNK < n) ? i0 + OCK_CHUNK : n;
      for (int32_t j = 0; j < k; ++j) {
        double s = 0.0, c = 0.0;
        for (int64_t i = i0; i < i1; ++i) neumaier(&s, &c, Z[(size_t)i * k + j] * Y[(size_t)i * k + j]);
        part[(size_t)ch * k + j] = s + c;
      }
    }
    for (int32_t j = 0; j < k; ++j) {
      double s = 0.0, c = 0.0;
      for (int64_t ch = 0; ch < n_chunks; ++ch) neumaier(&s, &c, part[(size_t)ch * k + j]);
      mu_pp[(size_t)j * M + m] = (s + c) * scale;
    }
    if (ldos)
      for (int64_t t = 0; t < n_rows; ++t) {
        const int64_t i = rows[t];
        double s = 0.0;
        for (int32_t j = 0; j < k; ++j) s += Z[(size_t)i * k + j] * Y[(size_t)i * k + j];
        ldos[(size_t)t * M + m] = s / (double)k;
      }
  }
  free(dinv); free(Z); free(Yp); free(Yc); free(part);
  return 0;
}
