/*
 * nd.h -- C ABI of the MI355X (gfx950) network density-of-states library.
 *
 * The library computes, on one GPU, the kernel-polynomial-method (KPM)
 * estimates of the spectral density of a graph's normalized adjacency
 * H = D^{-1/2} A D^{-1/2}, following Dong, Benson & Bindel, "Network Density
 * of States", KDD 2019:
 *
 *   - graph and operator: Sec. 2.1 (adjacency, degrees, normalized adjacency);
 *   - DOS / LDOS and their Chebyshev moments: Sec. 2.2 (eqn dos, eqn ldos),
 *     Sec. 3.1 (eq. cheb_3term, eqn doscoeff, eqn pdoscoeff);
 *   - stochastic trace / diagonal estimation with a block of probes:
 *     Sec. 3.1 (eq. probe_trace, eq. probe_diag);
 *   - motif (twin) detection by hashing and probe projection: Sec. 3.4;
 *   - Gauss quadrature and Lanczos (GQL) for the DOS: Sec. 3.2;
 *   - Jackson-damped reconstruction and spectral histograms: Sec. 2.2
 *     (eqn reg_dos and the histogram that follows it), Sec. 3.1 (eqn orth),
 *     Sec. 4.1 (Jackson's theorem).
 *
 * Conventions
 *   - Every entry point returns an nd_status; no exception crosses the ABI.
 *     On a non-OK status nd_last_error() returns a thread-local message.
 *     Inputs are validated before any kernel is launched.
 *   - "device" pointers are HIP device memory on the current device (e.g. a
 *     torch tensor's data_ptr()); "host" pointers are ordinary host memory.
 *     All output buffers are owned by the caller.  Opaque handles (nd_graph,
 *     nd_motifs) are owned by the library and released only by nd_*_free.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Moment and
 *     reconstruction calls are asynchronous on it.  Calls that must size
 *     allocations (nd_build_csr, nd_motif_filter) or fill host outputs
 *     (nd_*_info, nd_*_export) synchronise the stream before returning.
 *   - A graph handle keeps a workspace (probe blocks, recurrence state,
 *     partial sums) that grows on demand; calls that use the same graph
 *     handle must not overlap in time (on different streams or threads).
 *   - Device memory the library allocates comes from a per-device cache:
 *     memory released by nd_*_free (or by a workspace that grows) is kept
 *     for reuse until the process ends, up to ND_POOL_BYTES (default 32 GiB)
 *     of unused blocks; a block is handed out again only after the device has
 *     finished all queued work, and the cache is emptied when an allocation
 *     fails.  ND_ALLOC_LIMIT_BYTES caps the size of any single allocation.
 *   - Results are deterministic: the same (graph, seed, flags, sizes) give
 *     bit-identical outputs on the same device.  No floating-point atomics.
 *   - Node ids: the builder drops isolated nodes and renumbers the survivors
 *     0..N-1 in ascending order of their input id; every per-node array below
 *     (probes, LDOS rows, features) is indexed by that compact id.
 */
#ifndef ND_H_
#define ND_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ND_OK = 0,
  ND_EINVAL = -1,        /* bad argument (null pointer, size, id out of range) */
  ND_ENOMEM = -2,        /* device allocation failed or exceeded ND_ALLOC_LIMIT_BYTES */
  ND_EDEVICE = -3,       /* a HIP runtime call failed */
  ND_EOVERFLOW = -4,     /* a size exceeds what the index types hold */
  ND_EUNSUPPORTED = -5   /* valid request the library does not implement */
} nd_status;

typedef struct nd_graph nd_graph;   /* device CSR of the simple symmetric graph */
typedef struct nd_motifs nd_motifs; /* twin classes found in a graph */

/* ------------------------------------------------------------------ flags */
#define ND_INPUT_DEVICE 0x1u      /* nd_build_csr: src/dst are device pointers */

#define ND_PROBE_RADEMACHER 0x0u  /* probes with i.i.d. +/-1 entries (default) */
#define ND_PROBE_GAUSSIAN 0x1u    /* probes with i.i.d. standard normal entries */
#define ND_STATE_FP64 0x2u        /* run the recurrence in fp64 instead of fp32 */
#define ND_TIME_STEPS 0x4u        /* time each sparse-product step launch with HIP events
                                     (read back with nd_graph_step_timing; adds a
                                     host synchronisation at the end of the call) */
#define ND_MOMENT_DOUBLING 0x8u   /* nd_cheb_moments only: moments 2s-1 and 2s from
                                     Y_s.Y_{s-1} and Y_s.Y_s (floor(M/2) sparse
                                     products instead of M-1) */

#define ND_TWINS_OPEN 0x1u        /* nd_motif_filter: nodes with equal open neighbourhoods */
#define ND_TWINS_CLOSED 0x2u      /* nd_motif_filter: adjacent nodes with equal closed
                                     neighbourhoods N(i) + {i} */
#define ND_PENDANTS 0x4u          /* nd_motif_filter: pendant twins, nodes with one private
                                     leaf and equal remaining neighbourhoods */
#define ND_HUBPATHS 0x8u          /* nd_motif_filter: >= 2 two-node paths between the same
                                     two nodes */

#define ND_KERNEL_NONE 0u         /* nd_reconstruct: plain truncated series */
#define ND_KERNEL_JACKSON 1u      /* nd_reconstruct: Jackson damping factors */
#define ND_SPIKES_IN_MOMENTS 0x10u /* nd_reconstruct: the moments include the spikes;
                                     subtract w T_m(lambda) before the smooth part */

/* --------------------------------------------------------------- graph */

/* Build the graph of Sec. 2.1 from an undirected edge list.
 *   n_nodes  ids in src/dst must lie in [0, n_nodes); 1 <= n_nodes < 2^31.
 *   n_edges  number of input edges, 0 <= n_edges < 2^31.
 *   src,dst  int32 [n_edges] endpoints; host pointers, or device pointers
 *            with ND_INPUT_DEVICE.  Read only; not retained.
 * The edge list is symmetrised and read as a set: duplicate edges collapse
 * to weight 1 and self-loops are dropped (the paper's operators are built
 * from the 0/1 pattern here; weighted input is not supported).  Nodes of
 * degree 0 are dropped (D^{-1/2} is undefined there) and the rest renumbered
 * in ascending input-id order.  Rows list their columns in ascending order.
 * The stored per-node scale is fp32(1/sqrt(d)) with the inverse square root
 * taken in fp64.  On success *out owns the device CSR.
 * Errors: ND_EINVAL (null pointer, id out of range, bad size), ND_ENOMEM,
 * ND_EDEVICE.  Synchronises `stream`. */
nd_status nd_build_csr(int64_t n_nodes, int64_t n_edges, const int32_t* src, const int32_t* dst,
                       uint32_t flags, void* stream, nd_graph** out);

/* Sizes of a built graph (host outputs; any may be NULL). */
nd_status nd_graph_info(const nd_graph* g, int64_t* n, int64_t* nnz, int64_t* max_deg);

/* Copy the CSR to host buffers (any may be NULL): row_ptr int64 [n+1],
 * col int32 [nnz], old_id int32 [n] (input id of each compact node),
 * dinv_sqrt float [n].  Synchronous. */
nd_status nd_graph_export(const nd_graph* g, int64_t* row_ptr, int32_t* col, int32_t* old_id,
                          float* dinv_sqrt);

/* Device views of the CSR arrays (valid until nd_graph_free); any may be NULL. */
nd_status nd_graph_device_arrays(const nd_graph* g, const int64_t** row_ptr, const int32_t** col,
                                 const float** dinv_sqrt);

/* Total HIP-event time (ms) and count of the sparse-product step launches of
 * the last nd_cheb_moments / nd_ldos_moments call made with ND_TIME_STEPS. */
nd_status nd_graph_step_timing(const nd_graph* g, double* total_ms, int64_t* launches);

void nd_graph_free(nd_graph* g);

/* --------------------------------------------------------------- motifs */

/* Twin detection (Sec. 3.4 and its motif figure).  Nodes whose open
 * neighbourhoods are equal share the localized eigenvectors e_i - e_j with
 * eigenvalue 0 (the paper's node copies).  Adjacent nodes whose closed
 * neighbourhoods N(i) + {i} are equal have a common degree d and share
 * eigenvectors e_i - e_j with eigenvalue -1/d (the blade motif at -1/2 and
 * the -1/m family: an edge attached through the same m-1 nodes).  A node
 * cannot have twins of both kinds, so the classes never overlap.
 * Pendant twins (ND_PENDANTS; the figure's panels at +-1/sqrt(2) and, on the
 * right, +-1/2): c >= 2 nodes B of degree d >= 2 that each carry exactly one
 * leaf A and share the rest of their neighbourhood give two classes, the B's
 * and the A's, whose differences carry c-1 eigenvalues at +1/sqrt(d) and c-1
 * at -1/sqrt(d) (d = 2: pendant paths E - B - A on one node E).  Candidates
 * are grouped by the same hash-and-verify scheme on N(B) minus the leaf.
 * Pendant-twin nodes are never twins.
 * Hub paths (ND_HUBPATHS; the figure's left panel at +-1/2): c >= 2 paths
 * E - X - Y - F between the same two distinct nodes (deg X = deg Y = 2, no
 * other degree-2 neighbour) give two classes, the nodes next to the smaller
 * end and the others, carrying c-1 eigenvalues at +1/2 and c-1 at -1/2.
 * Candidates come from a random hash of each neighbourhood,
 * h_i = sum_{j in N(i)} r_j (+ r_i for closed neighbourhoods) over Z/2^64 with
 * seeded random r (the paper hashes with w = Hz); every candidate class is
 * then confirmed by exact comparison of sorted neighbour lists, so the
 * partition does not depend on the seed.
 *   kinds  any non-empty combination of ND_TWINS_OPEN, ND_TWINS_CLOSED,
 *          ND_PENDANTS, ND_HUBPATHS.
 * Output classes (size >= 2) are in canonical order: by smallest member,
 * members ascending.  Synchronises `stream`.
 * Errors: ND_EINVAL, ND_EUNSUPPORTED (other kinds), ND_ENOMEM, ND_EDEVICE. */
nd_status nd_motif_filter(const nd_graph* g, uint64_t seed, uint32_t kinds, void* stream,
                          nd_motifs** out);

/* Counts and spikes (host outputs; any may be NULL).  A twin class C removes
 * |C|-1 eigenvalues at lambda_C (0 or -1/d); a pendant-twin class removes
 * (|C|-1)/2 at each of +-1/sqrt(d), a hub-path class (|C|-1)/2 at each of
 * +-1/2.  The spikes are the distinct removed eigenvalues
 * in ascending order, each with its removed count over N (a fraction of the
 * DOS mass).  spike_lambda/spike_weight need room
 * for *n_spikes entries: call once with them NULL to learn the count. */
nd_status nd_motif_info(const nd_motifs* m, int64_t* n_classes, int64_t* n_motif_nodes,
                        int32_t* n_spikes, double* spike_lambda, double* spike_weight);

/* Host copies: class_ptr int64 [n_classes+1], members int32 [n_motif_nodes]. */
nd_status nd_motif_export(const nd_motifs* m, int64_t* class_ptr, int32_t* members);

/* Host copies (either may be NULL) of each class's removed eigenvalue,
 * class_lambda double [n_classes]: 0 for open twins, -1/d for closed twins of
 * degree d, 1/sqrt(d) for pendant-twin classes (B's of degree d), 1/2 for
 * hub-path classes; and class_paired int32 [n_classes]: 1 for pendant-twin
 * and hub-path classes (half of the class's removed dimensions at
 * +class_lambda, half at -class_lambda), else 0. */
nd_status nd_motif_export_lambda(const nd_motifs* m, double* class_lambda, int32_t* class_paired);

void nd_motifs_free(nd_motifs* m);

/* --------------------------------------------------------------- probes */

/* Write the probe block the moment calls use (for inspection and tests):
 * Z device [n][n_probes] (node-major, fp32 values; with ND_STATE_FP64 the
 * buffer is double).  Probe j, node i: SplitMix64 (Steele, Lea & Flood 2014)
 * as a counter-based generator -- output n >= 1 of the stream seeded with s is
 * mix(s + n*0x9E3779B97F4A7C15); probe j's stream is seeded with output j+1 of
 * the stream seeded with `seed`; Rademacher takes the sign from the top bit of
 * output i+1, Gaussian applies Box-Muller to outputs 2i+1, 2i+2 (53-bit
 * uniforms) and rounds to fp32.  With `motifs` the block is projected
 * (Sec. 3.4, Z_r = P P^T Z): each twin class's rows replaced by their mean. */
nd_status nd_make_probes(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes,
                         uint64_t seed, uint32_t flags, void* Z, void* stream);

/* --------------------------------------------------------------- moments */

/* Global DOS moments (Sec. 3.1, eqn doscoeff with eq. probe_trace):
 *   mu_pp[j][m] = (1/N) z_j^T T_m(H) z_j,  mu[m] = mean_j mu_pp[j][m],
 * m = 0..n_moments-1 (n_moments-1 sparse products per probe), by the
 * three-term recurrence (eq. cheb_3term) applied to the whole probe block.
 *   n_probes >= 1 (any count; blocks of up to 64 run one after another)
 *   n_moments >= 1
 *   flags    ND_PROBE_RADEMACHER | ND_PROBE_GAUSSIAN, optionally ND_STATE_FP64,
 *            ND_TIME_STEPS, ND_MOMENT_DOUBLING.  With ND_MOMENT_DOUBLING the
 *            same estimates come from floor(M/2) products through the
 *            identities T_s T_{s-1} = (T_{2s-1} + T_1)/2 and
 *            T_s^2 = (T_{2s} + T_0)/2 (the cited KPM review's doubling trick):
 *              mu_pp[j][2s]   = (2/N) y_s.y_s - mu_pp[j][0],
 *              mu_pp[j][2s-1] = (2/N) y_s.y_{s-1} - mu_pp[j][1],
 *            y_s = T_s(H) z_j; equal to the direct sums in exact arithmetic.
 *   motifs   NULL, or twin classes to filter: the probes are projected and
 *            mu/mu_pp hold the moments of the remaining (smooth) spectrum;
 *            the full-DOS moments are mu[m] + sum_s w_s T_m(lambda_s) over
 *            the spikes (lambda_s, w_s) of nd_motif_info.
 *   mu       device double [n_moments]
 *   mu_pp    device double [n_probes][n_moments], or NULL
 * The recurrence state is fp32 (fp64 with ND_STATE_FP64); every moment is
 * accumulated in fp64 with compensated sums in a fixed order. */
nd_status nd_cheb_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes,
                          int32_t n_moments, uint64_t probe_seed, uint32_t flags, double* mu,
                          double* mu_pp, void* stream);

/* nd_cheb_moments without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as nd_cheb_moments
 * (bit-identical), without motif filtering and without ND_TIME_STEPS.
 * Every buffer the kernels need besides the inputs and outputs (recurrence
 * state, probe sign words, moment partials, and the per-probe moments when
 * mu_pp is NULL) lives in one fixed device workspace of 64 MiB that the
 * library holds on each GPU it runs on until the process ends; the
 * recurrence state alone takes 3 x N x padded probes x 4 bytes (8 with
 * ND_STATE_FP64), so this serves graphs up to roughly 340k nodes at 16
 * probes or 85k nodes at 64.
 * Preconditions: an earlier allocating call (nd_cheb_moments or
 * nd_ldos_moments) with the same probe count has run on this graph (it
 * builds the graph's row schedule, which this call only reads).
 * Calls on one GPU share its workspace and leave their data in it: calls
 * that overlap in time on one GPU (different streams, or host threads)
 * race and must be serialised by the caller.  Nothing in the workspace needs
 * to start at zero (every buffer is written before it is read).
 * Errors: ND_EINVAL for a workspace need above 64 MiB (message states the
 * need), a graph without a schedule for this probe count, ND_TIME_STEPS,
 * or any argument error of nd_cheb_moments; no call fails for lack of
 * memory. */
nd_status nd_cheb_moments_noalloc(const nd_graph* g, int32_t n_probes, int32_t n_moments,
                                  uint64_t probe_seed, uint32_t flags, double* mu, double* mu_pp,
                                  void* stream);

/* Per-node LDOS / PDOS moments (Sec. 3.1, eqn pdoscoeff with eq. probe_diag):
 *   ldos[i][m] = (1/k) sum_j v_ijm,   v_ijm = z_ij (T_m(H) z_j)_i,
 * row-major [N][n_moments] (the matrix C of the paper's Algorithm 1 output).
 *   cv_g     NULL, or device float [N][n_moments]: a diagonal control variate
 *            g; then v_ijm = g_im + z_ij ((T_m(H) - diag g_m) z_j)_i, which
 *            is unbiased for any g (with +/-1 probes it equals the plain
 *            estimate exactly).  Not combined with motif filtering: the
 *            projected probe of a class member has E[z~_i^2] = 1/|C|, so
 *            g (1 - z~_i^2) would bias that row.  A cv_g together with
 *            motifs that hold classes is rejected with ND_EINVAL.
 *   motifs   NULL, or twin classes: probes projected as in nd_cheb_moments,
 *            and each class member i gets the removed part back exactly,
 *            ldos[i][m] += (1 - 1/|C|) T_m(lambda_C) (the mean of T_m(+-lambda_C)
 *            for pendant-twin classes), so rows stay unbiased
 *            (mu then includes sum_s w_s T_m(lambda_s) over the spikes).
 *   ldos     device double [N][n_moments]
 *   ldos_sq  NULL, or device double [N][n_moments]: (1/k) sum_j v_ijm^2,
 *            for the per-probe variance ldos_sq - ldos^2.
 *   mu       NULL, or device double [n_moments]: mean over nodes of ldos.
 * Workspace: besides the recurrence state, the graph keeps a staging block of
 * up to 32 launches' LDOS terms (8 bytes per node and launch, twice with
 * ldos_sq, at most 1 GiB); the output rows are written 32 moments at a time.
 * Errors: ND_EINVAL for NULL ldos, a graph without nodes, foreign motifs,
 * cv_g with twin classes, unknown flags or ND_MOMENT_DOUBLING (global
 * moments only); ND_ENOMEM when
 * the workspace cannot be allocated. */
nd_status nd_ldos_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes,
                          int32_t n_moments, uint64_t probe_seed, uint32_t flags,
                          const float* cv_g, double* ldos, double* ldos_sq, double* mu,
                          void* stream);

/* Exact PDOS moments of selected nodes (eqn pdoscoeff): for each listed node
 * v, pdos[i][m] = T_m(H)_vv = e_v^T T_m(H) e_v, from the same recurrence run
 * on unit probes (64 nodes per block of the probe block), m = 0..M-1.  The
 * paper obtains accurate PDOS for a node subset by nested dissection
 * (Sec. 3.3, Algorithm 1); this computes the same quantity directly, at the
 * cost of one probe column per node, with no partitioning.
 *   nodes   device int32 [n_nodes], compact node ids (duplicates allowed)
 *   flags   optionally ND_STATE_FP64, ND_TIME_STEPS
 *   pdos    device double [n_nodes][n_moments]
 * Synchronises `stream` once to validate the ids (ND_EINVAL when out of
 * range). */
nd_status nd_pdos_nodes(const nd_graph* g, const int32_t* nodes, int32_t n_nodes, int32_t n_moments, uint32_t flags,
                        double* pdos, void* stream);

/* Exact PDOS moments of every node by nested dissection (Sec. 3.3,
 * Algorithm 1, eqn ndchebsep): a nested-dissection tree of the graph, then
 * for every tree node the columns of T_m(H) at its separator restricted to
 * its partition, by the block recurrence with the couplings through the
 * ancestors' separators; the diagonals give T_m(H)_vv for all v.
 * The tree comes from recursive bisection (components split with an empty
 * separator; a connected partition takes the smaller of a BFS-level
 * separator and a multilevel one: heavy-edge coarsening, greedy growing,
 * Fiduccia-Mattheyses refinement, minimum vertex cover of the cut edges),
 * stopping at partitions of at most leaf_size nodes; see nd_nested_tree.
 * Block entries are fp64.
 *   n_moments    >= 1
 *   leaf_size    1..4096
 *   max_entries  cap on the total block entries sum_t |I_p| |I_s| (two fp64
 *                buffers of that size are allocated)
 *   flags        optionally ND_TIME_STEPS (per-moment launches)
 *   pdos         device double [N][n_moments], row-major
 *   stats        host int64 [4] or NULL: tree nodes, depth, separator
 *                nodes, block entries (left unset when the call fails)
 * Synchronises `stream`.  ND_EUNSUPPORTED when the graph has no small
 * separators: a partition over 4096 nodes without a separator, or more
 * block entries than max_entries (the tree build stops as soon as its
 * running count passes the cap; partitions over 4 M nodes are split by
 * BFS levels only). */
nd_status nd_pdos_nested(const nd_graph* g, int32_t n_moments, int32_t leaf_size, int64_t max_entries,
                         uint32_t flags, double* pdos, int64_t* stats, void* stream);

/* The nested-dissection tree of nd_pdos_nested on the host, for inspection
 * (Sec. 3.3, Algorithm 1's partition step; no device work).
 *   row_ptr, col  host CSR of a symmetric graph without self loops, n nodes
 *   owner    host int32 [n] or NULL: the tree node whose separator (or leaf)
 *            holds each node
 *   parent   host int32 [2n] or NULL: parent[t] of every tree node t
 *            (-1 for the root); tree nodes number fewer than 2n
 *   stats    host int64 [4] or NULL: as nd_pdos_nested
 * Every edge joins two nodes whose owners lie on one root-to-leaf path.
 * Errors: ND_EINVAL (arguments), ND_EUNSUPPORTED (a partition over 4096
 * nodes that no separator splits). */
nd_status nd_nested_tree(const int64_t* row_ptr, const int32_t* col, int64_t n, int32_t leaf_size,
                         int32_t* owner, int32_t* parent, int64_t* stats);

/* --------------------------------------------------------------- GQL */

/* Gauss quadrature and Lanczos (Sec. 3.2).  For every probe z_j (the same
 * probes as nd_cheb_moments: seed, flags, projection with `motifs`), K =
 * n_steps Lanczos steps on H from v_1 = z_j/|z_j| (three-term recurrence, no
 * reorthogonalization) give the tridiagonal Gamma (diagonal alpha, off-
 * diagonal beta); its eigenvalues tau_i and squared first eigenvector
 * components p_1i^2 form the K-node Gauss rule of the measure
 * sum_i (q_i^T z_j)^2 delta(lambda - lambda_i), so that
 *   (1/k) sum_j sum_i weights[j][i] delta(lambda - nodes[j][i])
 * estimates the DOS (Chebyshev moments equal to the KPM estimates of the
 * same probes up to degree 2K-1).
 *   n_steps  1..4096
 *   flags    ND_PROBE_RADEMACHER | ND_PROBE_GAUSSIAN, optionally ND_STATE_FP64
 *            (fp64 Lanczos vectors), ND_TIME_STEPS
 *   nodes    device double [n_probes][n_steps]: tau (unordered within a probe)
 *   weights  device double [n_probes][n_steps]: p_1i^2 |z_j|^2 / N
 *   steps    device int32 [n_probes] or NULL: steps taken; a probe stops
 *            early when beta falls below 1e-10 (1e-5 with fp32 vectors): an
 *            invariant subspace, where the rule is exact; entries past it
 *            are 0
 *   alpha, beta  device double [n_probes][n_steps] or NULL: the Lanczos
 *            coefficients (beta[j][i] couples steps i and i+1)
 * With motifs, the rule describes the smooth part; the spikes of
 * nd_motif_info carry the removed mass.  Synchronises `stream`.
 * Errors: ND_EINVAL (arguments), ND_EDEVICE (device failure or a tridiagonal
 * eigenproblem that did not converge), ND_ENOMEM. */
nd_status nd_gql(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_steps,
                 uint64_t probe_seed, uint32_t flags, double* nodes, double* weights, int32_t* steps,
                 double* alpha, double* beta, void* stream);

/* PDOS by GQL (Sec. 3.2 with z = e_v): for each listed node v, the K-node
 * Gauss rule of the measure sum_i q_i(v)^2 delta(lambda - lambda_i) (its
 * weights sum to 1), from K = n_steps Lanczos steps started at e_v.  Its
 * Chebyshev moments are the exact PDOS moments T_m(H)_vv for m <= 2K-1.
 *   vertices  device int32 [n_vertices], compact node ids
 *   flags     optionally ND_STATE_FP64, ND_TIME_STEPS
 *   nodes, weights, steps  as in nd_gql, one row per listed node.
 * Synchronises `stream`; ND_EINVAL for ids out of range. */
nd_status nd_gql_pdos(const nd_graph* g, const int32_t* vertices, int32_t n_vertices, int32_t n_steps,
                      uint32_t flags, double* nodes, double* weights, int32_t* steps, void* stream);

/* From the rules of nd_gql (device arrays [n_probes][n_steps]): Chebyshev
 * moments mu[m] = (1/k) sum_j sum_i w_ji T_m(tau_ji), m < n_moments (device
 * double, or NULL), and/or the histogram of the point masses over n_bins
 * equal bins of [lo, hi] (half-open except the last; device double
 * [n_bins], or NULL).  Nodes are clamped to [-1, 1], the interval holding
 * the spectrum of H, first.  Asynchronous on `stream`. */
nd_status nd_gql_density(const double* nodes, const double* weights, int32_t n_probes, int32_t n_steps,
                         int32_t n_moments, double* mu, int32_t n_bins, double lo, double hi, double* hist,
                         void* stream);

/* --------------------------------------------------------------- reconstruction */

/* Densities from moments (fp64), for each of n_rows moment vectors
 * mu device double [n_rows][n_moments]:
 *   series  rho(x) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi sqrt(1-x^2))
 *           (eqn orth / eqn doscoeff), g_m the Jackson factors for M moments
 *           g_m = [(M-m+1) cos(pi m/(M+1)) + sin(pi m/(M+1)) cot(pi/(M+1))]/(M+1)
 *           (ND_KERNEL_JACKSON) or 1 (ND_KERNEL_NONE);
 *   hist    device double [n_rows][n_bins] or NULL: exact integral of rho over
 *           n_bins equal bins of [lo, hi] (-1 <= lo < hi <= 1), bins half-open
 *           [e_b, e_{b+1}) except the last, plus point masses spike_weight[s]
 *           at spike_lambda[s] (host arrays of n_spikes entries, may be 0);
 *   rho     device double [n_rows][n_points] or NULL: rho at the Chebyshev
 *           nodes x_k = cos(pi (k + 1/2) / n_points), k = 0..n_points-1.
 * With ND_SPIKES_IN_MOMENTS in `kernel`, the rows hold the moments of the
 * point masses too: sum_s spike_weight[s] T_m(spike_lambda[s]) is taken out
 * before the series, so hist is the smooth part's plus the exact masses and
 * rho is the smooth part's density.
 * Errors: ND_EINVAL for null pointers or sizes outside the ranges above
 * (n_bins, n_points in 1..4096, n_spikes in 0..1024); ND_ENOMEM / ND_EDEVICE
 * from the device.  The call synchronises the stream before it returns
 * (it releases its temporary tables). */
nd_status nd_reconstruct(const double* mu, int64_t n_rows, int32_t n_moments, uint32_t kernel,
                         const double* spike_lambda, const double* spike_weight, int32_t n_spikes,
                         int32_t n_bins, double lo, double hi, double* hist, int32_t n_points,
                         double* rho, void* stream);

/* --------------------------------------------------------------- learned control variate */
/* Not in the paper.  A per-node MLP 5 -> 128 -> 128 -> n_out (ReLU, ReLU,
 * linear) predicts the first n_out PDOS moments; its output is the cv_g of
 * nd_ldos_moments.  Parameters are a flat float vector laid out
 * [W1 (5 x 128 row-major, in x out), b1, W2 (128 x 128), b2, W3 (128 x n_out), b3].
 * n_out must be 1..128. */

/* Node features feat device float [N][5]: log1p of (degree, mean neighbour
 * degree, max neighbour degree, local clustering 2t/(d(d-1)) (0 if d < 2),
 * number of nodes at distance exactly 2).  If mean/std (device float [5])
 * are given, each column is then standardised as (x - mean) / std.
 * Cost O(d_i + sum_{j in N(i)} d_j) per node.  Neighbourhood bitmaps live in
 * LDS up to N = 524288 and otherwise in a temporary device workspace of at
 * most 4 GiB (2 x N bits per block, fewer blocks for larger graphs);
 * ND_EUNSUPPORTED only if one block's bitmaps exceed that. */
nd_status nd_node_features(const nd_graph* g, const float* mean, const float* std, float* feat,
                           void* stream);

/* Exact diagonal of the first Chebyshev polynomials of H (Sec. 3.1; the
 * exactly known part of a diagonal control variate).  For every node i and
 * m < n_cols (1..4): cv_g[i * ld + m] = T_m(H)_ii, i.e.
 *   T_0: 1;  T_1: 0 (no self loops);  T_2: 2 sum_{j in N(i)} 1/(d_i d_j) - 1;
 *   T_3: 4 sum_{j in N(i)} sum_{k in N(i) & N(j)} 1/(d_i d_j d_k).
 * cv_g is device float [N][ld] (compact node order), typically an MLP
 * output whose first columns this overwrites.  Sums in fp64, fixed order.
 * Same workspace as nd_node_features.  Errors: ND_EINVAL for n_cols outside
 * 1..4 or ld < n_cols. */
nd_status nd_cv_exact_diag(const nd_graph* g, float* cv_g, int64_t ld, int32_t n_cols, void* stream);

/* The motif part of the diagonal (Sec. 3.4): for every member i of a class
 * C of `motifs` and m < n_cols,
 *   cv_g[i * ld + m] += scale (1 - 1/|C|) T_m(lambda_C)
 * (paired classes: T_m(lambda_C) at even m only), the exact contribution of
 * the class's removed eigenvectors to T_m(H)_ii -- the same term
 * nd_ldos_moments adds back to filtered per-node moments.  A control variate
 * uses it to split g into this exactly known part and a learned remainder
 * (scale -1 on training targets, +1 on the prediction).  cv_g: device float
 * [N][ld], compact node order.  Errors: ND_EINVAL for n_cols < 1 or
 * ld < n_cols. */
nd_status nd_motif_diag(const nd_motifs* motifs, float* cv_g, int64_t ld, int32_t n_cols, double scale,
                        void* stream);

/* Per-probe variance of per-node estimates (not in the paper; the figure of
 * merit of a control variate): from one run's ldos and ldos_sq
 * (nd_ldos_moments, device double [n][n_moments]) with k = n_probes >= 2,
 *   s2_im = k/(k-1) (ldos_sq_im - ldos_im^2),
 * out[0] = mean over nodes and m in [m_lo, n_moments) of s2 (device double),
 * per_m (device double [n_moments] or NULL) = mean over nodes for each m.
 * Fixed-order sums.  n_moments <= 1024.  Probes needed for a target
 * variance v: out[0] / v. */
nd_status nd_ldos_variance(const double* ldos, const double* ldos_sq, int64_t n, int32_t n_moments,
                           int32_t m_lo, int32_t n_probes, double* out, double* per_m, void* stream);

/* Column statistics of x device float [n_rows][n_cols] (n_cols <= 16):
 * mean[c] and std[c] = sqrt(max(E[x^2] - mean^2, 1e-12)) as device floats,
 * from fp64 sums in a fixed order. */
nd_status nd_column_stats(const float* x, int64_t n_rows, int32_t n_cols, float* mean, float* std,
                          void* stream);

/* g device float [n][n_out] = MLP(params, feat [n][5]). */
nd_status nd_mlp_forward(const float* params, const float* feat, int64_t n, int32_t n_out,
                         float* g, void* stream);

/* Loss and gradient of mean((MLP(feat[idx]) - target[idx])^2) over the
 * batch rows and the n_out outputs.  idx device int32 [n] (rows of feat and
 * target, which have ld_target columns) or NULL for rows 0..n-1.
 * grad device float [n_params], loss device float [1].  Sums over rows are
 * fixed-order (deterministic). */
nd_status nd_mlp_grad(const float* params, const float* feat, const float* target,
                      int32_t ld_target, const int32_t* idx, int64_t n, int32_t n_out,
                      float* grad, float* loss, void* stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * correction with step count t >= 1) on device float arrays of n_params.
 * nd_mlp_grad and nd_adam_step keep a library-owned scratch buffer for the
 * per-block gradient partials: calls must not overlap in time. */
nd_status nd_adam_step(float* params, float* m, float* v, const float* grad, int64_t n_params,
                       int32_t t, float lr, void* stream);

/* Thread-local message for the last non-OK status ("" if none). */
const char* nd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ND_H_ */
