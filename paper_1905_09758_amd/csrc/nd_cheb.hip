// KPM moments on the device (Sec. 3.1): probe block, optional twin projection
// (Sec. 3.4), the Chebyshev three-term recurrence (eq. cheb_3term) applied to
// the whole block with one sparse product per step, and the fused moment
// reductions of the trace estimator (eq. probe_trace) and the diagonal
// estimator (eq. probe_diag).
//
// The recurrence runs on X_m = D^{-1/2} Y_m, Y_m = T_m(H) Z, which satisfies
//   X_0 = D^{-1/2} Z,  X_1 = D^{-1} A X_0,  X_{m+1} = 2 D^{-1} A X_m - X_{m-1},
// since D^{-1/2} H D^{1/2} = D^{-1} A.  The gathered operand of each step is
// then a plain row of X (no per-neighbour scale), and Y_m = D^{1/2} X_m is
// formed in fp64 only inside the moment reductions.
//
// Layout: probe blocks are node-major [N][kp] (kp = padded probe count, a
// power of two), so the row of X gathered for one neighbour is one contiguous
// kp*sizeof(T)-byte load spread over L = kp*sizeof(T)/16 lanes of 16 bytes.
// X_{m+1} overwrites X_{m-1} in place: row i reads only its own old row.
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "nd_common.h"

namespace nd {
namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
  using type = float4;
};
template <>
struct VecOf<double> {
  using type = double2;
};

template <typename T>
__device__ inline void load16(const T* p, T (&v)[16 / sizeof(T)]) {
  using V = typename VecOf<T>::type;
  const V x = *reinterpret_cast<const V*>(p);
  if constexpr (sizeof(T) == 4) {
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    v[0] = x.x; v[1] = x.y;
  }
}

template <typename T>
__device__ inline void store16(T* p, const T (&v)[16 / sizeof(T)]) {
  using V = typename VecOf<T>::type;
  V x;
  if constexpr (sizeof(T) == 4) {
    x.x = v[0]; x.y = v[1]; x.z = v[2]; x.w = v[3];
  } else {
    x.x = v[0]; x.y = v[1];
  }
  *reinterpret_cast<V*>(p) = x;
}

// Streaming (non-temporal) 16-byte accesses for data touched once per step
// (the X_{m-1} / X_{m+1} rows and the probe rows), so that cache capacity
// stays with the gathered rows of X_m.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ inline void load16_nt(const T* p, T (&v)[16 / sizeof(T)]) {
  if constexpr (sizeof(T) == 4) {
    const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
  } else {
    const f64x2 x = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    v[0] = x[0]; v[1] = x[1];
  }
}

template <typename T>
__device__ inline void store16_nt(T* p, const T (&v)[16 / sizeof(T)]) {
  if constexpr (sizeof(T) == 4) {
    f32x4 x;
    x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
    __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(p));
  } else {
    f64x2 x;
    x[0] = v[0]; x[1] = v[1];
    __builtin_nontemporal_store(x, reinterpret_cast<f64x2*>(p));
  }
}

// Rademacher probe entry (j, node): the sign from the top bit of output
// node+1 of probe j's SplitMix64 stream, which is seeded with output j+1 of
// the stream seeded with `seed` (counter-based, so any row can be
// regenerated in place).
__device__ inline float rademacher_entry(uint64_t seed, int64_t j, int64_t node) {
  const uint64_t key = splitmix64(seed, static_cast<uint64_t>(j) + 1);
  return (splitmix64(key, static_cast<uint64_t>(node) + 1) >> 63) ? -1.0f : 1.0f;
}

// One DPP lane permutation of a double (two 32-bit moves): CTRL 0xB1 and
// 0x4E are the quad permutations [1,0,3,2] and [2,3,0,1] (lane xor 1, xor 2),
// 0x141 mirrors each half row of 8 lanes, 0x140 each row of 16.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                                     static_cast<unsigned>(lo)));
}

// Sum of v over each aligned group of G lanes (G a power of two), every lane
// of a group receiving the sum.  Within 16 lanes the partners come from DPP
// permutations; after the quad steps all lanes of a quad hold the same bits,
// so the mirrors pair each lane with a lane of the neighbouring quad / half
// row exactly as lane xor 4 / xor 8 would.  Wider groups continue with
// LDS-routed lane shuffles.  Every lane of the wavefront must be active.
template <int G>
__device__ inline double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1>(v);
  if constexpr (G >= 4) v += dpp_f64<0x4E>(v);
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);
  if constexpr (G >= 16) v += dpp_f64<0x140>(v);
#pragma unroll
  for (int off = 16; off < G; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Neumaier-compensated accumulation.
__device__ inline void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

struct StepArgs {
  const int64_t* row_ptr;  // internal CSR
  const int32_t* col;
  const int32_t* perm;     // internal row -> compact node id (LDOS / control-variate rows)
  int64_t n;
  int n_bins;
  int bin_log2p[kMaxBins];
  int64_t bin_row_start[kMaxBins + 1];
  int64_t bin_item_start[kMaxBins + 1];
  int64_t n_chunks;        // items [0, n_chunks) are chunks of the split rows
  int64_t n_items;
  const int64_t* split_chunk_ptr;
  const int32_t* chunk_owner;
  int64_t chunk_nnz;
  int64_t n_split;         // split rows are internal rows [0, n_split)
  int slot_nnz;            // nonzeros per slot and gather batch (4 or 8)
  int zmode;               // 0: probe rows read from z; 1: Rademacher rows regenerated;
                           // 2: doubling steps (products of Y_m with Y_m and Y_{m-1}, no probes);
                           // 3: Lanczos steps (per-probe scales, product with the current vector)
  uint64_t seed;           // probe seed and index of this block's first probe (zmode 1)
  int64_t j0;
  const uint64_t* zbits;   // zmode 1: sign bits of the Rademacher probe row, bit j set for -1
  const int32_t* zcls;     // zmode 1 with twin filtering: class of each internal row or -1
  const void* zcls_val;    // [n_classes][kp] projected probe rows of the classes
  void* chunk_part;
  const void* xg;   // X_m, gathered
  void* xio;        // X_{m-1} in, X_{m+1} out
  const void* z;    // probe block in internal row order (projected when filtering)
  int first;        // step m == 1: X_1 = D^{-1} A X_0
  int kp;           // padded probes per row
  int k_batch;      // real probes in this block
  double inv_k;     // 1 / (total probe count over all blocks)
  int m;            // moment index written by this launch
  double* partial;  // [step grid + split_blocks][sums][kp] per-probe partial sums of launch m
  int split_blocks; // grid of the split-row finisher; its slots follow the step kernel's
  double* ldos;     // [n][ld] (compact node order) or null
  double* ldos_sq;  // [n][ld] or null
  double* stage;    // with ldos: [S][n] LDOS terms of S consecutive launches by internal row
  double* stage_sq; // with ldos_sq: the same for the squares
  int stage_pos;    // row of the staging block written by this launch
  int64_t ld;       // leading dimension of ldos / cv_g (= number of moments)
  int accumulate;   // add to ldos instead of overwriting (later probe blocks)
  const float* cv_g;
  const double* lz;  // Lanczos steps: [2][kp] scales of the stored current and previous vectors
};

// Per-probe sums a row epilogue produces: z.Y_m (probe modes), or the two
// products Y_m.Y_{m-1} and Y_m.Y_m of the doubling steps.
template <int ZM>
constexpr int kSums = ZM == 2 ? 2 : 1;

// Modes whose rows need their own entry of the gathered block.
template <int ZM>
constexpr bool kOwnRow = ZM == 2 || ZM == 3;

// Per-row epilogue: given Y_m(i, probes of this lane) in fp64 and the probe
// values z, form the estimator terms v_ij = z_ij y_ij (+ g_im (1 - z_ij^2)
// with a control variate), add them to this lane's per-probe sums (kept in
// LDS: mom[c * kBlock] for probe c of the lane), and write the row's LDOS
// term to the staging block (by internal row, so that the rows of a
// wavefront write one contiguous segment; k_ldos_flush moves a block of
// launches into the [n][M] output).  Called by every lane of the wavefront;
// `own` selects the lanes that hold a row's values.
template <typename T, int L>
__device__ inline void emit_moments(const StepArgs& a, bool own, int64_t r, int64_t node,
                                    const double (&y)[16 / sizeof(T)], const T (&z)[16 / sizeof(T)], int q,
                                    double* mom) {
  constexpr int PPL = 16 / sizeof(T);
  double s1 = 0.0, s2 = 0.0;
  if (own) {
    const double g = a.cv_g ? static_cast<double>(a.cv_g[node * a.ld + a.m]) : 0.0;
#pragma unroll
    for (int c = 0; c < PPL; ++c) {
      const double zc = static_cast<double>(z[c]);
      double v = zc * y[c];
      if (a.cv_g) v += g * (1.0 - zc * zc);
      if (q * PPL + c >= a.k_batch) v = 0.0;
      mom[c * kBlock] += v;
      s1 += v;
      s2 += v * v;
    }
  }
  if (a.ldos) {
    s1 = group_sum<L>(s1);
    if (a.ldos_sq) s2 = group_sum<L>(s2);
    if (own && q == 0) {
      const int64_t t = static_cast<int64_t>(a.stage_pos) * a.n + r;
      a.stage[t] = s1 * a.inv_k;
      if (a.ldos_sq) a.stage_sq[t] = s2 * a.inv_k;
    }
  }
}

// The per-row operands that do not depend on the gathers: X_{m-1}(r), the
// node id and, when probe rows are read (ZM == 0), the probe values; in the
// doubling steps (ZM == 2) the row's own entry of the gathered block X_m.
// Issued before the gathers so that their latency overlaps with them.
template <typename T, int ZM>
struct RowOperands {
  T xp[16 / sizeof(T)];
  T z[ZM == 0 ? 16 / sizeof(T) : 1];
  T xo[kOwnRow<ZM> ? 16 / sizeof(T) : 1];
  uint64_t zw;  // ZM == 1: the row's probe sign bits
  int64_t node;
};

template <typename T, int ZM>
__device__ inline void load_row_operands(const StepArgs& a, bool own, int64_t r, int q, RowOperands<T, ZM>& o) {
  constexpr int PPL = 16 / sizeof(T);
  o.node = 0;
  o.zw = 0;
#pragma unroll
  for (int c = 0; c < PPL; ++c) o.xp[c] = T(0);
  if constexpr (ZM == 0) {
#pragma unroll
    for (int c = 0; c < PPL; ++c) o.z[c] = T(0);
  }
  if constexpr (kOwnRow<ZM>) {
#pragma unroll
    for (int c = 0; c < PPL; ++c) o.xo[c] = T(0);
  }
  if (own) {
    if (!a.first) load16_nt<T>(reinterpret_cast<const T*>(a.xio) + r * a.kp + q * PPL, o.xp);
    if constexpr (!kOwnRow<ZM>) {
      if (a.cv_g) o.node = a.perm[r];
    }
    if constexpr (ZM == 1) o.zw = a.zbits[r];
    if constexpr (ZM == 0) load16_nt<T>(reinterpret_cast<const T*>(a.z) + r * a.kp + q * PPL, o.z);
    if constexpr (kOwnRow<ZM>) load16<T>(reinterpret_cast<const T*>(a.xg) + r * a.kp + q * PPL, o.xo);
  }
}

// Probe values of row r for this lane: read (ZM == 0), or the Rademacher
// signs of the row's sign word (ZM == 1; the word is loaded with the other
// row operands), twin-class rows taken from the class table.
template <typename T, int ZM>
__device__ inline void row_probes(const StepArgs& a, bool own, int64_t r, int q, const RowOperands<T, ZM>& o,
                                  T (&z)[16 / sizeof(T)]) {
  constexpr int PPL = 16 / sizeof(T);
  if constexpr (ZM == 0) {
#pragma unroll
    for (int c = 0; c < PPL; ++c) z[c] = o.z[c];
  } else {
#pragma unroll
    for (int c = 0; c < PPL; ++c) z[c] = T(0);
    if (own) {
      const int32_t cls = a.zcls ? a.zcls[r] : -1;
      if (cls >= 0) {
        load16<T>(reinterpret_cast<const T*>(a.zcls_val) + static_cast<int64_t>(cls) * a.kp + q * PPL, z);
      } else {
#pragma unroll
        for (int c = 0; c < PPL; ++c) {
          const int j = q * PPL + c;
          if (j < a.k_batch) z[c] = ((o.zw >> j) & 1) ? T(-1) : T(1);
        }
      }
    }
  }
}

// Finish row r: X_{m+1} = 2/d * acc - X_{m-1} (or acc/d on the first step)
// evaluated in fp64 with one rounding to T, stored in place, then the moment
// epilogue on Y = sqrt(d) X.  (A scale 2/d rounded to fp32 would carry the
// same relative error into every step of the row: a fixed perturbation of
// D^{-1} A that moves the eigenvalue 1 by O(2^-24), which T_m, whose slope at
// 1 is m^2, turns into per-node errors growing like m^2 2^-24.)
// Doubling steps add Y_{m+1}.Y_m and Y_{m+1}.Y_{m+1} per probe instead (T_{m+1} T_m = (T_{2m+1} + T_1)/2 and
// T_{m+1}^2 = (T_{2m+2} + T_0)/2 turn them into two moments each).
// Lanczos steps (ZM == 3) store W = c1 D^{-1} A X - c2 X_prev with per-probe
// scales c1, c2 of the stored vectors, and add d c1 X(r) W(r) per probe (the
// numerator of alpha = <v, H v>).
template <typename T, int L, int ZM, typename A>
__device__ inline void finish_row(const StepArgs& a, bool own, int64_t r, int64_t d, const A (&acc)[16 / sizeof(T)],
                                  const RowOperands<T, ZM>& o, int q, double* mom) {
  constexpr int PPL = 16 / sizeof(T);
  if constexpr (ZM == 3) {
    if (own) {
      T* xo = reinterpret_cast<T*>(a.xio) + r * a.kp + q * PPL;
      T xn[PPL];
      const double invd = 1.0 / static_cast<double>(d);
#pragma unroll
      for (int c = 0; c < PPL; ++c) {
        const int j = q * PPL + c;
        const double c1 = a.lz[j], c2 = a.lz[a.kp + j];
        const double s = static_cast<double>(acc[c]) * invd * c1;
        xn[c] = a.first ? static_cast<T>(s) : static_cast<T>(s - c2 * static_cast<double>(o.xp[c]));
      }
      store16_nt<T>(xo, xn);
      const double dd = static_cast<double>(d);
#pragma unroll
      for (int c = 0; c < PPL; ++c) {
        const int j = q * PPL + c;
        if (j >= a.k_batch) continue;
        mom[c * kBlock] += dd * (a.lz[j] * static_cast<double>(o.xo[c])) * static_cast<double>(xn[c]);
      }
    }
    return;
  }
  double y[PPL];
  if (own) {
    T* xo = reinterpret_cast<T*>(a.xio) + r * a.kp + q * PPL;
    T xn[PPL];
    const double invd = 1.0 / static_cast<double>(d);
    if (a.first) {
#pragma unroll
      for (int c = 0; c < PPL; ++c) xn[c] = static_cast<T>(static_cast<double>(acc[c]) * invd);
    } else {
      const double two_invd = 2.0 * invd;
#pragma unroll
      for (int c = 0; c < PPL; ++c)
        xn[c] = static_cast<T>(two_invd * static_cast<double>(acc[c]) - static_cast<double>(o.xp[c]));
    }
    store16_nt<T>(xo, xn);
    const double sd = sqrt(static_cast<double>(d));
#pragma unroll
    for (int c = 0; c < PPL; ++c) y[c] = static_cast<double>(xn[c]) * sd;
  } else {
#pragma unroll
    for (int c = 0; c < PPL; ++c) y[c] = 0.0;
  }
  if constexpr (ZM == 2) {
    if (own) {
      const double sd = sqrt(static_cast<double>(d));
#pragma unroll
      for (int c = 0; c < PPL; ++c) {
        if (q * PPL + c >= a.k_batch) continue;
        const double y0 = static_cast<double>(o.xo[c]) * sd;
        mom[c * kBlock] += y[c] * y0;
        mom[(PPL + c) * kBlock] += y[c] * y[c];
      }
    }
  } else {
    T z[PPL];
    row_probes<T, ZM>(a, own, r, q, o, z);
    emit_moments<T, L>(a, own, r, o.node, y, z, q, mom);
  }
}

// Sum of X rows over the nonzeros e0+sub, e0+sub+P, ... < e1: U independent
// gathers in flight per lane (predicated), added in a fixed order.
template <typename T, int P, int U>
__device__ inline void gather_sum(const StepArgs& a, int64_t e0, int64_t e1, int sub, int q,
                                  T (&acc)[16 / sizeof(T)]) {
  constexpr int PPL = 16 / sizeof(T);
  const T* xg = reinterpret_cast<const T*>(a.xg) + q * PPL;
  const int64_t kp = a.kp;
  for (int64_t e = e0 + sub; e < e1; e += U * P) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t en = e + u * P;
      j[u] = (en < e1) ? __builtin_nontemporal_load(a.col + en) : -1;
    }
    T v[U][PPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] >= 0) {
        load16<T>(xg + static_cast<int64_t>(j[u]) * kp, v[u]);
      } else {
#pragma unroll
        for (int c = 0; c < PPL; ++c) v[u][c] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < PPL; ++c) acc[c] += v[u][c];
  }
}

// Column indices of the first gather batch of a row slice: nonzeros
// e0+sub, e0+sub+P, ... (U of them, -1 past e1).
template <int P, int U>
__device__ inline void load_cols(const StepArgs& a, int64_t e0, int64_t e1, int sub, int32_t (&j)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t en = e0 + sub + u * P;
    j[u] = (en < e1) ? __builtin_nontemporal_load(a.col + en) : -1;
  }
}

// All items of one bin handled by this wavefront (items w, w+W, ...): P
// nonzero slots per row, 64/(P*L) consecutive rows per item.  Software
// pipelined: while item i gathers, the column indices of item i+W and the
// row pointers of item i+2W load, so each item waits for one dependent
// memory round trip (the gathers) instead of two.
template <typename T, int L, int P, int U, int ZM>
__device__ inline void rows_bin(const StepArgs& a, int bin, int64_t w, int64_t W, int lane, double* mom) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int G = P * L;
  constexpr int RPW = kWave / G;
  const int grp = lane / G, sub = (lane % G) / L, q = lane % L;
  const int64_t rs = a.bin_row_start[bin], re = a.bin_row_start[bin + 1];
  const int64_t items = a.bin_item_start[bin + 1] - a.bin_item_start[bin];
  if (w >= items) return;
  auto rp = [&](int64_t li, int64_t& e0, int64_t& e1) {
    const int64_t r = rs + li * RPW + grp;
    if (li < items && r < re) {
      e0 = a.row_ptr[r];
      e1 = a.row_ptr[r + 1];
    } else {
      e0 = e1 = 0;
    }
  };
  const T* xg = reinterpret_cast<const T*>(a.xg) + q * PPL;
  int64_t e0, e1, e0n, e1n;
  rp(w, e0, e1);
  rp(w + W, e0n, e1n);
  int32_t j[U];
  load_cols<P, U>(a, e0, e1, sub, j);
  for (int64_t li = w; li < items; li += W) {
    const int64_t r = rs + li * RPW + grp;
    const bool own = r < re && sub == 0;
    RowOperands<T, ZM> o;
    load_row_operands<T, ZM>(a, own, r, q, o);
    T v[U][PPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] >= 0) {
        load16<T>(xg + static_cast<int64_t>(j[u]) * a.kp, v[u]);
      } else {
#pragma unroll
        for (int c = 0; c < PPL; ++c) v[u][c] = T(0);
      }
    }
    load_cols<P, U>(a, e0n, e1n, sub, j);
    int64_t e0nn, e1nn;
    rp(li + 2 * W, e0nn, e1nn);
    T acc[PPL];
#pragma unroll
    for (int c = 0; c < PPL; ++c) acc[c] = T(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < PPL; ++c) acc[c] += v[u][c];
    // rows longer than one batch (the widest bin only)
    if (e0 + sub + U * P < e1) gather_sum<T, P, U>(a, e0 + U * P, e1, sub, q, acc);
#pragma unroll
    for (int off = L; off < G; off <<= 1)
#pragma unroll
      for (int c = 0; c < PPL; ++c) acc[c] += __shfl_xor(acc[c], off, kWave);
    finish_row<T, L, ZM, T>(a, own, r, e1 - e0, acc, o, q, mom);
    e0 = e0n;
    e1 = e1n;
    e0n = e0nn;
    e1n = e1nn;
  }
}

// One chunk of a split row: its partial sum (fp64) goes to the chunk's slot.
// The rows are finished by k_split_finish after the step kernel, so no
// device-wide fence is needed here.
template <typename T, int L, int U>
__device__ inline void chunk_item(const StepArgs& a, int64_t c, int lane) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int P = kWave / L;
  const int sub = lane / L, q = lane % L;
  const int64_t r = a.chunk_owner[c];
  const int64_t c0 = a.split_chunk_ptr[r];
  const int64_t rb = a.row_ptr[r], re = a.row_ptr[r + 1];
  const int64_t e0 = rb + (c - c0) * a.chunk_nnz;
  const int64_t e1 = e0 + a.chunk_nnz < re ? e0 + a.chunk_nnz : re;
  T acc[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) acc[k] = T(0);
  gather_sum<T, P, U>(a, e0, e1, sub, q, acc);
#pragma unroll
  for (int off = L; off < kWave; off <<= 1)
#pragma unroll
    for (int k = 0; k < PPL; ++k) acc[k] += __shfl_xor(acc[k], off, kWave);
  double* part = reinterpret_cast<double*>(a.chunk_part);
  if (sub == 0) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) part[c * a.kp + q * PPL + k] = static_cast<double>(acc[k]);
  }
}

// Block-level fixed-order reduction of the per-lane probe sums (LDS
// s_mom[h * PPL + c][thread] for sum h of probe c of the thread's lane) into
// partial[blockIdx.x][h][0..kp).
template <typename T, int L, int NS>
__device__ inline void block_partials(const StepArgs& a, const double (*s_mom)[kBlock]) {
  constexpr int PPL = 16 / sizeof(T);
  __syncthreads();
  const int cols = NS * a.kp;
  if (static_cast<int>(threadIdx.x) < cols) {
    const int h = threadIdx.x / a.kp, j = threadIdx.x % a.kp, qq = j / PPL, cc = j % PPL;
    double s = 0.0, comp = 0.0;
    for (int t = qq; t < kBlock; t += L) neumaier(s, comp, s_mom[h * PPL + cc][t]);
    a.partial[static_cast<int64_t>(blockIdx.x) * cols + threadIdx.x] = s + comp;
  }
}

// Split rows: one wavefront per row sums the row's chunk partials (slot s of
// the wavefront takes chunks s, s+P, ... in order, then a fixed xor tree) and
// finishes the row.  Rows go to wavefronts in a fixed cyclic order and the
// moment terms are reduced per block like the step kernel's, into the slots
// after the step kernel's (the grid depends only on the graph, so the sums
// are reproducible).
template <typename T, int L, int ZM>
__global__ __launch_bounds__(kBlock) void k_split_finish(StepArgs a, int step_grid) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int P = kWave / L;
  constexpr int NS = kSums<ZM>;
  __shared__ double s_mom[NS * PPL][kBlock];
#pragma unroll
  for (int c = 0; c < NS * PPL; ++c) s_mom[c][threadIdx.x] = 0.0;
  double* mom = &s_mom[0][threadIdx.x];
  const int lane = threadIdx.x & (kWave - 1), sub = lane / L, q = lane % L;
  const double* part = reinterpret_cast<const double*>(a.chunk_part);
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; r < a.n_split;
       r += static_cast<int64_t>(gridDim.x) * kWavesPerBlock) {
    const int64_t c0 = a.split_chunk_ptr[r], c1 = a.split_chunk_ptr[r + 1];
    RowOperands<T, ZM> o;
    load_row_operands<T, ZM>(a, sub == 0, r, q, o);
    double tot[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) tot[k] = 0.0;
    for (int64_t c = c0 + sub; c < c1; c += P)
#pragma unroll
      for (int k = 0; k < PPL; ++k) tot[k] += part[c * a.kp + q * PPL + k];
#pragma unroll
    for (int off = L; off < kWave; off <<= 1)
#pragma unroll
      for (int k = 0; k < PPL; ++k) tot[k] += __shfl_xor(tot[k], off, kWave);
    finish_row<T, L, ZM, double>(a, sub == 0, r, a.row_ptr[r + 1] - a.row_ptr[r], tot, o, q, mom);
  }
  StepArgs b = a;
  b.partial = a.partial + static_cast<int64_t>(step_grid) * NS * a.kp;
  block_partials<T, L, NS>(b, s_mom);
}

// Four wavefronts per SIMD: the software-pipelined gather loop needs more
// than 128 VGPRs in the narrowest instantiations, where a few spilled
// registers cost less than a lost wavefront.
template <typename T, int L, int U, int ZM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_cheb_step(StepArgs a) {
  constexpr int PPL = 16 / sizeof(T);
  constexpr int PMAX = kWave / L;
  constexpr int NS = kSums<ZM>;
  __shared__ double s_mom[NS * PPL][kBlock];
#pragma unroll
  for (int c = 0; c < NS * PPL; ++c) s_mom[c][threadIdx.x] = 0.0;
  double* mom = &s_mom[0][threadIdx.x];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t W = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  for (int64_t c = w; c < a.n_chunks; c += W) chunk_item<T, L, U>(a, c, lane);
  // each bin continues the cyclic item order where the previous ones left
  // off, so that the wavefronts stay evenly loaded
  int64_t offset = a.n_chunks;
  for (int b = 0; b < a.n_bins; ++b) {
    const int64_t wb = ((w - offset) % W + W) % W;
    switch (a.bin_log2p[b]) {
#define ND_BIN(B) \
  case B:         \
    if constexpr ((1 << B) <= PMAX) rows_bin<T, L, (1 << B), U, ZM>(a, b, wb, W, lane, mom); \
    break;
      ND_BIN(0)
      ND_BIN(1)
      ND_BIN(2)
      ND_BIN(3)
      ND_BIN(4)
      ND_BIN(5)
      ND_BIN(6)
#undef ND_BIN
      default:
        break;
    }
    offset += a.bin_item_start[b + 1] - a.bin_item_start[b];
  }
  block_partials<T, L, NS>(a, s_mom);
}

// Moment 0: Y_0 = Z.  Internal rows in order, 64/L rows per wavefront.
template <typename T, int L, int ZM>
__global__ __launch_bounds__(kBlock) void k_moment0(StepArgs a) {
  static_assert(!kOwnRow<ZM>, "moment 0 needs the probes");
  constexpr int PPL = 16 / sizeof(T);
  constexpr int RPW = kWave / L;
  constexpr int NS = kSums<ZM>;
  __shared__ double s_mom[NS * PPL][kBlock];
#pragma unroll
  for (int c = 0; c < NS * PPL; ++c) s_mom[c][threadIdx.x] = 0.0;
  double* mom = &s_mom[0][threadIdx.x];
  const int lane = threadIdx.x & (kWave - 1), q = lane % L, grp = lane / L;
  const int64_t n_waves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  const int64_t items = ceil_div(a.n, RPW);
  for (int64_t it = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave; it < items;
       it += n_waves) {
    const int64_t r = it * RPW + grp;
    const bool own = r < a.n;
    RowOperands<T, ZM> o;
    load_row_operands<T, ZM>(a, own, r, q, o);
    T z[PPL];
    row_probes<T, ZM>(a, own, r, q, o, z);
    double y[PPL];
#pragma unroll
    for (int c = 0; c < PPL; ++c) y[c] = static_cast<double>(z[c]);
    emit_moments<T, L>(a, own, r, o.node, y, z, q, mom);
  }
  // no split rows at moment 0: clear the finisher's slots
  double* sp = a.partial + static_cast<int64_t>(gridDim.x) * a.kp;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < int64_t(a.split_blocks) * a.kp;
       t += static_cast<int64_t>(gridDim.x) * kBlock)
    sp[t] = 0.0;
  block_partials<T, L, NS>(a, s_mom);
}

}  // namespace
}  // namespace nd

// ====================================================================== probes
namespace nd {
namespace {

// Probe entry (j, i): see nd_make_probes in nd.h for the definition.
__device__ inline float probe_value(uint64_t seed, int64_t j, int64_t i, bool gaussian) {
  if (!gaussian) return rademacher_entry(seed, j, i);
  const uint64_t key = splitmix64(seed, static_cast<uint64_t>(j) + 1);
  const uint64_t b1 = splitmix64(key, 2 * static_cast<uint64_t>(i) + 1);
  const uint64_t b2 = splitmix64(key, 2 * static_cast<uint64_t>(i) + 2);
  const double u1 = (static_cast<double>(b1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = static_cast<double>(b2 >> 11) * 0x1.0p-53;
  const double g = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  return static_cast<float>(g);
}

// Z[r][ld] (probes j0 .. j0+k_batch-1 in columns 0..k_batch-1, zeros beyond)
// for rows r of an ordering whose node ids are perm[r] (identity if null);
// when X0 is given, X0 = D^{-1/2} Z with degrees from that ordering's row_ptr.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probes(int64_t n, int ld, int k_batch, int64_t j0, uint64_t seed,
                                                   int gaussian, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ perm, T* __restrict__ Z,
                                                   T* __restrict__ X0) {
  const int64_t total = n * ld;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = idx / ld;
    const int j = static_cast<int>(idx - i * ld);
    const int64_t node = perm ? static_cast<int64_t>(perm[i]) : i;
    const T z = j < k_batch ? static_cast<T>(probe_value(seed, j0 + j, node, gaussian != 0)) : T(0);
    Z[idx] = z;
    if (X0) {
      const double d = static_cast<double>(row_ptr[i + 1] - row_ptr[i]);
      X0[idx] = static_cast<T>(static_cast<double>(z) / sqrt(d));
    }
  }
}

// Unit probes: column j of the (zeroed) block is e_{node_j}: Z = 1 and
// X_0 = 1/sqrt(d) at the node's internal row.
template <typename T>
__global__ void k_unit_probes(int k_batch, int ld, const int32_t* __restrict__ nodes, const int32_t* __restrict__ inv,
                              const int64_t* __restrict__ row_ptr, T* __restrict__ Z, T* __restrict__ X0) {
  const int j = threadIdx.x;
  if (j >= k_batch) return;
  const int64_t r = inv[nodes[j]];
  Z[r * ld + j] = T(1);
  X0[r * ld + j] = static_cast<T>(1.0 / sqrt(static_cast<double>(row_ptr[r + 1] - row_ptr[r])));
}

// Sign bits of a Rademacher probe block, one 64-bit word per internal row
// (bit j set where probe j is -1; ld <= 64): the step kernels read these 8
// bytes per row instead of regenerating the row's entries.  One wavefront per
// row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sign_bits(int64_t n, int ld, const T* __restrict__ Z,
                                                      uint64_t* __restrict__ bits) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; i < n;
       i += static_cast<int64_t>(gridDim.x) * kWavesPerBlock) {
    const bool neg = lane < ld && Z[i * ld + lane] < T(0);
    const uint64_t w = __ballot(neg);
    if (lane == 0) bits[i] = w;
  }
}

// Twin projection Z <- P P^T Z (Sec. 3.4): each class's rows replaced by the
// class mean (fp64 sum in member order).  Members of a class share their
// neighbourhood and hence their degree.  Member node i lives in row inv[i]
// (row i if inv is null).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_project(const int64_t* __restrict__ class_ptr,
                                                    const int32_t* __restrict__ members, int64_t n_classes,
                                                    int ld, int k_batch, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ inv, T* __restrict__ Z,
                                                    T* __restrict__ X0, T* __restrict__ cmean) {
  const int64_t total = n_classes * k_batch;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t c = idx / k_batch;
    const int j = static_cast<int>(idx - c * k_batch);
    const int64_t p0 = class_ptr[c], p1 = class_ptr[c + 1];
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t i = inv ? static_cast<int64_t>(inv[members[p]]) : static_cast<int64_t>(members[p]);
      s += static_cast<double>(Z[i * ld + j]);
    }
    const T mean = static_cast<T>(s / static_cast<double>(p1 - p0));
    if (cmean) cmean[c * ld + j] = mean;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t i = inv ? static_cast<int64_t>(inv[members[p]]) : static_cast<int64_t>(members[p]);
      Z[i * ld + j] = mean;
      if (X0) {
        const double d = static_cast<double>(row_ptr[i + 1] - row_ptr[i]);
        X0[i * ld + j] = static_cast<T>(static_cast<double>(mean) / sqrt(d));
      }
    }
  }
}

// zcls[inv[i]] = class of member i (the array is -1 elsewhere).
__global__ __launch_bounds__(kBlock) void k_zcls(const int64_t* __restrict__ class_ptr,
                                                 const int32_t* __restrict__ members, int64_t n_classes,
                                                 const int32_t* __restrict__ inv, int32_t* __restrict__ zcls) {
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; c < n_classes;
       c += static_cast<int64_t>(gridDim.x) * kBlock)
    for (int64_t p = class_ptr[c]; p < class_ptr[c + 1]; ++p) zcls[inv[members[p]]] = static_cast<int32_t>(c);
}

// out[(j0 + j) * ld_out + (m0 + s) * NS + h] = (1/N) sum over the partial
// slots of sum h of probe j, for the launches m0 + s stored in consecutive
// partial blocks of step_stride doubles (slots x NS x kp each; one block per
// launch).  Thread t sums slots t/cols, t/cols + S, ... (cols = NS kp, S =
// 256/cols stripes) with compensation; the stripes are then combined in
// order: a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partial, int64_t slots,
                                                            int64_t step_stride, int NS, int kp, int k_batch,
                                                            int m0, double inv_n, double* __restrict__ out,
                                                            int64_t ld_out, int64_t j0) {
  __shared__ double red[kBlock];
  const int s = blockIdx.x;
  const int cols = NS * kp;
  const double* p = partial + static_cast<int64_t>(s) * step_stride;
  const int stripes = kBlock / cols;
  const int c = threadIdx.x % cols, st = threadIdx.x / cols;
  double sum = 0.0, comp = 0.0;
  if (st < stripes)
    for (int64_t b = st; b < slots; b += stripes) neumaier(sum, comp, p[b * cols + c]);
  red[threadIdx.x] = sum + comp;
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < cols && static_cast<int>(threadIdx.x) % kp < k_batch) {
    double t = 0.0, cc = 0.0;
    for (int q = 0; q < stripes; ++q) neumaier(t, cc, red[q * cols + threadIdx.x]);
    const int h = threadIdx.x / kp, j = threadIdx.x % kp;
    out[(j0 + j) * ld_out + static_cast<int64_t>(m0 + s) * NS + h] = (t + cc) * inv_n;
  }
}

// Moments from the doubling steps, per probe: with r1[s] = Y_s.Y_{s-1} / N
// and r2[s] = Y_s.Y_s / N (raw[j][2 s + 0/1], s >= 1),
//   mu_1 = r1[1],  mu_{2s-1} = 2 r1[s] - mu_1,  mu_{2s} = 2 r2[s] - mu_0
// (T_s T_{s-1} = (T_{2s-1} + T_1) / 2, T_s^2 = (T_{2s} + T_0) / 2); mu_0 is
// already in mu_pp.
__global__ __launch_bounds__(kBlock) void k_doubling_moments(const double* __restrict__ raw, int64_t ld_raw,
                                                             int k_batch, int64_t j0, int M,
                                                             double* __restrict__ mu_pp) {
  const int64_t total = static_cast<int64_t>(k_batch) * M;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t j = j0 + idx / M;
    const int m = static_cast<int>(idx % M);
    if (m == 0) continue;
    const double* r = raw + j * ld_raw;
    double v;
    if (m & 1) {
      const int sidx = (m + 1) / 2;
      v = (m == 1) ? r[2] : 2.0 * r[2 * sidx] - r[2];
    } else {
      v = 2.0 * r[2 * (m / 2) + 1] - mu_pp[j * M];
    }
    mu_pp[j * M + m] = v;
  }
}

// T_m(x) by the three-term recurrence (exact 1, 0, -1, 0, ... at x = 0).
__device__ inline double cheb_T(int m, double x) {
  double t0 = 1.0, t1 = x;
  if (m == 0) return t0;
  for (int i = 1; i < m; ++i) {
    const double t2 = 2.0 * x * t1 - t0;
    t0 = t1;
    t1 = t2;
  }
  return t1;
}

// mu[m] = (1/k) sum_j mu_pp[j][m] + sum_s w_s T_m(lambda_s) over the removed
// eigenvalues (spikes = lambdas then weights, n_spikes of each).
__global__ __launch_bounds__(kBlock) void k_mu_final(const double* __restrict__ mu_pp, int k, int M,
                                                     const double* __restrict__ spikes, int n_spikes,
                                                     double* __restrict__ mu) {
  for (int m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock) {
    double sum = 0.0, comp = 0.0;
    for (int j = 0; j < k; ++j) neumaier(sum, comp, mu_pp[static_cast<int64_t>(j) * M + m]);
    double add = 0.0;
    for (int s = 0; s < n_spikes; ++s) add += spikes[n_spikes + s] * cheb_T(m, spikes[s]);
    mu[m] = (sum + comp) / static_cast<double>(k) + add;
  }
}

// Moves the LDOS terms of launches m0 .. m0+S-1 from the staging block
// ([S][n] by internal row) into the output ([n][ld] by compact node, columns
// m0 ..), adding to what is there for the later probe blocks.  A block takes
// 64 internal rows: the tile is read along rows and written S contiguous
// entries per node, through LDS.
constexpr int kFlushRows = 64;
constexpr int kMaxStage = 32;

__global__ __launch_bounds__(kBlock) void k_ldos_flush(const double* __restrict__ stage, int64_t n, int S,
                                                       const int32_t* __restrict__ perm, double* __restrict__ out,
                                                       int64_t ld, int m0, int accumulate) {
  __shared__ double tile[kMaxStage][kFlushRows + 1];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kFlushRows;
  for (int t = threadIdx.x; t < S * kFlushRows; t += kBlock) {
    const int s = t / kFlushRows, rr = t % kFlushRows;
    const int64_t r = r0 + rr;
    tile[s][rr] = r < n ? stage[static_cast<int64_t>(s) * n + r] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < S * kFlushRows; t += kBlock) {
    const int rr = t / S, s = t % S;
    const int64_t r = r0 + rr;
    if (r >= n) continue;
    double* p = out + static_cast<int64_t>(perm[r]) * ld + m0 + s;
    *p = (accumulate ? *p : 0.0) + tile[s][rr];
  }
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Resident blocks of the step kernel on the whole device (occupancy times
// compute units): the persistent grid of the sparse product.  ND_STEP_GRID
// overrides it (tuning experiments).
template <typename T, int L>
int resident_grid() {
  static int grid = [] {
    const auto kern = k_cheb_step<T, L, 8, 1>;
    if (const char* e = std::getenv("ND_STEP_GRID")) {
      const int v = std::atoi(e);
      if (v > 0) return v;
    }
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0) {
      (void)hipGetLastError();
      return 2048;
    }
    return cus * per_cu;
  }();
  return grid;
}

template <typename T>
int step_grid(int L) {
  switch (L) {
    case 1: return resident_grid<T, 1>();
    case 2: return resident_grid<T, 2>();
    case 4: return resident_grid<T, 4>();
    case 8: return resident_grid<T, 8>();
    case 16: return resident_grid<T, 16>();
    case 32:
      if constexpr (sizeof(T) == 8) return resident_grid<T, 32>();
      break;
    default: break;
  }
  return 2048;
}

// ND_PROBE_BUFFER=1 makes the step kernels read the probe block instead of
// the per-row sign words of Rademacher probes (read on every call: tuning
// experiments, and tests that check both paths give identical results).
bool probe_buffer_forced() {
  const char* e = std::getenv("ND_PROBE_BUFFER");
  return e && std::atoi(e) == 1;
}

// Probes per block of the recurrence (a power of two, at most 64);
// ND_MAX_BLOCK_PROBES lowers it (tuning experiments).
int max_block_probes() {
  static int v = [] {
    int b = 64;
    if (const char* e = std::getenv("ND_MAX_BLOCK_PROBES")) {
      const int x = std::atoi(e);
      if (x >= 1 && x <= 64) b = pow2_at_least(x);
    }
    return b;
  }();
  return v;
}

// Launches per LDOS staging block: at most kMaxStage, fewer when the block
// would exceed 1 GiB; ND_LDOS_STAGE lowers the maximum (read on every call;
// tests use it to check that the grouping leaves the results unchanged).
int ldos_stage_launches(int64_t bytes_per_launch, int launches) {
  int smax = kMaxStage;
  if (const char* e = std::getenv("ND_LDOS_STAGE")) {
    const int v = std::atoi(e);
    if (v >= 1 && v < smax) smax = v;
  }
  const int64_t cap = (int64_t(1) << 30) / bytes_per_launch;
  int S = static_cast<int>(cap < smax ? (cap < 1 ? 1 : cap) : smax);
  return S > launches ? launches : S;
}

// Device memory of one moment call: each buffer is the graph's growable
// workspace of that name, or -- for the allocation-free entry point -- the
// next 256-byte-aligned slice of a fixed arena (no allocation at all).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

nd_status take(Arena* ar, Scratch& s, size_t bytes, void** out) {
  if (!ar) {
    ND_CHECK(s.ensure(bytes));
    *out = s.p;
    return ND_OK;
  }
  const size_t off = (ar->used + 255) & ~size_t(255);
  if (off > ar->cap || bytes > ar->cap - off) {
    set_error("internal: the fixed workspace is %zu bytes short", off + bytes - ar->cap);
    return ND_EINVAL;
  }
  *out = ar->base + off;
  ar->used = off + bytes;
  return ND_OK;
}

struct MomentJob {
  Arena* arena = nullptr;  // fixed device workspace instead of the graph's buffers
  const nd_motifs* motifs = nullptr;
  int k = 0, M = 0;
  uint64_t seed = 0;
  bool gaussian = false;
  const float* cv_g = nullptr;
  double* ldos = nullptr;
  double* ldos_sq = nullptr;
  double* mu = nullptr;
  double* mu_pp = nullptr;
  const double* spikes = nullptr;  // device: removed eigenvalues, then their weights
  int n_spikes = 0;                // (added to mu as sum_s w_s T_m(lambda_s))
  bool timed = false;
  bool doubling = false;  // global moments from products of Y_s (about M/2 launches)
  const int32_t* unit_nodes = nullptr;  // device [k]: probe j is the unit vector of node unit_nodes[j]
};

template <typename T, int L, int ZM>
nd_status launch_step_zm(const StepArgs& base, int grid, bool moment0, hipStream_t st) {
  if (moment0) {
    if constexpr (kOwnRow<ZM>) {
      set_error("internal: moment 0 launched as a doubling or Lanczos step");
      return ND_EUNSUPPORTED;
    } else {
      hipLaunchKernelGGL((k_moment0<T, L, ZM>), dim3(grid), dim3(kBlock), 0, st, base);
    }
  } else {
    hipLaunchKernelGGL((k_cheb_step<T, L, 8, ZM>), dim3(grid), dim3(kBlock), 0, st, base);
    if (base.n_split > 0) {
      ND_LAUNCH_CHECK();
      hipLaunchKernelGGL((k_split_finish<T, L, ZM>), dim3(base.split_blocks), dim3(kBlock), 0, st, base, grid);
    }
  }
  ND_LAUNCH_CHECK();
  return ND_OK;
}

template <typename T, int L>
nd_status launch_step_kernels(const StepArgs& base, int grid, bool moment0, hipStream_t st) {
  switch (base.zmode) {
    case 0: return launch_step_zm<T, L, 0>(base, grid, moment0, st);
    case 1: return launch_step_zm<T, L, 1>(base, grid, moment0, st);
    case 2: return launch_step_zm<T, L, 2>(base, grid, moment0, st);
    default: return launch_step_zm<T, L, 3>(base, grid, moment0, st);
  }
}

template <typename T>
nd_status launch_step(int L, const StepArgs& a, int grid, bool moment0, hipStream_t st) {
  switch (L) {
    case 1: return launch_step_kernels<T, 1>(a, grid, moment0, st);
    case 2: return launch_step_kernels<T, 2>(a, grid, moment0, st);
    case 4: return launch_step_kernels<T, 4>(a, grid, moment0, st);
    case 8: return launch_step_kernels<T, 8>(a, grid, moment0, st);
    case 16: return launch_step_kernels<T, 16>(a, grid, moment0, st);
    case 32:
      if constexpr (sizeof(T) == 8) return launch_step_kernels<T, 32>(a, grid, moment0, st);
      break;
    default: break;
  }
  set_error("internal: unsupported lane count %d", L);
  return ND_EUNSUPPORTED;
}

// Per-probe-block state shared by the moment and Lanczos drivers: schedule,
// recurrence buffers (Z, A = X_0, B), the probe block (projected when
// filtering) and the step arguments.
template <typename T>
struct BlockSetup {
  int kp = 0, L = 0, grid = 0, split_blocks = 0, zmode = 0;
  int64_t slots = 0;
  T *Z = nullptr, *A = nullptr, *B = nullptr;
  StepArgs a{};
};

template <typename T>
nd_status setup_block(nd_graph* g, const MomentJob& job, int j0, int kb, hipStream_t st, BlockSetup<T>& bs) {
  constexpr int PPL = 16 / sizeof(T);
  const int64_t N = g->n;
  const int M = job.M;
  const int kp = pow2_at_least(kb < PPL ? PPL : kb);
  const int L = kp * static_cast<int>(sizeof(T)) / 16;
  Schedule* sc = nullptr;
  if (job.arena) {
    // the allocation-free path only uses a schedule an earlier call built
    auto it = g->sched.find(L);
    if (it == g->sched.end() || !g->internal) {
      set_error("the graph has no row schedule for blocks of %d probes yet: run nd_cheb_moments once on it "
                "with the same probe count first", kp);
      return ND_EINVAL;
    }
    sc = it->second.get();
  } else {
    ND_CHECK(get_schedule(g, L, st, &sc));
  }
  Internal* in = g->internal.get();
  const size_t blk = static_cast<size_t>(N) * kp * sizeof(T);
  void *p_state = nullptr, *p_chunk = nullptr;
  ND_CHECK(take(job.arena, g->ws_state, 3 * blk, &p_state));
  ND_CHECK(take(job.arena, g->ws_chunk, static_cast<size_t>(sc->n_chunks > 0 ? sc->n_chunks : 1) * kp * sizeof(double),
                &p_chunk));
  T* Z = static_cast<T*>(p_state);
  T* A = Z + static_cast<int64_t>(N) * kp;
  T* B = A + static_cast<int64_t>(N) * kp;
  const int grid = grid_for(sc->n_items > 0 ? sc->n_items : 1, kWavesPerBlock, step_grid<T>(L));
  const int split_blocks = sc->n_split > 0 ? grid_for(sc->n_split, kWavesPerBlock, grid) : 0;
  const int64_t slots = static_cast<int64_t>(grid) + split_blocks;

  if (job.unit_nodes) {
    ND_HIP(hipMemsetAsync(Z, 0, 2 * blk, st));  // Z and A = X_0
    hipLaunchKernelGGL(k_unit_probes<T>, dim3(1), dim3(64), 0, st, kb, kp, job.unit_nodes + j0, in->inv, in->row_ptr,
                       Z, A);
  } else {
    hipLaunchKernelGGL(k_probes<T>, dim3(grid_for(N * kp, kBlock)), dim3(kBlock), 0, st, N, kp, kb,
                       static_cast<int64_t>(j0), job.seed, job.gaussian ? 1 : 0, in->row_ptr, in->perm, Z, A);
  }
  ND_LAUNCH_CHECK();
  // Rademacher rows reach the step kernels as one sign word per row (no
  // probe-block reads); the projected rows of twin classes come from a small
  // table
  const int zmode = (!job.gaussian && !job.unit_nodes && !probe_buffer_forced()) ? 1 : 0;
  uint64_t* zbits = nullptr;
  if (zmode) {
    void* p = nullptr;
    ND_CHECK(take(job.arena, g->ws_zbits, static_cast<size_t>(N) * sizeof(uint64_t), &p));
    zbits = static_cast<uint64_t*>(p);
    hipLaunchKernelGGL(k_sign_bits<T>, dim3(grid_for(N, kWavesPerBlock)), dim3(kBlock), 0, st, N, kp, Z, zbits);
    ND_LAUNCH_CHECK();
  }
  const bool filt = job.motifs && job.motifs->n_classes > 0;
  int32_t* zcls = nullptr;
  T* zcls_val = nullptr;
  if (filt) {
    if (job.arena) {
      set_error("internal: motif filtering on the fixed workspace");
      return ND_EUNSUPPORTED;
    }
    if (zmode) {
      const size_t nc = static_cast<size_t>(job.motifs->n_classes);
      ND_CHECK(g->ws_zcls.ensure(static_cast<size_t>(N) * 4 + 256 + nc * kp * sizeof(T)));
      zcls = g->ws_zcls.as<int32_t>();
      zcls_val = reinterpret_cast<T*>(reinterpret_cast<char*>(g->ws_zcls.p) + ((static_cast<size_t>(N) * 4 + 255) & ~size_t(255)));
      ND_HIP(hipMemsetAsync(zcls, 0xFF, static_cast<size_t>(N) * 4, st));
      ND_HIP(hipMemsetAsync(zcls_val, 0, nc * kp * sizeof(T), st));
      hipLaunchKernelGGL(k_zcls, dim3(grid_for(job.motifs->n_classes, kBlock)), dim3(kBlock), 0, st,
                         job.motifs->class_ptr, job.motifs->members, job.motifs->n_classes, in->inv, zcls);
      ND_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_project<T>, dim3(grid_for(job.motifs->n_classes * kb, kBlock)), dim3(kBlock), 0, st,
                       job.motifs->class_ptr, job.motifs->members, job.motifs->n_classes, kp, kb, in->row_ptr,
                       in->inv, Z, A, zcls_val);
    ND_LAUNCH_CHECK();
  }
  StepArgs a{};
  a.row_ptr = in->row_ptr;
  a.col = in->col;
  a.perm = in->perm;
  a.n = N;
  a.n_bins = sc->n_bins;
  for (int b = 0; b <= kMaxBins; ++b) {
    a.bin_row_start[b] = sc->bin_row_start[b];
    a.bin_item_start[b] = sc->bin_item_start[b];
    if (b < kMaxBins) a.bin_log2p[b] = sc->bin_log2p[b];
  }
  a.n_chunks = sc->n_chunks;
  a.n_items = sc->n_items;
  a.split_chunk_ptr = sc->split_chunk_ptr;
  a.chunk_owner = sc->chunk_owner;
  a.chunk_nnz = sc->chunk_nnz;
  a.n_split = sc->n_split;
  a.split_blocks = split_blocks;
  a.slot_nnz = sc->slot_nnz;
  a.zmode = zmode;
  a.seed = job.seed;
  a.j0 = j0;
  a.zbits = zbits;
  a.zcls = zcls;
  a.zcls_val = zcls_val;
  a.chunk_part = p_chunk;
  a.z = Z;
  a.kp = kp;
  a.k_batch = kb;
  a.inv_k = 1.0 / static_cast<double>(job.k);
  a.ldos = job.ldos;
  a.ldos_sq = job.ldos_sq;
  a.ld = M;
  a.accumulate = j0 > 0 ? 1 : 0;
  a.cv_g = job.cv_g;
  bs.kp = kp;
  bs.L = L;
  bs.grid = grid;
  bs.split_blocks = split_blocks;
  bs.zmode = zmode;
  bs.slots = slots;
  bs.Z = Z;
  bs.A = A;
  bs.B = B;
  bs.a = a;
  return ND_OK;
}

template <typename T>
nd_status run_moments(nd_graph* g, const MomentJob& job, hipStream_t st) {
  const int64_t N = g->n;
  const int M = job.M;
  double* mu_pp = job.mu_pp;
  std::vector<hipEvent_t> evs;
  if (job.timed) {
    g->step_ms = 0.0;
    g->step_launches = 0;
  }
  struct EvFree {
    std::vector<hipEvent_t>& e;
    ~EvFree() {
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
  } ev_free{evs};
  // doubling: launches s = 1..S give moments 2s-1 and 2s (S = floor(M/2));
  // otherwise launch m gives moment m
  const int last = job.doubling ? M / 2 : M - 1;
  const int64_t ld_raw = 2 * (static_cast<int64_t>(last) + 1);
  const size_t n_pp = job.mu_pp ? 0 : static_cast<size_t>(job.k) * M;
  const size_t n_raw = job.doubling ? static_cast<size_t>(job.k) * ld_raw : 0;
  double* misc = nullptr;
  if (n_pp + n_raw) {
    void* p = nullptr;
    ND_CHECK(take(job.arena, g->ws_misc, (n_pp + n_raw) * sizeof(double), &p));
    misc = static_cast<double*>(p);
  }
  if (!mu_pp) mu_pp = misc;
  double* raw = job.doubling ? misc + n_pp : nullptr;
  const int bmax = max_block_probes();
  // each probe block reuses the arena space after the call-wide buffers
  const size_t arena_mark = job.arena ? job.arena->used : 0;
  for (int j0 = 0; j0 < job.k; j0 += bmax) {
    const int kb = job.k - j0 < bmax ? job.k - j0 : bmax;
    if (job.arena) job.arena->used = arena_mark;
    BlockSetup<T> bs;
    ND_CHECK(setup_block<T>(g, job, j0, kb, st, bs));
    const int kp = bs.kp, L = bs.L, grid = bs.grid, zmode = bs.zmode;
    const int64_t slots = bs.slots;
    T* A = bs.A;
    T* B = bs.B;
    StepArgs& a = bs.a;
    const int NSd = job.doubling ? 2 : 1;          // sums per probe of the step launches
    const int64_t per_step = slots * kp * NSd;
    int R = static_cast<int>((int64_t(64) << 20) / (per_step * 8));
    if (job.arena) {  // as many launches as the rest of the arena holds
      const size_t used = (job.arena->used + 255) & ~size_t(255);
      const int64_t fit = used < job.arena->cap ? static_cast<int64_t>((job.arena->cap - used) / (per_step * 8)) : 0;
      if (fit < R) R = static_cast<int>(fit);
    }
    if (R < 1) R = 1;
    if (R > last + 1) R = last + 1;
    void* p_partial = nullptr;
    ND_CHECK(take(job.arena, g->ws_partial, static_cast<size_t>(R) * per_step * sizeof(double), &p_partial));
    double* partial = static_cast<double*>(p_partial);
    // unit probes: z^T T_m(H) z is the PDOS moment itself, no 1/N
    const double inv_n = job.unit_nodes ? 1.0 : 1.0 / static_cast<double>(N);
    // LDOS terms go through a staging block of S launches (at most 1 GiB)
    int S = 0;
    if (job.ldos) {
      const int64_t per_launch = N * 8 * (job.ldos_sq ? 2 : 1);
      S = ldos_stage_launches(per_launch, last + 1);
      void* p_stage = nullptr;
      ND_CHECK(take(job.arena, g->ws_stage, static_cast<size_t>(S) * per_launch, &p_stage));
      a.stage = static_cast<double*>(p_stage);
      a.stage_sq = job.ldos_sq ? a.stage + static_cast<int64_t>(S) * N : nullptr;
    }
    for (int m = 0; m <= last; ++m) {
      a.m = m;
      if (S) a.stage_pos = m % S;
      // ring position of this launch's partials; with doubling, moment 0 is
      // reduced on its own right away (one sum per probe) and the ring
      // starts at launch 1
      const int pos = job.doubling ? (m == 0 ? 0 : (m - 1) % R) : m % R;
      a.partial = partial + static_cast<int64_t>(pos) * per_step;
      if (m == 0) {
        a.first = 1;  // no X_{m-1} operand at moment 0
        a.xg = nullptr;
        a.xio = nullptr;
        a.zmode = zmode;
        ND_CHECK(launch_step<T>(L, a, grid, true, st));
        if (job.doubling) {
          hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, slots, per_step, 1, kp, kb, 0,
                             inv_n, mu_pp, static_cast<int64_t>(M), static_cast<int64_t>(j0));
          ND_LAUNCH_CHECK();
          continue;
        }
      } else {
        if (job.doubling) a.zmode = 2;
        a.first = (m == 1) ? 1 : 0;
        a.xg = (m & 1) ? A : B;
        a.xio = (m & 1) ? B : A;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (job.timed) {
          ND_HIP(hipEventCreate(&e0));
          evs.push_back(e0);
          ND_HIP(hipEventCreate(&e1));
          evs.push_back(e1);
          ND_HIP(hipEventRecord(e0, st));
        }
        ND_CHECK(launch_step<T>(L, a, grid, false, st));
        if (job.timed) ND_HIP(hipEventRecord(e1, st));
      }
      if (S && (a.stage_pos + 1 == S || m == last)) {
        const int nst = a.stage_pos + 1;
        const unsigned fgrid = static_cast<unsigned>(ceil_div(N, kFlushRows));
        hipLaunchKernelGGL(k_ldos_flush, dim3(fgrid), dim3(kBlock), 0, st, a.stage, N, nst, a.perm, job.ldos,
                           static_cast<int64_t>(M), m + 1 - nst, a.accumulate);
        ND_LAUNCH_CHECK();
        if (job.ldos_sq) {
          hipLaunchKernelGGL(k_ldos_flush, dim3(fgrid), dim3(kBlock), 0, st, a.stage_sq, N, nst, a.perm,
                             job.ldos_sq, static_cast<int64_t>(M), m + 1 - nst, a.accumulate);
          ND_LAUNCH_CHECK();
        }
      }
      if (pos + 1 == R || m == last) {
        const int m0 = m - pos;
        if (job.doubling)
          hipLaunchKernelGGL(k_reduce_partials, dim3(pos + 1), dim3(kBlock), 0, st, partial, slots, per_step, 2, kp,
                             kb, m0, inv_n, raw, ld_raw, static_cast<int64_t>(j0));
        else
          hipLaunchKernelGGL(k_reduce_partials, dim3(pos + 1), dim3(kBlock), 0, st, partial, slots, per_step, 1, kp,
                             kb, m0, inv_n, mu_pp, static_cast<int64_t>(M), static_cast<int64_t>(j0));
        ND_LAUNCH_CHECK();
      }
    }
    if (job.doubling) {
      hipLaunchKernelGGL(k_doubling_moments, dim3(grid_for(static_cast<int64_t>(kb) * M, kBlock)), dim3(kBlock), 0,
                         st, raw, ld_raw, kb, static_cast<int64_t>(j0), M, mu_pp);
      ND_LAUNCH_CHECK();
    }
  }
  if (job.timed) {
    ND_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i + 1 < evs.size(); i += 2) {
      float ms = 0.f;
      ND_HIP(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      g->step_ms += ms;
      g->step_launches++;
    }
  }
  if (job.mu) {
    hipLaunchKernelGGL(k_mu_final, dim3(grid_for(M, kBlock)), dim3(kBlock), 0, st, mu_pp, job.k, M, job.spikes,
                       job.n_spikes, job.mu);
    ND_LAUNCH_CHECK();
  }
  if (job.ldos && job.motifs && job.motifs->n_classes > 0) {
    hipLaunchKernelGGL(k_motif_diag<double>, dim3(grid_for(job.motifs->n_members, kBlock)), dim3(kBlock), 0, st,
                       job.motifs->class_ptr, job.motifs->members, job.motifs->class_lambda,
                       job.motifs->class_paired, job.motifs->n_classes, job.motifs->n_members,
                       static_cast<int64_t>(M), M, 1.0, job.ldos);
    ND_LAUNCH_CHECK();
  }
  return ND_OK;
}

// ---------------------------------------------------------------- Lanczos
// Gauss quadrature and Lanczos (Sec. 3.2) on the same sparse product: per
// probe j, v_1 = z_j / |z_j|, w = H v_k - beta_{k-1} v_{k-1},
// alpha_k = <v_k, w>, w -= alpha_k v_k, beta_k = |w|, v_{k+1} = w / beta_k.
// Vectors are kept in the form X = D^{-1/2} v like the Chebyshev state, and
// unnormalized: the stored current and previous vectors carry per-probe
// scales (lz[0][j], and beta_{k-1} times the previous scale in lz[1][j]).

// alpha_k is already reduced; W -= alpha_k c1 X_cur and per-probe sums of
// d W^2 (the square of beta_k) into block partials.  Thread t of the grid
// handles 16-byte slice t % L of rows t / L, ...
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_lanczos_update(int64_t n, int kp, int k_batch,
                                                           const int64_t* __restrict__ row_ptr, T* __restrict__ W,
                                                           const T* __restrict__ X, const double* __restrict__ lz,
                                                           const double* __restrict__ alpha, int64_t ld_alpha,
                                                           double* __restrict__ partial) {
  constexpr int PPL = 16 / sizeof(T);
  __shared__ double s_mom[PPL][kBlock];
#pragma unroll
  for (int c = 0; c < PPL; ++c) s_mom[c][threadIdx.x] = 0.0;
  const int q = threadIdx.x % L;
  double coef[PPL];
#pragma unroll
  for (int c = 0; c < PPL; ++c) {
    const int j = q * PPL + c;
    coef[c] = j < k_batch ? alpha[j * ld_alpha] * lz[j] : 0.0;
  }
  const int64_t total = n * L;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t r = t / L;
    T w[PPL], x[PPL];
    load16<T>(W + r * kp + q * PPL, w);
    load16<T>(X + r * kp + q * PPL, x);
    const double d = static_cast<double>(row_ptr[r + 1] - row_ptr[r]);
#pragma unroll
    for (int c = 0; c < PPL; ++c) {
      w[c] = static_cast<T>(static_cast<double>(w[c]) - coef[c] * static_cast<double>(x[c]));
      s_mom[c][threadIdx.x] += d * static_cast<double>(w[c]) * static_cast<double>(w[c]);
    }
    store16<T>(W + r * kp + q * PPL, w);
  }
  StepArgs b{};
  b.kp = kp;
  b.partial = partial;
  block_partials<T, L, 1>(b, s_mom);
}

// Per-probe scales before the first step: c1 = 1/|z|, c2 = 0.
__global__ void k_lanczos_init(int k_batch, int kp, double n, const double* __restrict__ norm2, double* __restrict__ lz,
                               int32_t* __restrict__ active) {
  const int j = threadIdx.x;
  if (j >= kp) return;
  const double z2 = j < k_batch ? norm2[j] * n : 0.0;
  const bool on = z2 > 0.0;
  lz[j] = on ? 1.0 / sqrt(z2) : 0.0;
  lz[kp + j] = 0.0;
  active[j] = on ? 1 : 0;
}

// After step k: beta_k = sqrt(sum d W^2); the next current vector is W with
// scale 1/beta_k, the next previous one X_cur with coefficient beta_k c1.
// A probe whose beta falls to `tol` or below (an invariant subspace: the
// Gauss rule is exact) stops; its remaining coefficients are 0 and n_steps
// records k + 1.
__global__ void k_lanczos_scalars(int k_batch, int kp, int k, double tol, const double* __restrict__ beta2,
                                  double* __restrict__ lz, int32_t* __restrict__ active, double* __restrict__ beta,
                                  int64_t ld_beta, int32_t* __restrict__ n_steps) {
  const int j = threadIdx.x;
  if (j >= k_batch) return;
  const double b = sqrt(beta2[j] > 0.0 ? beta2[j] : 0.0);
  const bool was = active[j] != 0;
  const bool on = was && b > tol;
  beta[j * ld_beta] = on ? b : 0.0;
  const double c1 = lz[j];
  lz[kp + j] = on ? b * c1 : 0.0;
  lz[j] = on ? 1.0 / b : 0.0;
  if (was && !on) n_steps[j] = k + 1;
  active[j] = on ? 1 : 0;
}

template <typename T, int L>
nd_status launch_lanczos_update(int grid, int64_t n, int kp, int kb, const int64_t* row_ptr, T* W, const T* X,
                                const double* lz, const double* alpha, int64_t ld_alpha, double* partial,
                                hipStream_t st) {
  hipLaunchKernelGGL((k_lanczos_update<T, L>), dim3(grid), dim3(kBlock), 0, st, n, kp, kb, row_ptr, W, X, lz, alpha,
                     ld_alpha, partial);
  ND_LAUNCH_CHECK();
  return ND_OK;
}

template <typename T>
nd_status lanczos_update(int L, int grid, int64_t n, int kp, int kb, const int64_t* row_ptr, T* W, const T* X,
                         const double* lz, const double* alpha, int64_t ld_alpha, double* partial, hipStream_t st) {
  switch (L) {
    case 1: return launch_lanczos_update<T, 1>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
    case 2: return launch_lanczos_update<T, 2>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
    case 4: return launch_lanczos_update<T, 4>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
    case 8: return launch_lanczos_update<T, 8>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
    case 16: return launch_lanczos_update<T, 16>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
    case 32:
      if constexpr (sizeof(T) == 8)
        return launch_lanczos_update<T, 32>(grid, n, kp, kb, row_ptr, W, X, lz, alpha, ld_alpha, partial, st);
      break;
    default: break;
  }
  set_error("internal: unsupported lane count %d", L);
  return ND_EUNSUPPORTED;
}

// alpha, beta: device [k][K]; norm2: device [k] (|z_j|^2 / N); n_steps:
// device int32 [k] (K unless a probe stops early).
template <typename T>
nd_status run_lanczos(nd_graph* g, const MomentJob& job, int K, double* alpha, double* beta, double* norm2,
                      int32_t* n_steps, hipStream_t st) {
  const int64_t N = g->n;
  const double tol = sizeof(T) == 8 ? 1e-10 : 1e-5;
  std::vector<hipEvent_t> evs;
  if (job.timed) {
    g->step_ms = 0.0;
    g->step_launches = 0;
  }
  struct EvFree {
    std::vector<hipEvent_t>& e;
    ~EvFree() {
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
  } ev_free{evs};
  {
    // n_steps = K until a probe stops
    std::vector<int32_t> ks(static_cast<size_t>(job.k), K);
    ND_HIP(hipMemcpyAsync(n_steps, ks.data(), ks.size() * 4, hipMemcpyHostToDevice, st));
    ND_HIP(hipStreamSynchronize(st));
  }
  const int bmax = max_block_probes();
  for (int j0 = 0; j0 < job.k; j0 += bmax) {
    const int kb = job.k - j0 < bmax ? job.k - j0 : bmax;
    BlockSetup<T> bs;
    ND_CHECK(setup_block<T>(g, job, j0, kb, st, bs));
    const int kp = bs.kp, L = bs.L, grid = bs.grid;
    StepArgs& a = bs.a;
    const int64_t per_step = bs.slots * kp;
    ND_CHECK(g->ws_partial.ensure(static_cast<size_t>(per_step) * sizeof(double)));
    double* partial = g->ws_partial.as<double>();
    // scalars: lz [2][kp], beta2 [kp], active (int32) [kp]
    ND_CHECK(g->ws_misc.ensure(static_cast<size_t>(4 * kp) * sizeof(double)));
    double* lz = g->ws_misc.as<double>();
    double* beta2 = lz + 2 * kp;
    int32_t* active = reinterpret_cast<int32_t*>(beta2 + kp);
    Internal* in = g->internal.get();
    // |z|^2 / N per probe: the moment-0 launch of the probe block
    a.first = 1;
    a.xg = nullptr;
    a.xio = nullptr;
    a.partial = partial;
    ND_CHECK(launch_step<T>(L, a, grid, true, st));
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, bs.slots, per_step, 1, kp, kb, 0,
                       job.unit_nodes ? 1.0 : 1.0 / static_cast<double>(N), norm2, int64_t(1),
                       static_cast<int64_t>(j0));
    ND_LAUNCH_CHECK();
    // |z|^2 = norm2 N (norm2 is already |z|^2 for unit probes)
    hipLaunchKernelGGL(k_lanczos_init, dim3(1), dim3(64), 0, st, kb, kp, job.unit_nodes ? 1.0 : static_cast<double>(N),
                       norm2 + j0, lz, active);
    ND_LAUNCH_CHECK();
    a.zmode = 3;
    a.lz = lz;
    for (int k = 0; k < K; ++k) {
      a.m = k + 1;
      a.first = (k == 0) ? 1 : 0;
      T* cur = (k & 1) ? bs.B : bs.A;
      T* prev = (k & 1) ? bs.A : bs.B;
      a.xg = cur;
      a.xio = prev;  // becomes W
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (job.timed) {
        ND_HIP(hipEventCreate(&e0));
        evs.push_back(e0);
        ND_HIP(hipEventCreate(&e1));
        evs.push_back(e1);
        ND_HIP(hipEventRecord(e0, st));
      }
      ND_CHECK(launch_step<T>(L, a, grid, false, st));
      if (job.timed) ND_HIP(hipEventRecord(e1, st));
      hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, bs.slots, per_step, 1, kp, kb, k,
                         1.0, alpha, static_cast<int64_t>(K), static_cast<int64_t>(j0));
      ND_LAUNCH_CHECK();
      if (k == K - 1) break;
      ND_CHECK(lanczos_update<T>(L, grid, N, kp, kb, in->row_ptr, prev, cur, lz, alpha + static_cast<int64_t>(j0) * K + k,
                                 K, partial, st));
      hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, static_cast<int64_t>(grid),
                         per_step, 1, kp, kb, 0, 1.0, beta2, int64_t(1), int64_t(0));
      ND_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_lanczos_scalars, dim3(1), dim3(64), 0, st, kb, kp, k, tol, beta2, lz, active,
                         beta + static_cast<int64_t>(j0) * K + k, static_cast<int64_t>(K), n_steps + j0);
      ND_LAUNCH_CHECK();
    }
  }
  if (job.timed) {
    ND_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i + 1 < evs.size(); i += 2) {
      float ms = 0.f;
      ND_HIP(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      g->step_ms += ms;
      g->step_launches++;
    }
  }
  return ND_OK;
}

// ------------------------------------------------ allocation-free workspace
// The fixed device workspace of nd_cheb_moments_noalloc: every GPU the
// library runs on holds one copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): it takes the device address from hipGetSymbolAddress,
// once per device, and uses that.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

nd_status scratch_address(int dev, char** out) {
  ND_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // the symbol's address is per device: look it up with `dev` current
    int cur = -1;
    ND_HIP(hipGetDevice(&cur));
    if (cur != dev) ND_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) ND_HIP(hipSetDevice(cur));
    ND_HIP(e);
    ND_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the fixed workspace");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return ND_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes the allocation-free path takes from the arena for this call (the
// largest probe block, one launch of moment partials), or an error when a
// probe block has no schedule yet.
template <typename T>
nd_status noalloc_bytes(const nd_graph* g, const MomentJob& job, size_t* need) {
  constexpr int PPL = 16 / sizeof(T);
  const int64_t N = g->n;
  const int M = job.M;
  const int last = job.doubling ? M / 2 : M - 1;
  const int64_t ld_raw = 2 * (static_cast<int64_t>(last) + 1);
  size_t misc = 0;
  if (!job.mu_pp) misc += static_cast<size_t>(job.k) * M;
  if (job.doubling) misc += static_cast<size_t>(job.k) * ld_raw;
  size_t worst = 0;
  const int bmax = max_block_probes();
  for (int j0 = 0; j0 < job.k; j0 += bmax) {
    const int kb = job.k - j0 < bmax ? job.k - j0 : bmax;
    const int kp = pow2_at_least(kb < PPL ? PPL : kb);
    const int L = kp * static_cast<int>(sizeof(T)) / 16;
    auto it = g->sched.find(L);
    if (it == g->sched.end() || !g->internal) {
      set_error("nd_cheb_moments_noalloc: the graph has no row schedule for blocks of %d probes yet: run "
                "nd_cheb_moments once on it with the same probe count first", kp);
      return ND_EINVAL;
    }
    const Schedule* sc = it->second.get();
    const int grid = grid_for(sc->n_items > 0 ? sc->n_items : 1, kWavesPerBlock, step_grid<T>(L));
    const int split_blocks = sc->n_split > 0 ? grid_for(sc->n_split, kWavesPerBlock, grid) : 0;
    const int64_t per_step = (static_cast<int64_t>(grid) + split_blocks) * kp * (job.doubling ? 2 : 1);
    size_t b = align256(3 * static_cast<size_t>(N) * kp * sizeof(T));
    b += align256(static_cast<size_t>(sc->n_chunks > 0 ? sc->n_chunks : 1) * kp * sizeof(double));
    if (!job.gaussian) b += align256(static_cast<size_t>(N) * sizeof(uint64_t));
    b += align256(static_cast<size_t>(per_step) * sizeof(double));
    if (b > worst) worst = b;
  }
  *need = align256(misc * sizeof(double)) + worst;
  return ND_OK;
}

nd_status check_common(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                       uint32_t flags, const char* who) {
  ND_REQUIRE(g != nullptr, "%s: graph is NULL", who);
  ND_REQUIRE(g->n > 0, "%s: the graph has no edges (no node survives)", who);
  ND_REQUIRE(n_probes >= 1, "%s: n_probes=%d must be >= 1", who, n_probes);
  ND_REQUIRE(n_moments >= 1, "%s: n_moments=%d must be >= 1", who, n_moments);
  ND_REQUIRE((flags & ~(ND_PROBE_GAUSSIAN | ND_STATE_FP64 | ND_TIME_STEPS | ND_MOMENT_DOUBLING)) == 0,
             "%s: unknown flags 0x%x", who, flags);
  ND_REQUIRE(motifs == nullptr || motifs->n == g->n, "%s: motifs belong to another graph", who);
  int dev = -1;
  ND_HIP(hipGetDevice(&dev));
  ND_REQUIRE(dev == g->device, "%s: graph lives on device %d, current device is %d", who, g->device, dev);
  return ND_OK;
}

}  // namespace

nd_status lanczos_coefficients(nd_graph* g, const nd_motifs* motifs, const int32_t* unit_nodes, int32_t n_probes,
                               int32_t n_steps, uint64_t seed, uint32_t flags, double* alpha, double* beta,
                               double* norm2, int32_t* steps, hipStream_t st) {
  MomentJob job;
  job.motifs = motifs;
  job.unit_nodes = unit_nodes;
  job.k = n_probes;
  job.M = n_steps;
  job.seed = seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.timed = (flags & ND_TIME_STEPS) != 0;
  if (flags & ND_STATE_FP64) return run_lanczos<double>(g, job, n_steps, alpha, beta, norm2, steps, st);
  return run_lanczos<float>(g, job, n_steps, alpha, beta, norm2, steps, st);
}

nd_status check_moment_args(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                            uint32_t flags, const char* who) {
  return check_common(g, motifs, n_probes, n_moments, flags, who);
}

}  // namespace nd

// ====================================================================== C ABI
extern "C" {

nd_status nd_make_probes(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, uint64_t seed,
                         uint32_t flags, void* Z, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, 1, flags, "nd_make_probes"));
  ND_REQUIRE(Z != nullptr, "nd_make_probes: Z is NULL");
  hipStream_t st = nd::as_stream(stream);
  const bool gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  const int64_t total = g->n * n_probes;
  if (flags & ND_STATE_FP64) {
    hipLaunchKernelGGL(nd::k_probes<double>, dim3(nd::grid_for(total, nd::kBlock)), dim3(nd::kBlock), 0, st, g->n,
                       n_probes, n_probes, int64_t(0), seed, gaussian ? 1 : 0, g->row_ptr,
                       static_cast<const int32_t*>(nullptr), static_cast<double*>(Z), static_cast<double*>(nullptr));
  } else {
    hipLaunchKernelGGL(nd::k_probes<float>, dim3(nd::grid_for(total, nd::kBlock)), dim3(nd::kBlock), 0, st, g->n,
                       n_probes, n_probes, int64_t(0), seed, gaussian ? 1 : 0, g->row_ptr,
                       static_cast<const int32_t*>(nullptr), static_cast<float*>(Z), static_cast<float*>(nullptr));
  }
  ND_LAUNCH_CHECK();
  if (motifs && motifs->n_classes > 0) {
    const int64_t t2 = motifs->n_classes * n_probes;
    if (flags & ND_STATE_FP64)
      hipLaunchKernelGGL(nd::k_project<double>, dim3(nd::grid_for(t2, nd::kBlock)), dim3(nd::kBlock), 0, st,
                         motifs->class_ptr, motifs->members, motifs->n_classes, n_probes, n_probes, g->row_ptr,
                         static_cast<const int32_t*>(nullptr), static_cast<double*>(Z), static_cast<double*>(nullptr),
                         static_cast<double*>(nullptr));
    else
      hipLaunchKernelGGL(nd::k_project<float>, dim3(nd::grid_for(t2, nd::kBlock)), dim3(nd::kBlock), 0, st,
                         motifs->class_ptr, motifs->members, motifs->n_classes, n_probes, n_probes, g->row_ptr,
                         static_cast<const int32_t*>(nullptr), static_cast<float*>(Z), static_cast<float*>(nullptr),
                         static_cast<float*>(nullptr));
    ND_LAUNCH_CHECK();
  }
  return ND_OK;
}

nd_status nd_cheb_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                          uint64_t probe_seed, uint32_t flags, double* mu, double* mu_pp, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, n_moments, flags, "nd_cheb_moments"));
  ND_REQUIRE(mu != nullptr || mu_pp != nullptr, "nd_cheb_moments: mu and mu_pp are both NULL");
  nd::MomentJob job;
  job.motifs = motifs;
  job.k = n_probes;
  job.M = n_moments;
  job.seed = probe_seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.mu = mu;
  job.mu_pp = mu_pp;
  job.timed = (flags & ND_TIME_STEPS) != 0;
  job.doubling = (flags & ND_MOMENT_DOUBLING) != 0;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (flags & ND_STATE_FP64) return nd::run_moments<double>(gm, job, nd::as_stream(stream));
  return nd::run_moments<float>(gm, job, nd::as_stream(stream));
}

nd_status nd_cheb_moments_noalloc(const nd_graph* g, int32_t n_probes, int32_t n_moments, uint64_t probe_seed,
                                  uint32_t flags, double* mu, double* mu_pp, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, nullptr, n_probes, n_moments, flags, "nd_cheb_moments_noalloc"));
  ND_REQUIRE((flags & ND_TIME_STEPS) == 0,
             "nd_cheb_moments_noalloc: ND_TIME_STEPS is not available here (it creates events)");
  ND_REQUIRE(mu != nullptr || mu_pp != nullptr, "nd_cheb_moments_noalloc: mu and mu_pp are both NULL");
  nd::MomentJob job;
  job.k = n_probes;
  job.M = n_moments;
  job.seed = probe_seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.mu = mu;
  job.mu_pp = mu_pp;
  job.doubling = (flags & ND_MOMENT_DOUBLING) != 0;
  const bool f64 = (flags & ND_STATE_FP64) != 0;
  size_t need = 0;
  ND_CHECK(f64 ? nd::noalloc_bytes<double>(g, job, &need) : nd::noalloc_bytes<float>(g, job, &need));
  ND_REQUIRE(need <= nd::kNoAllocBytes,
             "nd_cheb_moments_noalloc: this call needs %zu bytes of workspace, more than the fixed %zu (the "
             "recurrence state alone is 3 x N x padded probes x %d bytes); use nd_cheb_moments",
             need, nd::kNoAllocBytes, f64 ? 8 : 4);
  nd::Arena arena;
  ND_CHECK(nd::scratch_address(g->device, &arena.base));
  arena.cap = nd::kNoAllocBytes;
  job.arena = &arena;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (f64) return nd::run_moments<double>(gm, job, nd::as_stream(stream));
  return nd::run_moments<float>(gm, job, nd::as_stream(stream));
}

nd_status nd_pdos_nodes(const nd_graph* g, const int32_t* nodes, int32_t n_nodes, int32_t n_moments, uint32_t flags,
                        double* pdos, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, nullptr, n_nodes, n_moments, flags, "nd_pdos_nodes"));
  ND_REQUIRE((flags & ~(ND_STATE_FP64 | ND_TIME_STEPS)) == 0, "nd_pdos_nodes: flags 0x%x (only ND_STATE_FP64, "
             "ND_TIME_STEPS apply)", flags);
  ND_REQUIRE(nodes != nullptr && pdos != nullptr, "nd_pdos_nodes: nodes/pdos are NULL");
  hipStream_t st = nd::as_stream(stream);
  {
    std::vector<int32_t> h(static_cast<size_t>(n_nodes));
    ND_HIP(hipMemcpyAsync(h.data(), nodes, h.size() * 4, hipMemcpyDeviceToHost, st));
    ND_HIP(hipStreamSynchronize(st));
    for (int32_t v : h) ND_REQUIRE(v >= 0 && v < g->n, "nd_pdos_nodes: node id %d not in [0, %lld)", v, (long long)g->n);
  }
  nd::MomentJob job;
  job.k = n_nodes;
  job.M = n_moments;
  job.mu_pp = pdos;
  job.unit_nodes = nodes;
  job.timed = (flags & ND_TIME_STEPS) != 0;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (flags & ND_STATE_FP64) return nd::run_moments<double>(gm, job, st);
  return nd::run_moments<float>(gm, job, st);
}

nd_status nd_ldos_moments(const nd_graph* g, const nd_motifs* motifs, int32_t n_probes, int32_t n_moments,
                          uint64_t probe_seed, uint32_t flags, const float* cv_g, double* ldos, double* ldos_sq,
                          double* mu, void* stream) {
  nd::clear_error();
  ND_CHECK(nd::check_common(g, motifs, n_probes, n_moments, flags, "nd_ldos_moments"));
  ND_REQUIRE(ldos != nullptr, "nd_ldos_moments: ldos is NULL");
  ND_REQUIRE((flags & ND_MOMENT_DOUBLING) == 0,
             "nd_ldos_moments: ND_MOMENT_DOUBLING applies to global moments only (the per-node estimate "
             "needs every T_m(H) z)");
  ND_REQUIRE(cv_g == nullptr || motifs == nullptr || motifs->n_classes == 0,
             "nd_ldos_moments: a control variate cannot be combined with twin filtering (a projected probe "
             "entry of a class member has mean square 1/|C|, so g (1 - z_i^2) would bias its row)");
  nd::MomentJob job;
  job.motifs = motifs;
  job.k = n_probes;
  job.M = n_moments;
  job.seed = probe_seed;
  job.gaussian = (flags & ND_PROBE_GAUSSIAN) != 0;
  job.cv_g = cv_g;
  job.ldos = ldos;
  job.ldos_sq = ldos_sq;
  job.mu = mu;
  if (motifs) {
    job.spikes = motifs->spikes_d;
    job.n_spikes = static_cast<int>(motifs->spike_lambda.size());
  }
  job.timed = (flags & ND_TIME_STEPS) != 0;
  nd_graph* gm = const_cast<nd_graph*>(g);
  if (flags & ND_STATE_FP64) return nd::run_moments<double>(gm, job, nd::as_stream(stream));
  return nd::run_moments<float>(gm, job, nd::as_stream(stream));
}

}  // extern "C"
