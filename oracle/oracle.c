/*
 * oracle.c -- plain, slow CPU reference for the event-driven synaptic
 * propagation path of "A differentiable brain simulator bridging brain
 * simulation and brain-inspired computing" (BrainPy, ICLR 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header, table or constant with the GPU library: everything here is written
 * from the paper (and from the published definition of Philox-4x32-10) in
 * straightforward loops, in FP64 unless a function says otherwise.
 *
 * What each function follows:
 *   - or_philox / or_hash ........ Philox-4x32-10 (Salmon, Moraes, Dror, Shaw,
 *                                   SC'11), the counter-based source of every
 *                                   random draw of the method (the paper's
 *                                   listing of Appendix C draws from a seeded
 *                                   generator; a counter-based one keeps the
 *                                   matrix identical across calls, which the
 *                                   listing's caption requires).
 *                                   Pinned by the generator's published
 *                                   known-answer vectors and statistically
 *                                   (uniformity, avalanche, independence).
 *   - or_max_gap ................. Appendix C: gaps are uniform on [1, K] with
 *                                   K = floor(2/p - 1) (the text; the listing
 *                                   says ceil), mean 1/p.
 *   - or_row_block / or_row ...... Appendix C listing (with the fixes listed
 *                                   in the design notes) plus the block
 *                                   extension with a stationary first point.
 *   - or_csr_build ............... the CSR of Appendix B built from those rows.
 *   - or_compact ................. Appendix B: work happens only where the
 *                                   spike vector is true; the compacted list is
 *                                   that set in ascending order.
 *   - or_event_csr_* ............. Appendix B (event csrmv), definition y = M^T e.
 *   - or_jit_* ................... Appendix C / Section 4.2 and 5.2 (JIT
 *                                   connectivity, homogeneous / normal /
 *                                   uniform weights).
 *   - or_*_vjp ................... Section 4.1: reverse-mode derivative of the
 *                                   (linear) operators.
 *   - or_net_* ................... Appendix N (E/I balanced COBA-LIF network),
 *                                   Appendix F (LIF and conductance equations),
 *                                   Appendix E (exact exponential synapse).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10                                                           */
/* ------------------------------------------------------------------------ */

/* One Philox round on a 4-word counter: two 32x32->64 products, the high
 * halves are mixed with the other two words and the round key, and the words
 * are permuted. */
static void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k0;
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k1;
  uint32_t n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

/* Ten rounds; the key is bumped by the Weyl constants between rounds. */
void or_philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* H(seed, stream, a, b, k): word (k mod 4) of Philox-4x32-10 with
 * key = (low 32 bits of seed, high 32 bits of seed) and
 * counter = (a, b, floor(k / 4), stream). */
uint32_t or_hash(uint64_t seed, uint32_t stream, uint32_t a, uint32_t b, uint32_t k) {
  uint32_t ctr[4] = {a, b, k >> 2, stream};
  uint32_t out[4];
  or_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
  return out[k & 3u];
}

/* Batched form for statistical tests: ctr [n][4], key [n][2], out [n][4]. */
void or_philox_many(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) or_philox(ctr + 4 * i, key[2 * i], key[2 * i + 1], out + 4 * i);
}

void or_hash_many(uint64_t seed, uint32_t stream, const uint32_t* a, const uint32_t* b,
                  const uint32_t* k, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = or_hash(seed, stream, a[i], b[i], k[i]);
}

/* Random-stream identifiers. */
enum { OR_STREAM_CONN = 1, OR_STREAM_W = 2, OR_STREAM_V0 = 3 };

/* ------------------------------------------------------------------------ */
/* Appendix C: the maximum gap K                                            */
/* ------------------------------------------------------------------------ */

/* x = 2/p - 1 in FP64.  A value within 1e-9 relative of an integer is that
 * integer (so p = 0.02 gives 99 despite rounding); otherwise floor(x), the
 * text's rule.  K >= 1.  Returns -1 for p outside (0, 1]. */
int32_t or_max_gap(double p) {
  if (!(p > 0.0) || p > 1.0) return -1;
  double x = 2.0 / p - 1.0;
  double r = floor(x + 0.5);
  double K = (fabs(x - r) <= 1e-9 * x) ? r : floor(x);
  if (K < 1.0) K = 1.0;
  if (K > 2147483646.0) return -1;
  return (int32_t)K;
}

/* Uniform integer on {0, ..., m-1} from one 32-bit word (multiply-shift). */
static uint32_t below(uint32_t word, uint32_t m) {
  return (uint32_t)(((uint64_t)word * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Appendix C: one row (or one post block of a row) of the JIT matrix        */
/* ------------------------------------------------------------------------ */

/*
 * Positions of row j inside post block b, written to out (if non-NULL) in
 * increasing order; returns how many.  Draw i of the (j, b) sequence is
 * H(seed, CONN, j, b, i).
 *
 * B == 0 (one block covering [0, n_post)) is the paper's procedure: the first
 * target is one gap minus one (0-based), every further target is one more gap
 * later, gaps uniform on [1, K], stop at n_post.
 *
 * B > 0 restarts the procedure at each block [b*B, min((b+1)*B, n_post)).
 * The first target of a block is the block start plus min(ra, rb) with ra
 * uniform on {0..K-1} and rb uniform on {0..K}: that is the distance to the
 * first point of a stationary renewal process with gaps uniform on [1, K]
 * (P(R >= r) = (K-r)(K-r+1)/(K(K+1))), so every block has exactly the
 * expected density 2/(K+1).  Draws 0 and 1 give ra and rb, draw 2 on are gaps.
 */
int64_t or_row_block(uint64_t seed, int32_t K, int32_t n_post, int32_t B, int32_t j,
                     int32_t b, int32_t* out) {
  int64_t start, end, pos;
  uint32_t i;
  if (B > 0) {
    start = (int64_t)b * B;
    end = start + B;
    if (end > n_post) end = n_post;
    uint32_t ra = below(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, (uint32_t)b, 0), (uint32_t)K);
    uint32_t rb = below(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, (uint32_t)b, 1), (uint32_t)K + 1u);
    pos = start + (ra < rb ? ra : rb);
    i = 2;
  } else {
    start = 0;
    end = n_post;
    pos = (int64_t)below(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, 0, 0), (uint32_t)K);
    i = 1;
  }
  int64_t cnt = 0;
  while (pos < end) {
    if (out) out[cnt] = (int32_t)pos;
    ++cnt;
    pos += 1 + (int64_t)below(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, (uint32_t)b, i), (uint32_t)K);
    ++i;
  }
  return cnt;
}

static int32_t n_blocks(int32_t n_post, int32_t B) {
  return B > 0 ? (int32_t)(((int64_t)n_post + B - 1) / B) : 1;
}

/* Whole row j: the blocks in order. */
int64_t or_row(uint64_t seed, int32_t K, int32_t n_post, int32_t B, int32_t j, int32_t* out) {
  int64_t cnt = 0;
  int32_t nb = n_blocks(n_post, B);
  for (int32_t b = 0; b < nb; ++b) cnt += or_row_block(seed, K, n_post, B, j, b, out ? out + cnt : NULL);
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* Exact-statistics connectivity rules                                       */
/* ------------------------------------------------------------------------ */

/*
 * Two alternatives to the paper's uniform gaps, each a connectivity rule of
 * its own (a different matrix for the same seed):
 *
 * Rule 1, geometric gaps (Appendix C names them as the exact way to draw a
 * Bernoulli(p) process: the distance to the next connection is Geo[p],
 * sampled by inverting the CDF, gap = 1 + floor(log(U) / log(1 - p))).  Every
 * position is then connected independently with probability p, up to the
 * resolution of U (24 bits: gaps longer than 16.6 / p, probability 2^-24,
 * are cut there).  The logarithm decides an integer, so it is evaluated by a
 * fixed sequence of IEEE single-precision operations, ln_f32 below, the same
 * on every device; 1 / (-log(1 - p)) is computed once in FP64 and rounded to
 * FP32 (inv_rate).  Block restarts keep the law exactly: the gap process is
 * memoryless, so the first target of a block is its start plus gap - 1.
 *
 * Rule 2, exactly fixed out-degree k (each row connects to exactly k
 * distinct targets, each k-subset of [0, n_post) drawn by a keyed
 * pseudo-random permutation): target i of row j, i < k, is pi_j(i) with pi_j
 * a permutation of [0, n_post) built by cycle walking (Black and Rogaway,
 * "Ciphers with arbitrary finite domains", CT-RSA 2002) over a four-round
 * alternating Feistel network on [0, 2^b), 2^b the smallest power of two
 * >= n_post (halves of b - b/2 and b/2 bits), whose round function is the
 * 32-bit finalizer of MurmurHash3 (Appleby) applied to the other half xor a
 * round key; the four round keys are the four words of Philox block
 * (j, 0, 0, CONN).  Targets come in index order (not sorted); one post block
 * (B = 0) only.
 */

/* ln(k 2^-24) for k in [1, 2^24]: k = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(s), s = (m - 1) / (m + 1), by its series to s^9; each step is
 * one IEEE single-precision operation in the order written. */
float or_ln_f32(uint32_t k) {
  int e = 31 - __builtin_clz(k);
  float m = (float)k;
  /* m 2^-e, exact (a power-of-two scaling of an integer below 2^25) */
  m = m * ldexpf(1.0f, -e);
  if (m > 1.41421356f) {
    m = m * 0.5f;
    e += 1;
  }
  const float f = m - 1.0f;
  const float s = f / (2.0f + f);
  const float z = s * s;
  float poly = 0.222222222f;            /* 2/9 */
  poly = 0.285714286f + z * poly;       /* 2/7 */
  poly = 0.4f + z * poly;               /* 2/5 */
  poly = 0.666666667f + z * poly;       /* 2/3 */
  poly = 2.0f + z * poly;
  const float lnm = s * poly;
  const float ef = (float)(e - 24);
  return ef * 0.693145752f + (ef * 1.42860677e-06f + lnm); /* ln 2 = 0.693145752 + 1.42860677e-6 */
}

void or_ln_f32_many(const uint32_t* k, float* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = or_ln_f32(k[i]);
}

/* 1 / (-ln(1 - p)) in FP64, rounded once to FP32; 0 for p outside (0, 1). */
float or_geo_inv_rate(double p) {
  if (!(p > 0.0) || !(p < 1.0)) return 0.0f;
  return (float)(1.0 / -log1p(-p));
}

/* Geometric gap from one 32-bit word: 1 + floor(-ln(U) inv_rate), U =
 * ((w >> 8) + 1) 2^-24 in (0, 1], capped at 2^30. */
uint32_t or_geo_gap(uint32_t w, float inv_rate) {
  const float L = -or_ln_f32((w >> 8) + 1u);
  const float t = L * inv_rate;
  if (!(t < 1073741824.0f)) return 1073741824u;
  return 1u + (uint32_t)t;
}

void or_geo_gap_many(const uint32_t* w, float inv_rate, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = or_geo_gap(w[i], inv_rate);
}

static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

/* Bits b of the Feistel domain [0, 2^b): the smallest b >= 2 with 2^b >= n. */
static uint32_t fd_bits(int32_t n) {
  uint32_t b = 2;
  while (b < 31 && ((uint64_t)1 << b) < (uint64_t)n) ++b;
  return b;
}

/* pi(i) for the row whose round keys are key[0..3], i < n: x in [0, 2^b) is
 * split into a high part L of b - b/2 bits and a low part R of b/2 bits;
 * four alternating rounds L ^= F(R ^ key0), R ^= F(L ^ key1), L ^= F(R ^ key2),
 * R ^= F(L ^ key3), F the finalizer cut to the part's width (each round is
 * invertible, so the network permutes [0, 2^b)); values >= n are sent through
 * the network again until they land below n (cycle walking). */
uint32_t or_fd_target(const uint32_t key[4], int32_t n, uint32_t i) {
  const uint32_t b = fd_bits(n);
  const uint32_t hr = b / 2, hl = b - hr;
  const uint32_t ml = (1u << hl) - 1u, mr = (1u << hr) - 1u;
  uint32_t x = i;
  do {
    uint32_t L = x >> hr, R = x & mr;
    L ^= fmix32(R ^ key[0]) & ml;
    R ^= fmix32(L ^ key[1]) & mr;
    L ^= fmix32(R ^ key[2]) & ml;
    R ^= fmix32(L ^ key[3]) & mr;
    x = (L << hr) | R;
  } while (x >= (uint32_t)n);
  return x;
}

/* Positions of row j inside post block b under `rule` (0: the paper's
 * uniform gaps, or_row_block; 1: geometric gaps; 2: exactly `degree`
 * targets, block 0 only), in generation order; returns how many.  Target m
 * of (j, b) in this order is connection m of the JIT weight streams. */
int64_t or_rule_row_block(uint64_t seed, int32_t rule, int32_t K, float inv_rate, int32_t degree,
                          int32_t n_post, int32_t B, int32_t j, int32_t b, int32_t* out) {
  if (rule == 0) return or_row_block(seed, K, n_post, B, j, b, out);
  if (rule == 2) {
    if (b != 0 || n_post <= 0) return 0;
    uint32_t key[4];
    const uint32_t ctr[4] = {(uint32_t)j, 0u, 0u, OR_STREAM_CONN};
    or_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), key);
    const int32_t k = degree < n_post ? degree : n_post;
    for (int32_t i = 0; i < k; ++i)
      if (out) out[i] = (int32_t)or_fd_target(key, n_post, (uint32_t)i);
    return k;
  }
  /* rule 1: draw 0 places the first target gap - 1 after the block start,
   * every later draw is one more gap */
  int64_t start = B > 0 ? (int64_t)b * B : 0;
  int64_t end = B > 0 ? start + B : n_post;
  if (end > n_post) end = n_post;
  int64_t pos = start + (int64_t)or_geo_gap(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, (uint32_t)b, 0), inv_rate) - 1;
  uint32_t i = 1;
  int64_t cnt = 0;
  while (pos < end) {
    if (out) out[cnt] = (int32_t)pos;
    ++cnt;
    pos += (int64_t)or_geo_gap(or_hash(seed, OR_STREAM_CONN, (uint32_t)j, (uint32_t)b, i), inv_rate);
    ++i;
  }
  return cnt;
}

/* The whole matrix of a rule as CSR in generation order: row j holds its
 * blocks in order, blk[e] / idx[e] give each entry's block and its index in
 * the block's generation order (the JIT weight coordinates).  Returns nnz,
 * or -1 if it exceeds cap; indices / blk / idx may be NULL to count. */
int64_t or_rule_csr(uint64_t seed, int32_t rule, int32_t K, float inv_rate, int32_t degree, int32_t n_pre,
                    int32_t n_post, int32_t B, int32_t* indptr, int32_t* indices, int32_t* blk, int32_t* idx,
                    int64_t cap) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  const int32_t nb = rule == 2 ? 1 : n_blocks(n_post, B);
  int64_t nnz = 0;
  indptr[0] = 0;
  for (int32_t j = 0; j < n_pre; ++j) {
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = or_rule_row_block(seed, rule, K, inv_rate, degree, n_post, B, j, b, buf);
      if (nnz + c > cap) {
        free(buf);
        return -1;
      }
      for (int64_t m = 0; m < c; ++m) {
        if (indices) indices[nnz + m] = buf[m];
        if (blk) blk[nnz + m] = b;
        if (idx) idx[nnz + m] = (int32_t)m;
      }
      nnz += c;
    }
    indptr[j + 1] = (int32_t)nnz;
  }
  free(buf);
  return nnz;
}

/* ------------------------------------------------------------------------ */
/* Appendix B: CSR (data, indices, indptr) built from the seeded rows        */
/* ------------------------------------------------------------------------ */

/* Row lengths; returns nnz. */
int64_t or_csr_count(uint64_t seed, int32_t K, int32_t n_pre, int32_t n_post, int32_t B,
                     int32_t* rowlen) {
  int64_t nnz = 0;
  for (int32_t j = 0; j < n_pre; ++j) {
    int64_t c = or_row(seed, K, n_post, B, j, NULL);
    if (rowlen) rowlen[j] = (int32_t)c;
    nnz += c;
  }
  return nnz;
}

/* indptr[n_pre+1], indices[nnz]; returns nnz or -1 if it exceeds cap. */
int64_t or_csr_build(uint64_t seed, int32_t K, int32_t n_pre, int32_t n_post, int32_t B,
                     int32_t* indptr, int32_t* indices, int64_t cap) {
  int64_t nnz = 0;
  indptr[0] = 0;
  for (int32_t j = 0; j < n_pre; ++j) {
    int64_t c = or_row(seed, K, n_post, B, j, NULL);
    if (nnz + c > cap) return -1;
    or_row(seed, K, n_post, B, j, indices + nnz);
    nnz += c;
    indptr[j + 1] = (int32_t)nnz;
  }
  return nnz;
}

/* ------------------------------------------------------------------------ */
/* Spike compaction                                                          */
/* ------------------------------------------------------------------------ */

int32_t or_compact(const uint8_t* s, int32_t n, int32_t* ids) {
  int32_t c = 0;
  for (int32_t j = 0; j < n; ++j)
    if (s[j]) ids[c++] = j;
  return c;
}

/* ------------------------------------------------------------------------ */
/* Appendix B: event-driven CSR matvec, y = M^T e                            */
/* ------------------------------------------------------------------------ */

/* y[k] = sum over rows j with e[j] != 0 of the entries of row j in column k
 * (data[idx], or w when data is NULL).  y is overwritten. */
void or_event_csr_matvec(const int32_t* indptr, const int32_t* indices, const float* data, double w,
                         int32_t n_pre, int32_t n_post, const uint8_t* ev, double* y) {
  for (int32_t k = 0; k < n_post; ++k) y[k] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (!ev[j]) continue;
    for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx)
      y[indices[idx]] += data ? (double)data[idx] : w;
  }
}

/* Integer count of firing rows reaching each column (homogeneous case). */
void or_event_csr_counts(const int32_t* indptr, const int32_t* indices, int32_t n_pre, int32_t n_post,
                         const uint8_t* ev, int64_t* cnt) {
  for (int32_t k = 0; k < n_post; ++k) cnt[k] = 0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (!ev[j]) continue;
    for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) cnt[indices[idx]] += 1;
  }
}

/* Reverse mode of y = M^T e (Section 4.1):
 *   d_ev[j]     = sum over row j of M[j,k] * dy[k]            (every row)
 *   d_data[idx] = e[j] * dy[indices[idx]]                       (firing rows)
 *   d_w         = sum over firing rows of sum over the row of dy (data NULL) */
void or_event_csr_vjp(const int32_t* indptr, const int32_t* indices, const float* data, double w,
                      int32_t n_pre, int32_t n_post, const uint8_t* ev, const double* dy,
                      double* d_ev, double* d_data, double* d_w) {
  (void)n_post;
  double gw = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    double acc = 0.0, accw = 0.0;
    for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) {
      double m = data ? (double)data[idx] : w;
      acc += m * dy[indices[idx]];
      accw += dy[indices[idx]];
      if (d_data) d_data[idx] = ev[j] ? dy[indices[idx]] : 0.0;
    }
    if (d_ev) d_ev[j] = acc;
    if (ev[j]) gw += accw;
  }
  if (d_w) *d_w = gw;
}

/* ------------------------------------------------------------------------ */
/* Appendix C, Section 5.2: JIT connectivity matvec                           */
/* ------------------------------------------------------------------------ */

enum { OR_W_HOMO = 0, OR_W_NORMAL = 1, OR_W_UNIFORM = 2 };

/* Uniform on (0, 1] and [0, 1) from the top 24 bits of a word. */
static double u_open0(uint32_t word) { return ((double)(word >> 8) + 1.0) * (1.0 / 16777216.0); }
static double u_open1(uint32_t word) { return (double)(word >> 8) * (1.0 / 16777216.0); }

/* Weight of connection m (0-based, in generation order) of row j, block b.
 * Homogeneous: w0.  Uniform: w0 + (w1 - w0) u.  Normal: w0 + w1 z with z from
 * Box-Muller on draws 2q and 2q+1 of stream W, q = m / 2 (cosine half for
 * even m, sine half for odd m).  Also returns the unit draw
 * (u, or z) in *unit for the reverse mode. */
double or_jit_weight(uint64_t seed, int32_t wkind, double w0, double w1, int32_t j, int32_t b,
                     int64_t m, double* unit) {
  if (wkind == OR_W_NORMAL) {
    /* Box-Muller, both halves of each pair: targets 2q and 2q + 1 share the
     * draws 2q, 2q + 1 and take r cos(2 pi u2) and r sin(2 pi u2). */
    const int64_t q = m >> 1;
    double u1 = u_open0(or_hash(seed, OR_STREAM_W, (uint32_t)j, (uint32_t)b, (uint32_t)(2 * q)));
    double u2 = u_open1(or_hash(seed, OR_STREAM_W, (uint32_t)j, (uint32_t)b, (uint32_t)(2 * q + 1)));
    double r = sqrt(-2.0 * log(u1));
    double z = (m & 1) ? r * sin(2.0 * M_PI * u2) : r * cos(2.0 * M_PI * u2);
    if (unit) *unit = z;
    return w0 + w1 * z;
  }
  if (wkind == OR_W_UNIFORM) {
    double u = u_open1(or_hash(seed, OR_STREAM_W, (uint32_t)j, (uint32_t)b, (uint32_t)m));
    if (unit) *unit = u;
    return w0 + (w1 - w0) * u;
  }
  if (unit) *unit = 1.0;
  return w0;
}

/* w[e] = weight of entry e of a rule CSR in generation order (row j, block
 * blk[e], index idx[e]): the JIT weight kinds, FP64. */
void or_rule_weights(uint64_t seed, int32_t wkind, double w0, double w1, int32_t n_pre, const int32_t* indptr,
                     const int32_t* blk, const int32_t* idx, double* w) {
  for (int32_t j = 0; j < n_pre; ++j)
    for (int32_t e = indptr[j]; e < indptr[j + 1]; ++e)
      w[e] = or_jit_weight(seed, wkind, w0, w1, j, blk[e], idx[e], NULL);
}

/* y[k] = sum over firing rows j of the weight of (j, k) if connected. */
void or_jit_matvec(uint64_t seed, int32_t K, int32_t B, int32_t wkind, double w0, double w1,
                   int32_t n_pre, int32_t n_post, const uint8_t* ev, double* y) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  for (int32_t k = 0; k < n_post; ++k) y[k] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (!ev[j]) continue;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t m = 0; m < c; ++m) y[buf[m]] += or_jit_weight(seed, wkind, w0, w1, j, b, m, NULL);
    }
  }
  free(buf);
}

/* Float-vector JIT product (Section 5.2: y = J v with J given by its
 * probability, weight distribution and seed; every row j contributes its
 * weights times v[j]; rows with v[j] == 0 contribute nothing). */
void or_jit_matvec_dense(uint64_t seed, int32_t K, int32_t B, int32_t wkind, double w0, double w1,
                         int32_t n_pre, int32_t n_post, const double* v, double* y) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  for (int32_t k = 0; k < n_post; ++k) y[k] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (v[j] == 0.0) continue;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t m = 0; m < c; ++m) y[buf[m]] += or_jit_weight(seed, wkind, w0, w1, j, b, m, NULL) * v[j];
    }
  }
  free(buf);
}

/* Batched form (Section 5.2's operator on m vectors at once): Y = J^T X with
 * X row-major [n_pre][m] and Y row-major [n_post][m]; column c of Y is the
 * float-vector product of column c of X, each in the same row order. */
void or_jit_matmat_dense(uint64_t seed, int32_t K, int32_t B, int32_t wkind, double w0, double w1,
                         int32_t n_pre, int32_t n_post, int32_t m, const double* X, double* Y) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  for (int64_t i = 0; i < (int64_t)n_post * m; ++i) Y[i] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    const double* x = X + (size_t)j * m;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t cnt = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t t = 0; t < cnt; ++t) {
        const double w = or_jit_weight(seed, wkind, w0, w1, j, b, t, NULL);
        for (int32_t c = 0; c < m; ++c)
          if (x[c] != 0.0) Y[(size_t)buf[t] * m + c] += w * x[c];
      }
    }
  }
  free(buf);
}

/* Sum of the magnitudes of the terms of the batched product:
 * S[k][c] = sum over rows j of (|a_jk| + |b_jk|) |X[j][c]|, X row-major
 * [n_pre][m], where w_jk = a_jk + b_jk are the two terms of the weight
 * formula (Section 5.2's distributions): a = w0, b = w1 z (normal),
 * b = (w1 - w0) u (uniform), b = 0 (homogeneous).  An FP32 evaluation of the
 * weight errs by a multiple of the unit roundoff times |a| + |b| (more than
 * |w| times it when the two terms cancel), and FP32 sums of the products
 * w_jk X[j][c] by a multiple of it times the sum of their magnitudes, so
 * parity tolerances are stated relative to S.  m = 1 serves the
 * single-vector products (X = v, or the spike vector as 0/1). */
void or_jit_abs_terms(uint64_t seed, int32_t K, int32_t B, int32_t wkind, double w0, double w1,
                      int32_t n_pre, int32_t n_post, int32_t m, const double* X, double* S) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  for (int64_t i = 0; i < (int64_t)n_post * m; ++i) S[i] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    const double* x = X + (size_t)j * m;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t cnt = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t t = 0; t < cnt; ++t) {
        double unit = 0.0;
        (void)or_jit_weight(seed, wkind, w0, w1, j, b, t, &unit);
        const double tb = wkind == OR_W_NORMAL ? w1 * unit : wkind == OR_W_UNIFORM ? (w1 - w0) * unit : 0.0;
        const double w = fabs(w0) + fabs(tb);
        for (int32_t c = 0; c < m; ++c) S[(size_t)buf[t] * m + c] += w * fabs(x[c]);
      }
    }
  }
  free(buf);
}

void or_jit_counts(uint64_t seed, int32_t K, int32_t B, int32_t n_pre, int32_t n_post,
                   const uint8_t* ev, int64_t* cnt) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  for (int32_t k = 0; k < n_post; ++k) cnt[k] = 0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (!ev[j]) continue;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t m = 0; m < c; ++m) cnt[buf[m]] += 1;
    }
  }
  free(buf);
}

/* Reverse mode of the JIT matvec:
 *   d_ev[j] = sum over the row of w_jk dy[k]                  (every row)
 *   d_w0, d_w1: derivatives with respect to the two weight parameters,
 *   summed over firing rows (homogeneous: d_w0 = sum dy, d_w1 = 0;
 *   normal: d_mu = sum dy, d_sigma = sum z dy; uniform: d_lo = sum (1-u) dy,
 *   d_hi = sum u dy). */
void or_jit_vjp(uint64_t seed, int32_t K, int32_t B, int32_t wkind, double w0, double w1,
                int32_t n_pre, int32_t n_post, const uint8_t* ev, const double* dy, double* d_ev,
                double* d_w0, double* d_w1) {
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_post > 0 ? n_post : 1));
  int32_t nb = n_blocks(n_post, B);
  double g0 = 0.0, g1 = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    double acc = 0.0;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = or_row_block(seed, K, n_post, B, j, b, buf);
      for (int64_t m = 0; m < c; ++m) {
        double unit;
        double wjk = or_jit_weight(seed, wkind, w0, w1, j, b, m, &unit);
        double g = dy[buf[m]];
        acc += wjk * g;
        if (ev[j]) {
          if (wkind == OR_W_NORMAL) { g0 += g; g1 += unit * g; }
          else if (wkind == OR_W_UNIFORM) { g0 += (1.0 - unit) * g; g1 += unit * g; }
          else { g0 += g; }
        }
      }
    }
    if (d_ev) d_ev[j] = acc;
  }
  if (d_w0) *d_w0 = g0;
  if (d_w1) *d_w1 = g1;
  free(buf);
}

/* ------------------------------------------------------------------------ */
/* Appendix N / F / E: the E/I LIF network                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t model;   /* 0 conductance-based (COBA), 1 current-based (CUBA) */
  int32_t n, n_exc;
  int32_t conn;    /* 0 stored CSR (indptr/indices passed in), 1 regenerated (JIT) */
  int32_t max_gap, block;
  uint64_t seed;
  float w_exc, w_inh;
  float tau_m, tau_e, tau_i, tau_ref;
  float v_rest, v_th, v_reset, e_exc, e_inh, r, i_ext, dt;
  float v0_lo, v0_hi;
} or_net;

/* V0[k] = v0_lo + (v0_hi - v0_lo) u_k in FP64 with u_k the top 24 bits of
 * H(seed, V0, k, 0, 0) over 2^24, rounded once to FP32. */
void or_net_v0(const or_net* P, float* V) {
  for (int32_t k = 0; k < P->n; ++k) {
    double u = u_open1(or_hash(P->seed, OR_STREAM_V0, (uint32_t)k, 0, 0));
    V[k] = (float)((double)P->v0_lo + ((double)P->v0_hi - (double)P->v0_lo) * u);
  }
}

int32_t or_net_ref_steps(const or_net* P) {
  return (int32_t)floor((double)P->tau_ref / (double)P->dt + 0.5);
}

/* Counts of excitatory and inhibitory firing presynaptic rows reaching each
 * neuron: the synaptic input of one step (one-step delay: s_prev are the
 * spikes of the previous step).
 * The rows are independent and the counts are integers, so the OpenMP build
 * of this file (the CPU baseline) deals the rows to threads and adds the
 * counts atomically: the same counts in any order.  A plain build ignores
 * the pragmas and runs the loops as written. */
static void net_inputs(const or_net* P, const int32_t* indptr, const int32_t* indices,
                       const uint8_t* s_prev, int64_t* ce, int64_t* ci, int64_t* events) {
  int32_t n = P->n;
  int32_t nb = n_blocks(n, P->block);
  int64_t ev = 0;
  for (int32_t k = 0; k < n; ++k) { ce[k] = 0; ci[k] = 0; }
#pragma omp parallel reduction(+ : ev)
  {
    int32_t* buf = P->conn == 0 ? NULL : (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 256)
    for (int32_t j = 0; j < n; ++j) {
      if (!s_prev[j]) continue;
      int64_t* c = (j < P->n_exc) ? ce : ci;
      if (P->conn == 0) {
        for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) {
#pragma omp atomic
          c[indices[idx]] += 1;
        }
        ev += indptr[j + 1] - indptr[j];
      } else {
        for (int32_t b = 0; b < nb; ++b) {
          int64_t m = or_row_block(P->seed, P->max_gap, n, P->block, j, b, buf);
          for (int64_t q = 0; q < m; ++q) {
#pragma omp atomic
            c[buf[q]] += 1;
          }
          ev += m;
        }
      }
    }
    free(buf);
  }
  *events += ev;
}

/* Threads the network loops may use: the OpenMP build sets and reports them
 * (threads <= 0 keeps the runtime's default), a plain build always has one. */
int32_t or_set_threads(int32_t threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  return (int32_t)omp_get_max_threads();
#else
  (void)threads;
  return 1;
#endif
}

/*
 * T steps in FP32, every operation rounded to FP32 in this order (the spike
 * threshold decision is taken in the precision the GPU computes in):
 *   ge = ge*d_e + (float)ce*w_e ;  gi = gi*d_i + (float)ci*w_i     (Appendix E)
 *   refractory: ref -= 1, no spike, V held
 *   else: I = ge*(E_e - V) + gi*(E_i - V) + I_ext   (COBA, Appendix F)
 *         I = ge + gi + I_ext                        (CUBA)
 *         V = V + a*((V_rest - V) + R*I)             (forward Euler)
 *         spike if V > V_th: V = V_reset, ref = ref_steps
 * with d_e = exp(-dt/tau_e), d_i = exp(-dt/tau_i), a = dt/tau_m computed in
 * FP64 and rounded to FP32.  iext_vec (nullable) adds a per-neuron current.
 */
void or_net_run_f32(const or_net* P, const int32_t* indptr, const int32_t* indices, int32_t T,
                    float* V, float* ge, float* gi, int32_t* ref, uint8_t* s_prev,
                    const float* iext_vec, uint8_t* raster, int32_t* counts, int64_t* events) {
  int32_t n = P->n;
  float de = (float)exp(-(double)P->dt / (double)P->tau_e);
  float di = (float)exp(-(double)P->dt / (double)P->tau_i);
  float a = (float)((double)P->dt / (double)P->tau_m);
  int32_t ref_steps = or_net_ref_steps(P);
  int64_t* ce = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* ci = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  uint8_t* s = (uint8_t*)malloc((size_t)n);
  int64_t ev = 0;
  for (int32_t t = 0; t < T; ++t) {
    net_inputs(P, indptr, indices, s_prev, ce, ci, &ev);
    int32_t cnt = 0;
#pragma omp parallel for reduction(+ : cnt)
    for (int32_t k = 0; k < n; ++k) {
      float xe = (float)ce[k] * P->w_exc;
      float xi = (float)ci[k] * P->w_inh;
      ge[k] = ge[k] * de + xe;
      gi[k] = gi[k] * di + xi;
      s[k] = 0;
      if (ref[k] > 0) {
        ref[k] -= 1;
      } else {
        float iext = P->i_ext;
        if (iext_vec) iext = iext + iext_vec[k];
        float I;
        if (P->model == 0) I = ge[k] * (P->e_exc - V[k]) + gi[k] * (P->e_inh - V[k]) + iext;
        else I = ge[k] + gi[k] + iext;
        float v = V[k] + a * ((P->v_rest - V[k]) + P->r * I);
        if (v > P->v_th) {
          s[k] = 1;
          v = P->v_reset;
          ref[k] = ref_steps;
        }
        V[k] = v;
      }
      cnt += s[k];
    }
    memcpy(s_prev, s, (size_t)n);
    if (raster) memcpy(raster + (size_t)t * n, s, (size_t)n);
    if (counts) counts[t] = cnt;
  }
  if (events) *events = ev;
  free(ce); free(ci); free(s);
}

/* The same recursion carried in FP64 (parameters are the FP32 values, the
 * constants d_e, d_i, a are FP64).  Used to measure how far the FP32 result
 * is from the exact-arithmetic trajectory. */
void or_net_run_f64(const or_net* P, const int32_t* indptr, const int32_t* indices, int32_t T,
                    double* V, double* ge, double* gi, int32_t* ref, uint8_t* s_prev,
                    const double* iext_vec, uint8_t* raster, int32_t* counts, int64_t* events) {
  int32_t n = P->n;
  double de = exp(-(double)P->dt / (double)P->tau_e);
  double di = exp(-(double)P->dt / (double)P->tau_i);
  double a = (double)P->dt / (double)P->tau_m;
  int32_t ref_steps = or_net_ref_steps(P);
  int64_t* ce = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* ci = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  uint8_t* s = (uint8_t*)malloc((size_t)n);
  int64_t ev = 0;
  for (int32_t t = 0; t < T; ++t) {
    net_inputs(P, indptr, indices, s_prev, ce, ci, &ev);
    int32_t cnt = 0;
#pragma omp parallel for reduction(+ : cnt)
    for (int32_t k = 0; k < n; ++k) {
      ge[k] = ge[k] * de + (double)ce[k] * (double)P->w_exc;
      gi[k] = gi[k] * di + (double)ci[k] * (double)P->w_inh;
      s[k] = 0;
      if (ref[k] > 0) {
        ref[k] -= 1;
      } else {
        double iext = (double)P->i_ext + (iext_vec ? iext_vec[k] : 0.0);
        double I;
        if (P->model == 0) I = ge[k] * ((double)P->e_exc - V[k]) + gi[k] * ((double)P->e_inh - V[k]) + iext;
        else I = ge[k] + gi[k] + iext;
        double v = V[k] + a * (((double)P->v_rest - V[k]) + (double)P->r * I);
        if (v > (double)P->v_th) {
          s[k] = 1;
          v = (double)P->v_reset;
          ref[k] = ref_steps;
        }
        V[k] = v;
      }
      cnt += s[k];
    }
    memcpy(s_prev, s, (size_t)n);
    if (raster) memcpy(raster + (size_t)t * n, s, (size_t)n);
    if (counts) counts[t] = cnt;
  }
  if (events) *events = ev;
  free(ce); free(ci); free(s);
}
