// Device-side building blocks shared by the kernels: the Philox-4x32-10
// counter-based generator, the seeded row/block generator of the
// fixed-probability connectivity, wave64 primitives and device-coherent
// accesses used for cross-workgroup exchange.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bp {

constexpr int kWave = 64;
constexpr uint32_t kStreamConn = 1, kStreamW = 2, kStreamV0 = 3;
constexpr int kWHomo = 0, kWNormal = 1, kWUniform = 2;

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products mixed into the other two counter words and the round
// key; the key advances by the golden-ratio Weyl constants between rounds.
// ---------------------------------------------------------------------------
// Four named words (not an array: a select over array elements can be turned
// into an indexed private-memory load, i.e. scratch traffic in inner loops).
struct Words4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                           uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const Words4& q, uint32_t i) {
  const uint32_t lo = (i & 1u) ? q.y : q.x;
  const uint32_t hi = (i & 1u) ? q.w : q.z;
  return (i & 2u) ? hi : lo;
}

// hash(seed, stream, a, b, k): word k mod 4 of Philox(counter (a, b, k/4, stream)).
__device__ __forceinline__ uint32_t hash_word(uint64_t seed, uint32_t stream, uint32_t a, uint32_t b, uint32_t k) {
  return pick(philox10(a, b, k >> 2, stream, (uint32_t)seed, (uint32_t)(seed >> 32)), k);
}

// Sequential reader of the draws of one (a, b) sub-stream: one Philox call
// per four draws.
struct DrawSeq {
  uint32_t k0, k1, a, b, stream;
  uint32_t blk;
  Words4 cur;
  __device__ __forceinline__ DrawSeq(uint64_t seed, uint32_t stream_, uint32_t a_, uint32_t b_)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), a(a_), b(b_), stream(stream_), blk(0xFFFFFFFFu) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t i) {
    const uint32_t want = i >> 2;
    if (want != blk) {
      blk = want;
      cur = philox10(a, b, want, stream, k0, k1);
    }
    return pick(cur, i);
  }
};

// Uniform integer on {0..m-1} from one word (multiply-shift).
__device__ __forceinline__ uint32_t below(uint32_t word, uint32_t m) { return __umulhi(word, m); }

// u in (0, 1] and [0, 1) from the top 24 bits (exact in FP32).
__device__ __forceinline__ float u_open0(uint32_t w) { return (float)((w >> 8) + 1u) * (1.0f / 16777216.0f); }
__device__ __forceinline__ float u_open1(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// Connectivity rules.  0: the paper's sampler (gaps uniform on [1, K]).
// 1: geometric gaps, the exact Bernoulli(p) process (gap = 1 +
// floor(-ln(U) / -ln(1 - p)), the logarithm by the fixed FP32 operation
// sequence of ln_f32 so that every device decides the same gaps).
// 2: exactly `degree` distinct targets per row (one post block): target i is
// pi_j(i) for a keyed permutation of the columns: four alternating Feistel
// rounds over the high b - b/2 and low b/2 bits of [0, 2^b), 2^b the smallest
// power of two >= n_post, whose round function is MurmurHash3's 32-bit
// finalizer of the other part xor a round key, cycle-walked into [0, n_post)
// (Black and Rogaway, CT-RSA 2002); the round keys are the four words of
// Philox block (j, 0, 0, CONN).
// ---------------------------------------------------------------------------
constexpr int kRuleUniform = 0, kRuleGeometric = 1, kRuleFixedDegree = 2;

struct ConnGen {
  uint64_t seed;
  uint32_t K;        // rule 0
  int32_t n_post, B;
  int32_t rule;
  float inv_rate;    // rule 1: 1 / -ln(1 - p), FP32
  int32_t degree;    // rule 2
};

// ln(k 2^-24) for k in [1, 2^24]: k = m 2^e, m folded into
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s), s = (m - 1) / (m + 1), by its
// series to s^9; every step one IEEE single-precision operation in this order
// (contraction is disabled for the library; the division is correctly
// rounded), with ln 2 split into a head of 16 bits and a tail.
__device__ __forceinline__ float ln_f32(uint32_t k) {
  int e = 31 - __clz((int)k);
  float m = (float)k * __uint_as_float((uint32_t)(127 - e) << 23);  // k 2^-e, exact
  if (m > 1.41421356f) {
    m = m * 0.5f;
    e += 1;
  }
  const float f = m - 1.0f;
  const float s = f / (2.0f + f);
  const float z = s * s;
  float poly = 0.222222222f;
  poly = 0.285714286f + z * poly;
  poly = 0.4f + z * poly;
  poly = 0.666666667f + z * poly;
  poly = 2.0f + z * poly;
  const float lnm = s * poly;
  const float ef = (float)(e - 24);
  return ef * 0.693145752f + (ef * 1.42860677e-06f + lnm);
}

// Geometric gap from one word: 1 + floor(-ln(U) inv_rate), U = ((w >> 8) + 1)
// 2^-24, capped at 2^30.
__device__ __forceinline__ uint32_t geo_gap(uint32_t w, float inv_rate) {
  const float t = -ln_f32((w >> 8) + 1u) * inv_rate;
  return t < 1073741824.0f ? 1u + (uint32_t)t : 1073741824u;
}

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Bits b of the Feistel domain [0, 2^b): the smallest b >= 2 with 2^b >= n.
__device__ __forceinline__ uint32_t fd_bits(int32_t n) {
  const uint32_t b = n > 1 ? 32u - (uint32_t)__clz(n - 1) : 0u;
  return b < 2u ? 2u : b;
}

// pi(i), i < n, for the round keys `key` on [0, 2^b): a high part of
// b - b/2 bits and a low part of b/2 bits, four alternating rounds (each
// xors one part with the finalizer of the other part and a key, cut to the
// part's width), cycle-walked until the value lands below n.
__device__ __forceinline__ uint32_t fd_target(const Words4& key, uint32_t b, int32_t n, uint32_t i) {
  const uint32_t hr = b >> 1, hl = b - hr;
  const uint32_t ml = (1u << hl) - 1u, mr = (1u << hr) - 1u;
  uint32_t x = i;
  do {
    uint32_t L = x >> hr, R = x & mr;
    L ^= fmix32(R ^ key.x) & ml;
    R ^= fmix32(L ^ key.y) & mr;
    L ^= fmix32(R ^ key.z) & ml;
    R ^= fmix32(L ^ key.w) & mr;
    x = (L << hr) | R;
  } while (x >= (uint32_t)n);
  return x;
}

__device__ __forceinline__ Words4 fd_keys(uint64_t seed, uint32_t j) {
  return philox10(j, 0u, 0u, kStreamConn, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// Positions of row j inside post block b of the connectivity (rule 0: gaps
// uniform on [1, K]; block == 0: one block, first target = gap - 1; block >
// 0: stationary start block_start + min(ra, rb); rule 1: first target gap - 1
// after the block start, then geometric gaps; rule 2: the degree targets of
// the row in index order), restricted to the window [lo, hi).  emit(pos, m)
// receives every target in the window, m being its index among all targets
// of (j, b) in generation order (the JIT weight coordinate).
// ---------------------------------------------------------------------------
template <int RULE, class Emit>
__device__ __forceinline__ void gen_walk(const ConnGen& g, uint32_t j, uint32_t b, int64_t lo, int64_t hi,
                                         Emit&& emit) {
  DrawSeq d(g.seed, kStreamConn, j, b);
  int64_t start, end, pos;
  uint32_t i;
  if (g.B > 0) {
    start = (int64_t)b * g.B;
    end = start + g.B;
    if (end > g.n_post) end = g.n_post;
  } else {
    start = 0;
    end = g.n_post;
  }
  if constexpr (RULE == kRuleGeometric) {
    pos = start + (int64_t)geo_gap(d(0), g.inv_rate) - 1;
    i = 1;
  } else if (g.B > 0) {
    const uint32_t ra = below(d(0), g.K);
    const uint32_t rb = below(d(1), g.K + 1u);
    pos = start + (int64_t)(ra < rb ? ra : rb);
    i = 2;
  } else {
    pos = (int64_t)below(d(0), g.K);
    i = 1;
  }
  if (hi < end) end = hi;
  uint32_t m = 0;
  while (pos < end) {
    if (pos >= lo) emit((int32_t)pos, m);
    ++m;
    if constexpr (RULE == kRuleGeometric) pos += (int64_t)geo_gap(d(i), g.inv_rate);
    else pos += 1 + (int64_t)below(d(i), g.K);
    ++i;
  }
}

// Rule 0 alone with the parameters passed one by one (the network kernel's
// lean variant, whose register allocation the general form above disturbs).
template <class Emit>
__device__ __forceinline__ void gen_block_uniform(uint64_t seed, uint32_t K, int32_t n_post, int32_t B, uint32_t j,
                                                  uint32_t b, int64_t lo, int64_t hi, Emit&& emit) {
  DrawSeq d(seed, kStreamConn, j, b);
  int64_t start, end, pos;
  uint32_t i;
  if (B > 0) {
    start = (int64_t)b * B;
    end = start + B;
    if (end > n_post) end = n_post;
    const uint32_t ra = below(d(0), K);
    const uint32_t rb = below(d(1), K + 1u);
    pos = start + (int64_t)(ra < rb ? ra : rb);
    i = 2;
  } else {
    start = 0;
    end = n_post;
    pos = (int64_t)below(d(0), K);
    i = 1;
  }
  if (hi < end) end = hi;
  uint32_t m = 0;
  while (pos < end) {
    if (pos >= lo) emit((int32_t)pos, m);
    ++m;
    pos += 1 + (int64_t)below(d(i), K);
    ++i;
  }
}

template <class Emit>
__device__ __forceinline__ void gen_block(const ConnGen& g, uint32_t j, uint32_t b, int64_t lo, int64_t hi,
                                          Emit&& emit) {
  if (g.rule == kRuleFixedDegree) {
    if (b != 0u) return;
    const Words4 key = fd_keys(g.seed, j);
    const uint32_t fb = fd_bits(g.n_post);
    const int32_t k = g.degree < g.n_post ? g.degree : g.n_post;
    for (int32_t i = 0; i < k; ++i) {
      const int32_t t = (int32_t)fd_target(key, fb, g.n_post, (uint32_t)i);
      if (t >= lo && t < hi) emit(t, (uint32_t)i);
    }
  } else if (g.rule == kRuleGeometric) {
    gen_walk<kRuleGeometric>(g, j, b, lo, hi, emit);
  } else {
    gen_walk<kRuleUniform>(g, j, b, lo, hi, emit);
  }
}

// Weight of connection m of (j, b) for the JIT weight kinds, read from the
// W sub-stream of (j, b) through `wd` (connections are visited in increasing
// m, so one Philox call serves four normal or four uniform weights); *unit
// receives the unit draw (z or u) for the reverse mode.
__device__ __forceinline__ float jit_weight(DrawSeq& wd, int wkind, float w0, float w1, uint32_t m, float* unit) {
  if (wkind == kWNormal) {
    // Box-Muller with the hardware log2 / sqrt / cos(2 pi x) instructions;
    // connections 2q and 2q + 1 share draws 2q, 2q + 1 and take the cosine
    // and the sine half (sin(2 pi x) = cos(2 pi (x - 1/4)); x - 1/4 is exact
    // for x on the 2^-24 grid)
    const uint32_t q = m >> 1;
    const uint32_t wa = wd(2u * q), wb = wd(2u * q + 1u);
    const float u1 = u_open0(wa), u2 = u_open1(wb);
    const float x = u2 - ((m & 1u) ? 0.25f : 0.0f);
    const float z = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1)) * __builtin_amdgcn_cosf(x);
    *unit = z;
    return w0 + w1 * z;
  }
  if (wkind == kWUniform) {
    const float u = u_open1(wd(m));
    *unit = u;
    return w0 + (w1 - w0) * u;
  }
  *unit = 1.0f;
  return w0;
}

// ---------------------------------------------------------------------------
// wave64 / workgroup primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int mask_rank(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum across the wave with DPP: shifts by 1, 2, 4, 8 inside
// each row of 16 lanes, then the last lane of row 0 / 2 is added to rows 1 / 3
// (row_bcast:15) and the last lane of row 1 to rows 2 and 3 (row_bcast:31).
// Lanes without a source keep the `old` operand, 0.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Exclusive prefix sum over the workgroup; *total receives the sum.
// `scratch` holds at least blockDim.x / 64 + 1 ints of LDS.
__device__ __forceinline__ int block_excl_scan(int v, int* scratch, int* total) {
  const int l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int inc = wave_incl_scan(v);
  if (l == kWave - 1) scratch[w] = inc;
  __syncthreads();
  if (w == 0) {
    const int s = (l < nw) ? scratch[l] : 0;
    const int si = wave_incl_scan(s);
    if (l < nw) scratch[l] = si - s;
    if (l == nw - 1) scratch[nw] = si;
  }
  __syncthreads();
  const int r = scratch[w] + inc - v;
  *total = scratch[nw];
  __syncthreads();
  return r;
}

// Two exclusive prefix sums over the workgroup sharing one set of barriers.
// `scratch` holds at least 2 * (blockDim.x / 64 + 1) ints of LDS.
__device__ __forceinline__ void block_excl_scan2(int a, int b, int* scratch, int* ea, int* eb, int* ta, int* tb) {
  const int l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  int* sa = scratch;
  int* sb = scratch + nw + 1;
  if (l == kWave - 1) {
    sa[w] = ia;
    sb[w] = ib;
  }
  __syncthreads();
  if (w == 0) {
    const int xa = (l < nw) ? sa[l] : 0, xb = (l < nw) ? sb[l] : 0;
    const int ya = wave_incl_scan(xa), yb = wave_incl_scan(xb);
    if (l < nw) {
      sa[l] = ya - xa;
      sb[l] = yb - xb;
    }
    if (l == nw - 1) {
      sa[nw] = ya;
      sb[nw] = yb;
    }
  }
  __syncthreads();
  *ea = sa[w] + ia - a;
  *eb = sb[w] + ib - b;
  *ta = sa[nw];
  *tb = sb[nw];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Device-coherent accesses for data exchanged between workgroups of one
// launch (possibly on different XCDs, whose L2 caches are not coherent with
// each other).  These compile to sc1 loads/stores that bypass the
// non-coherent L2 state, without the L2 writeback/invalidate that an
// agent-scope fence performs.  A writer makes its coherent stores complete
// (vm_drain) before the workgroup barrier that precedes its flag store; a
// reader issues its coherent data loads only after it has observed the flag.
// ---------------------------------------------------------------------------
// FP32 add into LDS by compare-and-swap: on gfx950 the native LDS float
// atomic add runs about 8x slower than this loop at low contention.
__device__ __forceinline__ void lds_add_f32(float* p, float v) {
  uint32_t* q = reinterpret_cast<uint32_t*>(p);
  uint32_t old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (true) {
    const uint32_t seen = old;
    old = atomicCAS(q, seen, __float_as_uint(__uint_as_float(seen) + v));
    if (old == seen) break;
  }
}

// Device-coherent (agent scope) relaxed loads and stores through the global
// address space: global_* instructions count only in vmcnt, so a workgroup
// barrier (which waits for lgkmcnt) never waits for them, as it would for
// the generic flat_* forms.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ int ld_coh(const int* p) {
  return __hip_atomic_load(as_global(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh(const uint32_t* p) {
  return __hip_atomic_load(as_global(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int* p, int v) {
  __hip_atomic_store(as_global(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(uint32_t* p, uint32_t v) {
  __hip_atomic_store(as_global(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_coh64(const uint64_t* p) {
  return __hip_atomic_load(as_global(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(as_global(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// 16-byte device-coherent accesses through a raw buffer resource (one
// buffer_load/store_dwordx4 with sc1, the same coherence as the 8-byte forms
// above).  The resource spans `bytes` bytes from `base`; offsets beyond it
// read zeros and drop the store.  The base is made wave-uniform here (a
// buffer resource lives in scalar registers).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t coh_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = (uint64_t)base;
  const uint64_t u = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
  return __builtin_amdgcn_make_buffer_rsrc((void*)u, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                           0x00020000);
}
constexpr int kCohSc1 = 16;  // cache-policy operand of the buffer builtins: sc1
__device__ __forceinline__ void ld_coh128(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t* a, uint64_t* b) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kCohSc1);
  *a = ((uint64_t)v.y << 32) | v.x;
  *b = ((uint64_t)v.w << 32) | v.z;
}
__device__ __forceinline__ void st_coh128(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t a, uint64_t b) {
  u32x4 v;
  v.x = (uint32_t)a;
  v.y = (uint32_t)(a >> 32);
  v.z = (uint32_t)b;
  v.w = (uint32_t)(b >> 32);
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kCohSc1);
}
// Wait until every vector memory operation this wave issued has completed
// (s_waitcnt vmcnt(0); stores are counted by vmcnt on gfx9-family targets).
// The compiler barriers keep the memory operations on their own side.
__device__ __forceinline__ void vm_drain() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace bp
