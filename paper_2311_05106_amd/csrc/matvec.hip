// Event-driven CSR matvec (Appendix B), JIT-connectivity matvec (Appendix C,
// Section 5.2) on spike vectors and on dense float vectors, and their reverse
// modes (Section 4.1).  The float-vector product lists the rows with
// v[j] != 0 (64 bytes of v per lane and sweep) in place of the firing rows
// and scales each generated weight by v[j]; it always sums in FP32.
//
// Forward layout: the postsynaptic range is cut into tiles of P columns that
// fit in LDS, the presynaptic range into C chunks of rows.  Workgroup
// (tile, chunk) sweeps the spike bytes of its rows 16 per lane (one 16-byte
// load), appends the firing rows to an LDS list (wave scan + one LDS atomic
// per wave, so one barrier per sweep), and when the list is nearly full or
// the rows are done, streams the part of every listed row that falls in its
// tile into its LDS accumulator (integer counts for homogeneous weights,
// FP32 otherwise).  With one chunk the tile is written to y directly; with
// several, each chunk stores its tile to a partial buffer (16-bit counts when
// homogeneous: a chunk adds at most one per row to any column) and a second
// kernel sums the partials in chunk order (no global atomics: device atomics
// run far below HBM rate on this chip).
//   CSR segments are streamed by quarter-waves (16 lanes), several rows per
//   group at once (40 loads in flight per lane for counts, the next rows'
//   bounds fetched ahead), so a wave reads four segments per instruction,
//   coalesced.
//   JIT rows are regenerated per (row, block) by one lane each (a lane whose
//   walk leaves the block takes the next listed row, so the lanes of a wave
//   do not wait for its longest walk), or by four lanes (one generator call
//   each, positions by a quad prefix sum) when a pass lists at most 256
//   rows; the tile is one block, so no lane generates targets outside its
//   tile.
#include <mutex>

#include "bp_device.h"
#include "bp_host.h"

namespace bp {

constexpr int kMvThreads = 1024;
constexpr int kRowsPerLane = 16;                   // one 16-byte load of spike bytes
constexpr int kSweep = kMvThreads * kRowsPerLane;  // rows examined per sweep
constexpr int kIdCap = kSweep + 4096;              // firing rows listed before a flush
constexpr int kTileMax = 16384;                    // LDS tile columns (64 KB)
constexpr int kGroup = 16;                         // lanes streaming one CSR segment
constexpr int kSegLoads = 10;                      // loads per lane and segment pass (160 entries)
constexpr int kMinChunkRows = 256;                 // row chunks of small operators
constexpr int64_t kSmallPartialBytes = 4 << 20;    // partials those may use

enum MvMode {
  kCsrHomo = 0, kCsrData = 1, kJitHomo = 2, kJitWeighted = 3, kJitVec = 4, kJitMat = 5,
  // batched spike products: the same four operators on `batch` spike
  // vectors at once, up to kMatCols per workgroup (blockIdx.y = group)
  kCsrHomoB = 6, kCsrDataB = 7, kJitHomoB = 8, kJitWeightedB = 9,
  // stored CSR on a dense float vector: y = M^T v over the rows with v[j] != 0
  kCsrVec = 16
};
constexpr int kMatCols = 8;  // kJitMat / batched: columns per workgroup
constexpr bool is_batch(int m) { return m >= kCsrHomoB && m <= kJitWeightedB; }
constexpr int base_mode(int m) { return is_batch(m) ? m - kCsrHomoB : m; }
constexpr bool counts_mode(int m) { return base_mode(m) == kCsrHomo || base_mode(m) == kJitHomo; }

struct MvArgs {
  const int32_t* indptr;
  const int32_t* indices;
  const float* data;
  const int32_t* tile_ptr;  // [n_pre][n_tiles + 1] or null (single tile)
  const uint8_t* events;
  const float* vec;         // kJitVec: dense input vector (rows with v[j] != 0 are listed)
  const float* x;           // kJitMat: X row-major [n_pre][m] (every row is listed)
  int32_t m, mg;            // kJitMat: columns of X, columns per group
  int32_t batch, mb;        // batched: spike vectors, vectors per group
  int64_t ev_stride, y_stride;  // batched: bytes between spike vectors, floats between outputs
  void* out;                // y (chunks == 1) or partials [chunks][n_post]
  bp_jit_conn jit;
  float w;
  int32_t n_pre, n_post;
  int32_t tile, n_tiles;    // tile width P, number of tiles
  int32_t chunks, chunk_rows;
  int32_t search;           // sorted CSR without a tile index: find each row's tile segment in the kernel
};

// Segment [*first, *last) of the sorted row [b, e) whose columns lie in
// [x0, x1), found by the 16 lanes of one quarter-wave (gl = lane in the group,
// gshift = first bit of the group in a wave ballot): each round every lane
// probes one of 16 evenly spaced entries for each bound, so a row of n
// entries takes about log16(n) rounds of one load per lane and bound.
// Every lane of the group must call it with the same arguments.
__device__ __forceinline__ void group_bounds(const int32_t* __restrict__ idx, int32_t b, int32_t e, int32_t x0,
                                             int32_t x1, int gl, int gshift, int32_t* first, int32_t* last) {
  int32_t b0 = b, e0 = e, b1 = b, e1 = e;
  bool d0 = false, d1 = false;
  while (!(d0 && d1)) {
    // the answer of bound i lies in [bi, ei]; entries at or past ei are not
    // below xi (or do not exist)
    const int32_t n0 = e0 - b0, n1 = e1 - b1;
    const int32_t s0 = n0 <= 16 ? 1 : (n0 + 15) >> 4, s1 = n1 <= 16 ? 1 : (n1 + 15) >> 4;
    const int32_t q0 = b0 + (gl + 1) * s0 - 1, q1 = b1 + (gl + 1) * s1 - 1;
    const bool lt0 = !d0 && q0 < e0 && idx[q0] < x0;
    const bool lt1 = !d1 && q1 < e1 && idx[q1] < x1;
    const int c0 = __popc((uint32_t)(__ballot(lt0) >> gshift) & 0xFFFFu);
    const int c1 = __popc((uint32_t)(__ballot(lt1) >> gshift) & 0xFFFFu);
    if (!d0) {
      b0 += c0 * s0;
      if (s0 == 1) d0 = true;
      else e0 = min(e0, b0 + s0 - 1);
    }
    if (!d1) {
      b1 += c1 * s1;
      if (s1 == 1) d1 = true;
      else e1 = min(e1, b1 + s1 - 1);
    }
  }
  *first = b0;
  *last = b1;
}

struct MvShared {
  int ids[kIdCap];
  int cnt[3];  // per-sweep append counters, rotated so one barrier per sweep suffices
  int grab;    // next listed row of the balanced JIT walks
};

// Bit q set iff byte q of v is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t v) {
  const uint32_t t = (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
  return (t >> 7 | t >> 14 | t >> 21 | t >> 28) & 0xFu;
}

// Bit q set iff row r + q < r_end fires.
__device__ __forceinline__ uint32_t spike_bits16(const uint8_t* __restrict__ ev, int32_t r, int32_t r_end,
                                                 bool vec) {
  if (vec && r + kRowsPerLane <= r_end) {
    const uint4 v = *reinterpret_cast<const uint4*>(ev + r);
    return nonzero_bytes(v.x) | nonzero_bytes(v.y) << 4 | nonzero_bytes(v.z) << 8 | nonzero_bytes(v.w) << 12;
  }
  uint32_t b = 0;
  for (int q = 0; q < kRowsPerLane; ++q)
    if (r + q < r_end && ev[r + q]) b |= 1u << q;
  return b;
}

// Bit q set iff row r + q < r_end has v[r + q] != 0 (sign bit ignored, so
// -0 is zero and NaN is not).
__device__ __forceinline__ uint32_t nonzero_floats16(const float* __restrict__ v, int32_t r, int32_t r_end,
                                                     bool vec) {
  uint32_t b = 0;
  if (vec && r + kRowsPerLane <= r_end) {
    const uint4* p = reinterpret_cast<const uint4*>(v + r);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 x = p[i];
      b |= (uint32_t)((x.x << 1) != 0u) << (4 * i) | (uint32_t)((x.y << 1) != 0u) << (4 * i + 1) |
           (uint32_t)((x.z << 1) != 0u) << (4 * i + 2) | (uint32_t)((x.w << 1) != 0u) << (4 * i + 3);
    }
    return b;
  }
  for (int q = 0; q < kRowsPerLane; ++q)
    if (r + q < r_end && v[r + q] != 0.f) b |= 1u << q;
  return b;
}

// Appends entry(q) for every set bit q of bits to ids[total + ...]: one LDS
// atomic per wave reserves the wave's slots, a wave scan places each lane's
// rows.  entry(q) is the row r + q, or for batched products
// (r + q) << 8 | (bit b set iff vector b of the group fires row r + q).
template <class Entry>
__device__ __forceinline__ void append_rows(uint32_t bits, int total, int* cnt, int* ids, Entry&& entry) {
  const int c = __popc(bits);
  const int inc = wave_incl_scan(c);
  const int wtot = __builtin_amdgcn_readlane(inc, kWave - 1);
  if (wtot == 0) return;
  int base = 0;
  if (lane_id() == kWave - 1) base = atomicAdd(cnt, wtot);
  base = __builtin_amdgcn_readlane(base, kWave - 1);
  int off = total + base + inc - c;
  while (bits) {
    const int q = __ffs(bits) - 1;
    bits &= bits - 1;
    if (off < kIdCap) ids[off] = entry(q);
    ++off;
  }
}

// Batched products, one target of a row firing in the group's vectors
// `mask` (bit b: vector b) at LDS offset off.  Counts: two vectors per
// 32-bit word (vector b in word b / 2, half b % 2; a row chunk adds at most
// 65520 to a column, host plan), so one add serves a pair.  Sums: vector b
// at acc[b * width + off].
__device__ __forceinline__ void batch_count(uint32_t* acc, int off, int width, uint32_t mask) {
#pragma unroll
  for (int q = 0; q < kMatCols / 2; ++q) {
    const uint32_t inc = ((mask >> (2 * q)) & 1u) | (((mask >> (2 * q + 1)) & 1u) << 16);
    if (inc) atomicAdd(&acc[q * width + off], inc);
  }
}
__device__ __forceinline__ void batch_sum(float* acc, int off, int width, uint32_t mask, float v) {
#pragma unroll
  for (int b = 0; b < kMatCols; ++b)
    if ((mask >> b) & 1u) lds_add_f32(&acc[b * width + off], v);
}

// The factor(s) of one listed row: v[j] for kJitVec, X[j][c0 .. c0 + mg)
// for kJitMat (clamped loads, masked adds), 1 for kJitWeighted.
template <int MODE>
struct RowScale {
  float v[MODE == kJitMat ? kMatCols : 1];
  __device__ __forceinline__ void load(const MvArgs& a, uint32_t j, int c0, int mg) {
    if constexpr (MODE == kJitMat) {
      const float* row = a.x + (size_t)j * a.m + c0;
#pragma unroll
      for (int cc = 0; cc < kMatCols; ++cc) v[cc] = row[cc < mg ? cc : mg - 1];
    } else if constexpr (MODE == kJitVec) {
      v[0] = a.vec[j];
    } else {
      v[0] = 1.f;
    }
  }
  // kJitMat: acc holds column cc of the group at acc[cc * width .. + width)
  // (column-major, so the lanes of one add hit banks spread by their random
  // offsets; a row-major [width][8] tile put all 64 on 4 of the banks)
  __device__ __forceinline__ void add(float* acc, int off, float w, int mg, int width) const {
    if constexpr (MODE == kJitMat) {
#pragma unroll
      for (int cc = 0; cc < kMatCols; ++cc)
        if (cc < mg) lds_add_f32(&acc[cc * width + off], w * v[cc]);
    } else {
      lds_add_f32(&acc[off], w * v[0]);
    }
  }
};

// One generated target of a JIT row at LDS offset off: a count (homogeneous),
// or the m-th weight of the row's W sub-stream times the row's factor(s);
// batched products add to the vectors in mk.
template <int MODE>
__device__ __forceinline__ void jit_put(void* accv, int off, int width, uint32_t mk, const RowScale<MODE>& sc,
                                        DrawSeq& wd, int wkind, float w0, float w1, uint32_t m, int mg) {
  if constexpr (MODE == kJitHomo) {
    atomicAdd(reinterpret_cast<uint32_t*>(accv) + off, 1u);
  } else if constexpr (MODE == kJitHomoB) {
    batch_count(reinterpret_cast<uint32_t*>(accv), off, width, mk);
  } else {
    float unit;
    const float w = jit_weight(wd, wkind, w0, w1, m, &unit);
    if constexpr (MODE == kJitWeightedB) batch_sum(reinterpret_cast<float*>(accv), off, width, mk, w);
    else sc.add(reinterpret_cast<float*>(accv), off, w, mg, width);
  }
}

template <int MODE>
__global__ void __launch_bounds__(kMvThreads) mv_scatter_k(MvArgs a) {
  constexpr bool kB = is_batch(MODE);
  constexpr int BM = base_mode(MODE);
  using Acc = typename std::conditional<counts_mode(MODE), uint32_t, float>::type;
  __shared__ Acc acc[kTileMax];
  __shared__ MvShared sh;
  const int t = blockIdx.x % a.n_tiles;
  const int c = blockIdx.x / a.n_tiles;
  const int32_t lo = t * a.tile;
  const int32_t hi = min(lo + a.tile, a.n_post);
  const int32_t width = hi - lo;
  const int32_t r_begin = c * a.chunk_rows;
  const int32_t r_end = min(r_begin + a.chunk_rows, a.n_pre);
  const int c0 = MODE == kJitMat ? (int)blockIdx.y * a.mg : kB ? (int)blockIdx.y * a.mb : 0;
  const int mg = MODE == kJitMat ? min(a.mg, a.m - c0) : kB ? min(a.mb, a.batch - c0) : 1;
  // LDS words per column: mg floats (kJitMat, batched sums), mg / 2 rounded
  // up for batched counts, else 1; width * words <= kTileMax (host plan)
  const int words = (kB && counts_mode(MODE)) ? (mg + 1) / 2 : (MODE == kJitMat || kB) ? mg : 1;
  for (int i = threadIdx.x; i < (width * words + 3) / 4; i += kMvThreads)  // kTileMax is a multiple of 4
    reinterpret_cast<uint4*>(acc)[i] = make_uint4(0u, 0u, 0u, 0u);
  if (threadIdx.x < 3) sh.cnt[threadIdx.x] = 0;
  __syncthreads();
  constexpr bool kFV = MODE == kJitVec || MODE == kCsrVec;  // rows listed where v[j] != 0
  const uintptr_t src = kFV ? reinterpret_cast<uintptr_t>(a.vec) : reinterpret_cast<uintptr_t>(a.events);
  const bool vec = ((src | (uintptr_t)r_begin | (kB ? (uintptr_t)a.ev_stride : 0)) & 15) == 0;
  const uint8_t* evg = kB ? a.events + (size_t)c0 * a.ev_stride : a.events;  // the group's first vector

  int total = 0;  // listed rows, equal in every lane
  int s = 0;
  for (int32_t r0 = r_begin; r0 < r_end; r0 += kSweep, ++s) {
    const int32_t r = r0 + (int32_t)threadIdx.x * kRowsPerLane;
    uint32_t bits = 0u;
    uint32_t vb[kB ? kMatCols : 1] = {};  // batched: the spike bits of each vector of the group
    if (r < r_end) {
      if constexpr (MODE == kJitMat) {
        bits = r + kRowsPerLane <= r_end ? 0xFFFFu : (1u << (r_end - r)) - 1u;
      } else if constexpr (kFV) {
        bits = nonzero_floats16(a.vec, r, r_end, vec);
      } else if constexpr (kB) {
#pragma unroll
        for (int b = 0; b < kMatCols; ++b) {
          vb[b] = b < mg ? spike_bits16(evg + (size_t)b * a.ev_stride, r, r_end, vec) : 0u;
          bits |= vb[b];
        }
      } else {
        bits = spike_bits16(a.events, r, r_end, vec);
      }
    }
    // the counter of the next sweep was last read before the previous barrier
    if (threadIdx.x == 0) sh.cnt[(s + 1) % 3] = 0;
    if constexpr (kB) {
      append_rows(bits, total, &sh.cnt[s % 3], sh.ids, [&](int q) {
        uint32_t mk = 0;
#pragma unroll
        for (int b = 0; b < kMatCols; ++b) mk |= ((vb[b] >> q) & 1u) << b;
        return (int)((uint32_t)(r + q) << 8 | mk);
      });
    } else {
      append_rows(bits, total, &sh.cnt[s % 3], sh.ids, [&](int q) { return r + q; });
    }
    __syncthreads();
    total += sh.cnt[s % 3];
    if (total <= kIdCap - kSweep && r0 + kSweep < r_end) continue;
    if (total > kIdCap) total = kIdCap;  // unreachable: a sweep adds at most kSweep rows

    if constexpr (BM == kCsrHomo || BM == kCsrData || BM == kCsrVec) {
      // quarter-wave g streams the segments of rows g, g + G, ...; lane l
      // reads entries l, l + 16, ... of a segment.  Rows go in batches of R
      // per group: the loads of all R segments (kSegLoads per lane, 160
      // entries each) are issued together, then the bounds of the next batch,
      // then the LDS adds; the rare entries beyond 160 follow row by row.
      constexpr int R = BM == kCsrHomo ? 4 : 2;
      constexpr bool kLoadVal = BM == kCsrData || BM == kCsrVec;  // per-entry values (kCsrVec: data or w)
      constexpr int U = kSegLoads;
      constexpr int kPass = kGroup * U;
      const int G = kMvThreads / kGroup;
      const int g = threadIdx.x / kGroup, l = threadIdx.x % kGroup;
      auto segment = [&](int i, int& st, int& ln, uint32_t& mk) {
        st = 0;
        ln = 0;
        mk = 0;
        if (i >= total) return;
        const int32_t id = sh.ids[i];
        const int32_t j = kB ? (int32_t)((uint32_t)id >> 8) : id;
        if constexpr (kB) mk = (uint32_t)id & 0xFFu;
        if constexpr (MODE == kCsrVec) mk = __float_as_uint(a.vec[j]);  // the row's factor v[j]
        if (a.tile_ptr) {
          const int32_t* tp = a.tile_ptr + (size_t)j * (a.n_tiles + 1) + t;
          st = tp[0];
          ln = tp[1] - st;
        } else if (a.search) {
          int32_t en;
          group_bounds(a.indices, a.indptr[j], a.indptr[j + 1], lo, hi, l, lane_id() & ~(kGroup - 1), &st, &en);
          ln = en - st;
        } else {
          st = a.indptr[j];
          ln = a.indptr[j + 1] - st;
        }
      };
      auto add = [&](int c, float v, uint32_t mk) {
        if constexpr (MODE == kCsrHomo) atomicAdd(&acc[c - lo], 1u);
        else if constexpr (MODE == kCsrData) lds_add_f32(&acc[c - lo], v);
        else if constexpr (MODE == kCsrVec) lds_add_f32(&acc[c - lo], v * __uint_as_float(mk));
        else if constexpr (MODE == kCsrHomoB) batch_count(reinterpret_cast<uint32_t*>(acc), c - lo, width, mk);
        else batch_sum(reinterpret_cast<float*>(acc), c - lo, width, mk, v);
      };
      int st[R], ln[R];
      uint32_t mk[R];
#pragma unroll
      for (int r = 0; r < R; ++r) segment(g + r * G, st[r], ln[r], mk[r]);
      for (int i0 = g; i0 < total; i0 += R * G) {
        int col[R][U];
        float val[R][U];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = l + kGroup * u;
            col[r][u] = e < ln[r] ? a.indices[st[r] + e] : -1;
            if constexpr (BM == kCsrData) val[r][u] = e < ln[r] ? a.data[st[r] + e] : 0.f;
            if constexpr (BM == kCsrVec) val[r][u] = a.data ? (e < ln[r] ? a.data[st[r] + e] : 0.f) : a.w;
          }
        }
        int nst[R], nln[R];
        uint32_t nmk[R];
#pragma unroll
        for (int r = 0; r < R; ++r) segment(i0 + (R + r) * G, nst[r], nln[r], nmk[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (col[r][u] >= 0) add(col[r][u], kLoadVal ? val[r][u] : 0.f, mk[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          for (int base = kPass; base < ln[r]; base += kPass) {
            int c2[U];
            float v2[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int e = base + l + kGroup * u;
              c2[u] = e < ln[r] ? a.indices[st[r] + e] : -1;
              if constexpr (BM == kCsrData) v2[u] = e < ln[r] ? a.data[st[r] + e] : 0.f;
              if constexpr (BM == kCsrVec) v2[u] = a.data ? (e < ln[r] ? a.data[st[r] + e] : 0.f) : a.w;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
              if (c2[u] >= 0) add(c2[u], kLoadVal ? v2[u] : 0.f, mk[r]);
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          st[r] = nst[r];
          ln[r] = nln[r];
          mk[r] = nmk[r];
        }
      }
    } else {
      // JIT: one lane per (firing row, block overlapping the tile)
      const int32_t B = a.jit.block;
      const int32_t b_lo = B > 0 ? lo / B : 0;
      const int32_t b_hi = B > 0 ? (hi - 1) / B : 0;
      const int32_t nbt = b_hi - b_lo + 1;
      const int items = total * nbt;
      const uint64_t seed = a.jit.seed;
      const uint32_t K = (uint32_t)a.jit.max_gap;
      const ConnGen G = conn_gen(a.jit);
      const int32_t wkind = a.jit.wkind, n_post = a.n_post;
      const float w0 = a.jit.w0, w1 = a.jit.w1;
      // the four-lane walk emits every target from the block start, so it
      // needs the tile to begin there (a block wider than the LDS tile is cut
      // into several tiles, the later ones starting inside the block)
      // (uniform gaps only: it reads the gap law off the draws directly)
      if (a.jit.rule == kRuleFixedDegree) {
        // exactly k targets per row, each computed on its own from the row's
        // permutation: one wave per listed row, lane l takes targets l,
        // l + 64, ... (every tile evaluates all k and keeps its own)
        const int32_t k = a.jit.degree < n_post ? a.jit.degree : n_post;
        const uint32_t fb = fd_bits(n_post);
        const int wv = (int)threadIdx.x / kWave, ln = lane_id();
        for (int ai = wv; ai < total; ai += kMvThreads / kWave) {
          const uint32_t id = (uint32_t)sh.ids[ai];
          const uint32_t j = kB ? id >> 8 : id, mk = kB ? id & 0xFFu : 0u;
          RowScale<MODE> sc;
          sc.load(a, j, c0, mg);
          const Words4 key = fd_keys(seed, j);
          for (int32_t i = ln; i < k; i += kWave) {
            const int32_t t = (int32_t)fd_target(key, fb, n_post, (uint32_t)i);
            if (t >= lo && t < hi) {
              DrawSeq wd(seed, kStreamW, j, 0u);
              jit_put<MODE>(acc, t - lo, width, mk, sc, wd, wkind, w0, w1, (uint32_t)i, mg);
            }
          }
        }
      } else if (a.jit.rule == kRuleUniform && B > 0 && nbt == 1 && lo == (int64_t)b_lo * B &&
                 items * 4 <= kMvThreads) {
        // Few rows in the pass: four lanes per row.  In pass P lane q draws
        // generator block 4P + q (draws 16P + 4q .. 16P + 4q + 3); a prefix
        // of the lanes' gap sums over the quad places the targets, so a row
        // of up to 14 targets takes one generator call per lane instead of
        // a sequential walk.  Positions and target indices are those of
        // the walk (target m >= 1 at the previous one plus 1 + draw m + 1).
        const int ai = (int)threadIdx.x >> 2, q = (int)threadIdx.x & 3;
        const int qb = lane_id() & ~3;
        const bool act = ai < items;
        const uint32_t b = (uint32_t)b_lo;
        const int64_t end = hi;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        const uint32_t id = act ? (uint32_t)sh.ids[ai] : 0u;
        const uint32_t j = kB ? id >> 8 : id, mk = kB ? id & 0xFFu : 0u;
        RowScale<MODE> sc;
        sc.load(a, j, c0, mg);  // row 0 exists whenever a pass runs
        DrawSeq wd(seed, kStreamW, j, b);
        auto shfl64 = [](int64_t v, int src) {
          const uint32_t lo32 = (uint32_t)__shfl((int)(uint32_t)v, src, kWave);
          const uint32_t hi32 = (uint32_t)__shfl((int)(uint32_t)((uint64_t)v >> 32), src, kWave);
          return (int64_t)(((uint64_t)hi32 << 32) | lo32);
        };
        bool live = act;
        int64_t prev = 0;  // last position of the previous pass
        for (uint32_t pass = 0;; ++pass) {
          const uint32_t blk = 4 * pass + (uint32_t)q;
          const Words4 w = philox10(j, b, blk, kStreamConn, k0, k1);
          int64_t g[4];
          g[0] = 1 + (int64_t)below(w.x, K);
          g[1] = 1 + (int64_t)below(w.y, K);
          g[2] = 1 + (int64_t)below(w.z, K);
          g[3] = 1 + (int64_t)below(w.w, K);
          int64_t first = 0;
          if (blk == 0) {  // draws 0 and 1 give the first target, not gaps
            const uint32_t ra = below(w.x, K), rb = below(w.y, K + 1u);
            first = (int64_t)b * B + (int64_t)(ra < rb ? ra : rb);
            g[0] = 0;
            g[1] = 0;
          }
          const int64_t sum = g[0] + g[1] + g[2] + g[3];
          const int64_t s0 = shfl64(sum, qb), s1 = shfl64(sum, qb + 1), s2 = shfl64(sum, qb + 2);
          const int64_t b0 = pass == 0 ? shfl64(first, qb) : prev;
          const int64_t excl = (q > 0 ? s0 : 0) + (q > 1 ? s1 : 0) + (q > 2 ? s2 : 0);
          int64_t pos = b0 + excl;
          if (live && blk == 0 && pos < end)  // target 0
            jit_put<MODE>(acc, (int)(pos - lo), width, mk, sc, wd, wkind, w0, w1, 0u, mg);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            pos += g[u];
            if (live && g[u] > 0 && pos < end)
              jit_put<MODE>(acc, (int)(pos - lo), width, mk, sc, wd, wkind, w0, w1, 4u * blk - 1u + (uint32_t)u, mg);
          }
          prev = shfl64(pos, qb + 3);  // the pass's last position
          live = live && prev < end;
          if (__ballot(live) == 0) break;
        }
      } else if (a.jit.rule == kRuleUniform && B > 0 && nbt == 1 && lo == (int64_t)b_lo * B) {
        // Balanced walks: a lane runs its (row, block) walk one generator
        // call (four draws) at a time and, when the walk leaves the block,
        // takes the next listed row (a wave claims rows for all its idle
        // lanes with one LDS atomic), so lanes stay busy until the list is
        // used up instead of each waiting for the longest walk of its wave.
        // Targets and their indices are those of the sequential walk.
        if (threadIdx.x == 0) sh.grab = 0;
        __syncthreads();
        const uint32_t b = (uint32_t)b_lo;
        const int64_t start = (int64_t)b * B;
        const int64_t end = hi;  // the tile is the block, clipped at n_post
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        bool act = false, more = true;
        uint32_t j = 0, mk = 0, call = 0, m = 0;
        int64_t pos = 0;
        RowScale<MODE> sc;
        DrawSeq wd(seed, kStreamW, 0u, b);
        while (true) {
          if (more) {
            const uint64_t need = __ballot(!act);
            if (need) {
              const int nn = (int)__popcll(need);
              const int leader = __ffsll((long long)need) - 1;
              int base = 0;
              if (lane_id() == leader) base = atomicAdd(&sh.grab, nn);
              base = __builtin_amdgcn_readlane(base, leader);
              if (!act) {
                const int it = base + mask_rank(need);
                if (it < items) {
                  const uint32_t id = (uint32_t)sh.ids[it];
                  j = kB ? id >> 8 : id;
                  mk = kB ? id & 0xFFu : 0u;
                  sc.load(a, j, c0, mg);
                  wd = DrawSeq(seed, kStreamW, j, b);
                  call = 0;
                  m = 0;
                  act = true;
                }
              }
              if (base + nn >= items) more = false;
            }
          }
          if (__ballot(act) == 0) break;
          if (act) {
            const Words4 w = philox10(j, b, call, kStreamConn, k0, k1);
            const uint32_t d[4] = {w.x, w.y, w.z, w.w};
            const int u0 = call == 0 ? 2 : 0;
            if (call == 0) {  // draws 0 and 1 give the first target, not gaps
              const uint32_t ra = below(d[0], K), rb = below(d[1], K + 1u);
              pos = start + (int64_t)(ra < rb ? ra : rb);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (u >= u0 && pos < end) {
                jit_put<MODE>(acc, (int)(pos - lo), width, mk, sc, wd, wkind, w0, w1, m, mg);
                ++m;
                pos += 1 + (int64_t)below(d[u], K);
              }
            }
            ++call;
            if (pos >= end) act = false;
          }
        }
      } else
      for (int it = threadIdx.x; it < items; it += kMvThreads) {
        const int ai = nbt == 1 ? it : it / nbt;
        const uint32_t b = (uint32_t)(b_lo + (nbt == 1 ? 0 : it % nbt));
        const uint32_t id = (uint32_t)sh.ids[ai];
        const uint32_t j = kB ? id >> 8 : id, mk = kB ? id & 0xFFu : 0u;
        RowScale<MODE> sc;
        sc.load(a, j, c0, mg);
        DrawSeq wd(seed, kStreamW, j, b);
        gen_block(G, j, b, lo, hi, [&](int32_t pos, uint32_t m) {
          jit_put<MODE>(acc, pos - lo, width, mk, sc, wd, wkind, w0, w1, m, mg);
        });
      }
    }
    __syncthreads();  // list consumed before the next sweep overwrites it
    total = 0;
  }
  __syncthreads();
  if constexpr (MODE == kJitMat) {
    // acc[cc * width + i] is Y[lo + i][c0 + cc]; Y (or the chunk's partial) is [n_post][m]
    float* dst = reinterpret_cast<float*>(a.out) + (size_t)c * a.n_post * a.m;
    for (int i2 = threadIdx.x; i2 < width * mg; i2 += kMvThreads) {
      const int i = i2 / mg, cc = i2 - i * mg;
      dst[(size_t)(lo + i) * a.m + c0 + cc] = acc[cc * width + i];
    }
    return;
  }
  if constexpr (kB) {
    // vector c0 + b of the group: Y[c0 + b][lo + i] (one chunk), or the
    // partial [c][c0 + b][lo + i] of [chunks][batch][n_post]
    for (int i2 = threadIdx.x; i2 < width * mg; i2 += kMvThreads) {
      const int b = i2 / width, i = i2 - b * width;
      uint32_t cnt = 0;
      float sum = 0.f;
      if constexpr (counts_mode(MODE)) cnt = (acc[(b >> 1) * width + i] >> (16 * (b & 1))) & 0xFFFFu;
      else sum = acc[b * width + i];
      if (a.chunks == 1) {
        reinterpret_cast<float*>(a.out)[(size_t)(c0 + b) * a.y_stride + lo + i] =
            counts_mode(MODE) ? (float)cnt * a.w : sum;
      } else {
        const size_t at = ((size_t)c * a.batch + c0 + b) * a.n_post + lo + i;
        if constexpr (counts_mode(MODE)) reinterpret_cast<uint16_t*>(a.out)[at] = (uint16_t)cnt;
        else reinterpret_cast<float*>(a.out)[at] = sum;
      }
    }
    return;
  }
  if (a.chunks == 1) {
    float* y = reinterpret_cast<float*>(a.out);
    for (int i = threadIdx.x; i < width; i += kMvThreads) {
      if constexpr (MODE == kCsrHomo || MODE == kJitHomo) y[lo + i] = (float)acc[i] * a.w;
      else y[lo + i] = acc[i];
    }
  } else if constexpr (MODE == kCsrHomo || MODE == kJitHomo) {
    uint16_t* part = reinterpret_cast<uint16_t*>(a.out) + (size_t)c * a.n_post;
    uint16_t* dst = part + lo;
    if ((reinterpret_cast<uintptr_t>(dst) & 7) == 0) {  // four counts per 8-byte store
      const int w4 = width / 4;
      for (int i = threadIdx.x; i < w4; i += kMvThreads) {
        const uint4 v = reinterpret_cast<const uint4*>(acc)[i];
        reinterpret_cast<uint2*>(dst)[i] = make_uint2(v.x | (v.y << 16), v.z | (v.w << 16));
      }
      for (int i = 4 * w4 + threadIdx.x; i < width; i += kMvThreads) dst[i] = (uint16_t)acc[i];
    } else {
      for (int i = threadIdx.x; i < width; i += kMvThreads) dst[i] = (uint16_t)acc[i];
    }
  } else {
    float* part = reinterpret_cast<float*>(a.out) + (size_t)c * a.n_post;
    for (int i = threadIdx.x; i < width; i += kMvThreads) part[lo + i] = acc[i];
  }
}

// First of the two columns of this thread in the reductions: workgroup b
// takes 512 columns of tile b mod n_tiles, the same tile-to-workgroup order
// as the scatter, so with a multiple of 8 tiles the partials of a tile are
// read on the XCD that wrote them (workgroups are dealt to the 8 XCDs in
// turn).  With an odd tile width the second column may be the next tile's
// first, which that tile's thread also writes, with the same value.
__device__ __forceinline__ int32_t reduce_col(int32_t tile, int32_t n_tiles) {
  const int32_t t = (int32_t)blockIdx.x % n_tiles, sl = (int32_t)blockIdx.x / n_tiles;
  const int32_t k = sl * 512 + (int32_t)threadIdx.x * 2;
  return k < tile ? t * tile + k : INT32_MAX;
}

// y[k] = w * sum_c counts[c][k]  (integer sum, one FP32 rounding); two
// consecutive columns per thread, eight chunk loads in flight.
__global__ void mv_reduce_counts_k(const uint16_t* __restrict__ part, int32_t chunks, int32_t n_post, float w,
                                   float* __restrict__ y, int32_t tile, int32_t n_tiles) {
  const int32_t k = reduce_col(tile, n_tiles);
  if (k >= n_post) return;
  const bool vec = ((reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(y)) & 7) == 0;
  if (vec && (tile & 1) == 0 && k + 2 <= n_post && (n_post & 1) == 0) {
    uint32_t s0 = 0, s1 = 0;
#pragma unroll 8
    for (int c = 0; c < chunks; ++c) {
      const uint32_t v = *reinterpret_cast<const uint32_t*>(part + (size_t)c * n_post + k);
      s0 += v & 0xFFFFu;
      s1 += v >> 16;
    }
    *reinterpret_cast<float2*>(y + k) = make_float2((float)s0 * w, (float)s1 * w);
  } else {
    for (int q = 0; q < 2 && k + q < n_post; ++q) {
      uint32_t s = 0;
#pragma unroll 8
      for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n_post + k + q];
      y[k + q] = (float)s * w;
    }
  }
}
// y[k] = sum_c part[c][k] in chunk order; two consecutive columns per thread,
// eight chunk loads in flight.
__global__ void mv_reduce_f32_k(const float* __restrict__ part, int32_t chunks, int32_t n_post, float* __restrict__ y,
                                int32_t tile, int32_t n_tiles) {
  const int32_t k = reduce_col(tile, n_tiles);
  if (k >= n_post) return;
  const bool vec = ((reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(y)) & 7) == 0;
  if (vec && (tile & 1) == 0 && k + 2 <= n_post && (n_post & 1) == 0) {
    float s0 = 0.f, s1 = 0.f;
#pragma unroll 8
    for (int c = 0; c < chunks; ++c) {
      const float2 v = *reinterpret_cast<const float2*>(part + (size_t)c * n_post + k);
      s0 += v.x;
      s1 += v.y;
    }
    *reinterpret_cast<float2*>(y + k) = make_float2(s0, s1);
  } else {
    for (int q = 0; q < 2 && k + q < n_post; ++q) {
      float s = 0.f;
#pragma unroll 8
      for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n_post + k + q];
      y[k + q] = s;
    }
  }
}

// The same sums with 16-byte loads, for 8-column-aligned partial rows
// (n_post a multiple of 8, 16-byte-aligned part and y).  A lane holds 8
// consecutive columns and every fourth chunk: lanes l, l + 16, l + 32, l + 48
// of a wave take chunks q, q + 4, ... (q = l / 16) of the same 8 columns, so
// one load instruction fetches four 256-byte runs and a lane has all its
// chunk loads in flight at once (8 for 32 chunks).  The four lanes' sums are
// combined by two lane exchanges, ((q0 + q1) + (q2 + q3)): a fixed order,
// so repeated calls give the same bits.  Workgroup b takes 512 columns of
// the 8-aligned range that starts at or before tile b mod n_tiles (the
// scatter's tile-to-workgroup order, so partials are read on the XCD that
// wrote them).
constexpr int kRedThreads = 256;
constexpr int kRedCols = kRedThreads / 4 * 8;  // columns per workgroup
constexpr int kRedLoads = 8;                   // chunk loads in flight per lane
// used from 16 chunks up: with fewer (two or fewer loads per lane) the
// two-column kernels above measured faster
constexpr int kRedMinChunks = 16;

__host__ __device__ inline int32_t reduce_slices(int32_t tile) { return (tile + 7 + kRedCols - 1) / kRedCols; }

template <bool COUNTS>
__global__ void __launch_bounds__(kRedThreads) mv_reduce_wide_k(const void* __restrict__ part, int32_t chunks,
                                                                  int32_t n_post, float w, float* __restrict__ y,
                                                                  int32_t tile, int32_t n_tiles) {
  const int32_t t = (int32_t)blockIdx.x % n_tiles, sl = (int32_t)blockIdx.x / n_tiles;
  const int32_t start = (int32_t)(((int64_t)t * tile) & ~7ll);
  const int32_t end = t == n_tiles - 1 ? n_post : (int32_t)(((int64_t)(t + 1) * tile) & ~7ll);
  const int l = lane_id(), q = l >> 4;
  const int32_t col = start + sl * kRedCols + ((int32_t)threadIdx.x / kWave * 16 + (l & 15)) * 8;
  const bool act = col < end;  // every lane takes part in the exchanges
  if constexpr (COUNTS) {
    uint32_t s[8] = {};
    if (act) {
      const uint16_t* p = reinterpret_cast<const uint16_t*>(part) + col;
      for (int c0 = q; c0 < chunks; c0 += 4 * kRedLoads) {
        // kRedLoads loads issued back to back (chunks past the end re-read
        // the last one and are dropped), then summed
        uint4 v[kRedLoads];
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i)
          v[i] = *reinterpret_cast<const uint4*>(p + (size_t)min(c0 + 4 * i, chunks - 1) * n_post);
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i) {
          if (c0 + 4 * i >= chunks) v[i] = make_uint4(0u, 0u, 0u, 0u);
          s[0] += v[i].x & 0xFFFFu; s[1] += v[i].x >> 16; s[2] += v[i].y & 0xFFFFu; s[3] += v[i].y >> 16;
          s[4] += v[i].z & 0xFFFFu; s[5] += v[i].z >> 16; s[6] += v[i].w & 0xFFFFu; s[7] += v[i].w >> 16;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s[i] += (uint32_t)__shfl_xor((int)s[i], 16, kWave);
      s[i] += (uint32_t)__shfl_xor((int)s[i], 32, kWave);
    }
    if (act && q == 0) {
      float4* o = reinterpret_cast<float4*>(y + col);
      o[0] = make_float4((float)s[0] * w, (float)s[1] * w, (float)s[2] * w, (float)s[3] * w);
      o[1] = make_float4((float)s[4] * w, (float)s[5] * w, (float)s[6] * w, (float)s[7] * w);
    }
  } else {
    float s[8] = {};
    if (act) {
      const float* p = reinterpret_cast<const float*>(part) + col;
      for (int c0 = q; c0 < chunks; c0 += 4 * kRedLoads) {
        float4 a[kRedLoads], b[kRedLoads];
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i) {
          const float* r = p + (size_t)min(c0 + 4 * i, chunks - 1) * n_post;
          a[i] = *reinterpret_cast<const float4*>(r);
          b[i] = *reinterpret_cast<const float4*>(r + 4);
        }
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i) {
          if (c0 + 4 * i >= chunks) a[i] = b[i] = make_float4(0.f, 0.f, 0.f, 0.f);
          s[0] += a[i].x; s[1] += a[i].y; s[2] += a[i].z; s[3] += a[i].w;
          s[4] += b[i].x; s[5] += b[i].y; s[6] += b[i].z; s[7] += b[i].w;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s[i] += __shfl_xor(s[i], 16, kWave);
      s[i] += __shfl_xor(s[i], 32, kWave);
    }
    if (act && q == 0) {
      float4* o = reinterpret_cast<float4*>(y + col);
      o[0] = make_float4(s[0], s[1], s[2], s[3]);
      o[1] = make_float4(s[4], s[5], s[6], s[7]);
    }
  }
}

// Batched products: Y[b][k] = (w *) sum_c part[c][b][k] in chunk order, part
// [chunks][batch][n_post] (16-bit counts or FP32 sums); blockIdx.y = b, two
// consecutive columns per thread.
template <bool COUNTS>
__global__ void mv_reduce_batch_k(const void* __restrict__ part, int32_t chunks, int32_t batch, int32_t n_post,
                                  float w, float* __restrict__ y, int64_t y_stride) {
  const int32_t b = blockIdx.y;
  const int32_t k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 2;
  const size_t cs = (size_t)batch * n_post;
  for (int q = 0; q < 2; ++q) {
    const int32_t k = k0 + q;
    if (k >= n_post) break;
    const size_t at = (size_t)b * n_post + k;
    if constexpr (COUNTS) {
      uint32_t sum = 0;
#pragma unroll 8
      for (int c = 0; c < chunks; ++c) sum += reinterpret_cast<const uint16_t*>(part)[c * cs + at];
      y[(size_t)b * y_stride + k] = (float)sum * w;
    } else {
      float sum = 0.f;
#pragma unroll 8
      for (int c = 0; c < chunks; ++c) sum += reinterpret_cast<const float*>(part)[c * cs + at];
      y[(size_t)b * y_stride + k] = sum;
    }
  }
}

// Unsorted CSR wider than one tile: counts / sums with device atomics.
__global__ void mv_zero_k(uint32_t* p, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
template <bool HOMO>
__global__ void mv_atomic_k(MvArgs a, uint32_t* acc) {
  const int wv = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nw = gridDim.x * blockDim.x / kWave;
  for (int32_t j = wv; j < a.n_pre; j += nw) {
    if (!a.events[j]) continue;
    for (int32_t idx = a.indptr[j] + lane_id(); idx < a.indptr[j + 1]; idx += kWave) {
      if (HOMO) atomicAdd(&acc[a.indices[idx]], 1u);
      else atomicAdd(reinterpret_cast<float*>(acc) + a.indices[idx], a.data[idx]);
    }
  }
}
__global__ void mv_counts_to_y_k(const uint32_t* acc, int32_t n, float w, float* y) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)acc[i] * w;
}

// ---------------------------------------------------------------- reverse mode
__global__ void zero_f32_k(float* p, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// One wave per row.
__global__ void csr_backward_k(bp_csr m, const uint8_t* __restrict__ ev, const float* __restrict__ dy,
                               float* __restrict__ d_ev, float* __restrict__ d_data, float* __restrict__ d_w) {
  const int wv = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nw = gridDim.x * blockDim.x / kWave;
  float gw = 0.f;
  for (int32_t j = wv; j < m.n_pre; j += nw) {
    const bool on = ev[j] != 0;
    float acc = 0.f, accw = 0.f;
    for (int32_t idx = m.indptr[j] + lane_id(); idx < m.indptr[j + 1]; idx += kWave) {
      const float g = dy[m.indices[idx]];
      acc += (m.data ? m.data[idx] : m.w) * g;
      accw += g;
      if (d_data) d_data[idx] = on ? g : 0.f;
    }
    acc = wave_sum_f(acc);
    if (d_ev && lane_id() == 0) d_ev[j] = acc;
    if (on) gw += accw;
  }
  if (d_w) {
    gw = wave_sum_f(gw);
    if (lane_id() == 0 && gw != 0.f) atomicAdd(d_w, gw);
  }
}

// LPR lanes per row (a power of two up to 64, groups aligned in the wave):
// lane q of the group walks the row's blocks q, q + LPR, ... (for exactly
// fixed out-degree, the targets q, q + LPR, ... of the row's permutation);
// the group's partial sums are then combined by shuffles in a fixed order,
// so d_events does not depend on scheduling.
template <int LPR>
__global__ void jit_backward_k(bp_jit_conn c, const uint8_t* __restrict__ ev, const float* __restrict__ dy,
                               float* __restrict__ d_ev, float* __restrict__ d_w) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t j = (int32_t)(gt / LPR);
  const int q = (int)(gt % LPR);
  float acc = 0.f, g0 = 0.f, g1 = 0.f;
  if (j < c.n_pre) {
    const bool on = ev[j] != 0;
    const uint64_t seed = c.seed;
    const int32_t n_post = c.n_post, wkind = c.wkind;
    const float w0 = c.w0, w1 = c.w1;
    auto term_g = [&](DrawSeq& wd, float g, uint32_t m) {
      float unit;
      const float wjk = jit_weight(wd, wkind, w0, w1, m, &unit);
      acc += wjk * g;
      if (on) {
        // d w / d w0 and d w / d w1: (1, z) normal, (1 - u, u) uniform, (1, 0) homogeneous
        g0 += (wkind == kWUniform ? 1.f - unit : 1.f) * g;
        g1 += (wkind == kWHomo ? 0.f : unit) * g;
      }
    };
    auto term = [&](DrawSeq& wd, int32_t pos, uint32_t m) { term_g(wd, dy[pos], m); };
    if (c.rule == kRuleUniform || c.rule == kRuleGeometric) {
      // gap walks: one generator call (four draws) at a time, the dy loads
      // of its up to four targets issued together before any is used (one
      // load at a time left each lane waiting a cache round trip per
      // target); targets, their order and indices are the walk's
      const bool geo = c.rule == kRuleGeometric;
      const float inv_rate = c.geo_inv_rate;
      const uint32_t K = (uint32_t)c.max_gap;
      const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
      const int32_t nb = c.block > 0 ? (int32_t)(((int64_t)n_post + c.block - 1) / c.block) : 1;
      for (int32_t b = q; b < nb; b += LPR) {
        DrawSeq wd(seed, kStreamW, (uint32_t)j, (uint32_t)b);
        const int64_t start = c.block > 0 ? (int64_t)b * c.block : 0;
        const int64_t end = c.block > 0 && start + c.block < n_post ? start + c.block : n_post;
        int64_t pos = 0;
        uint32_t m = 0;
        for (uint32_t call = 0;; ++call) {
          const Words4 w = philox10((uint32_t)j, (uint32_t)b, call, kStreamConn, k0, k1);
          const uint32_t d[4] = {w.x, w.y, w.z, w.w};
          int u0 = 0;
          if (call == 0) {  // the first target: draw 0 (geometric), draws 0 and 1 in a block, draw 0 in a whole row
            if (geo) {
              pos = start + (int64_t)geo_gap(d[0], inv_rate) - 1;
              u0 = 1;
            } else if (c.block > 0) {
              const uint32_t ra = below(d[0], K), rb = below(d[1], K + 1u);
              pos = start + (int64_t)(ra < rb ? ra : rb);
              u0 = 2;
            } else {
              pos = (int64_t)below(d[0], K);
              u0 = 1;
            }
          }
          int32_t tp[4];
          bool tv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            tv[u] = u >= u0 && pos < end;
            tp[u] = tv[u] ? (int32_t)pos : 0;
            if (tv[u]) pos += geo ? (int64_t)geo_gap(d[u], inv_rate) : 1 + (int64_t)below(d[u], K);
          }
          float gy[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) gy[u] = tv[u] ? dy[tp[u]] : 0.f;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (tv[u]) term_g(wd, gy[u], m++);
          if (pos >= end) break;
        }
      }
    } else if (c.rule == kRuleFixedDegree) {
      const Words4 key = fd_keys(seed, (uint32_t)j);
      const uint32_t fb = fd_bits(n_post);
      const int32_t k = c.degree < n_post ? c.degree : n_post;
      for (int32_t i = q; i < k; i += LPR) {
        DrawSeq wd(seed, kStreamW, (uint32_t)j, 0u);
        term(wd, (int32_t)fd_target(key, fb, n_post, (uint32_t)i), (uint32_t)i);
      }
    } else {
      const ConnGen G = conn_gen(c);
      const int32_t nb = c.block > 0 ? (int32_t)(((int64_t)n_post + c.block - 1) / c.block) : 1;
      for (int32_t b = q; b < nb; b += LPR) {
        DrawSeq wd(seed, kStreamW, (uint32_t)j, (uint32_t)b);
        gen_block(G, (uint32_t)j, (uint32_t)b, 0, n_post,
                  [&](int32_t pos, uint32_t m) { term(wd, pos, m); });
      }
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (j < c.n_pre && q == 0 && d_ev) d_ev[j] = acc;
  if (d_w) {
    g0 = wave_sum_f(g0);
    g1 = wave_sum_f(g1);
    if (lane_id() == 0) {
      if (g0 != 0.f) atomicAdd(&d_w[0], g0);
      if (g1 != 0.f) atomicAdd(&d_w[1], g1);
    }
  }
}

// ---------------------------------------------------------------- planning
struct MvPlan {
  int32_t tile, n_tiles, chunks, chunk_rows;
  bool atomic_path;
  bool unsupported;
  size_t ws;
};

// Row chunks per column tile.  The scatter kernel holds one workgroup per
// compute unit (LDS), so the grid aims at one wave of workgroups: as many
// chunks as keep tiles x chunks within the compute units, each at least a
// quarter sweep of rows.  Chunk starts are multiples of 16 (aligned spike
// loads); 16-bit partial counts cap homogeneous chunks at 65520 rows.
static void set_chunks(MvPlan& p, int32_t n_pre, bool homo, int32_t n_post, bool packed = false,
                       bool small_chunks = false) {
  const int32_t cus = device_cu_count();
  const int32_t cap = max(1, cus / p.n_tiles);
  int32_t want = max(1, min(cap, (n_pre + kSweep / 4 - 1) / (kSweep / 4)));
  // products on dense float vectors (every row listed) over few rows (a few
  // thousand): chunks of kMinChunkRows, so that more than a handful of
  // workgroups share the rows (one workgroup streaming 4000 listed rows
  // takes 30 batches of dependent loads one after another), while the
  // partials stay within kSmallPartialBytes; spike products over few rows
  // list few rows and keep one chunk (no second launch)
  if (want < 4 && small_chunks) {
    const int64_t by_bytes = kSmallPartialBytes / ((int64_t)max(n_post, 1) * 4);
    int64_t w2 = (n_pre + kMinChunkRows - 1) / kMinChunkRows;
    if (w2 > cap) w2 = cap;
    if (w2 > by_bytes) w2 = by_bytes;
    if (w2 > want) want = (int32_t)w2;
  }
  // 16-bit partial counts (and the batched products' packed 16-bit LDS
  // counts, even with one chunk) hold at most 65520 rows' worth per column
  if (homo && (want > 1 || packed)) want = max(want, (n_pre + 65519) / 65520);
  int32_t rows = (n_pre + want - 1) / want;
  rows = (rows + 15) & ~15;
  p.chunk_rows = max(16, rows);
  p.chunks = max(1, (n_pre + p.chunk_rows - 1) / p.chunk_rows);
  p.ws = p.chunks > 1 ? (size_t)p.chunks * n_post * (homo ? 2 : 4) : 0;
}

static MvPlan plan_csr(const bp_csr* m, bool vec_input = false) {
  MvPlan p{};
  if (m->n_post <= kTileMax) {
    p.tile = m->n_post > 0 ? m->n_post : 1;
    p.n_tiles = 1;
  } else if (m->sorted && m->tile_ptr && m->tile_width > 0 && m->tile_width <= kTileMax) {
    p.tile = m->tile_width;
    p.n_tiles = (int32_t)(((int64_t)m->n_post + p.tile - 1) / p.tile);
  } else if (m->sorted) {
    // no tile index: equal tiles of at most kTileMax columns, each row's
    // segment found by a search inside the kernel
    const int32_t nt = (int32_t)(((int64_t)m->n_post + kTileMax - 1) / kTileMax);
    p.tile = (int32_t)(((int64_t)m->n_post + nt - 1) / nt);
    p.n_tiles = (int32_t)(((int64_t)m->n_post + p.tile - 1) / p.tile);
  } else {
    if (vec_input) {  // float-vector products of unsorted rows: one tile only
      p.unsupported = true;
      return p;
    }
    p.atomic_path = true;
    p.ws = (size_t)(m->n_post > 0 ? m->n_post : 1) * sizeof(uint32_t);
    return p;
  }
  set_chunks(p, m->n_pre, !vec_input && m->data == nullptr, m->n_post, false, vec_input);
  // 16-bit partial counts need at most one entry per row and column
  if (!vec_input && !m->data && !m->sorted && p.chunks > 1) {
    p.atomic_path = true;
    p.ws = (size_t)(m->n_post > 0 ? m->n_post : 1) * sizeof(uint32_t);
  }
  return p;
}

// counts: homogeneous weights summed as integer counts (event input only).
// vec: the product on dense float vectors (every row listed).
static MvPlan plan_jit(const bp_jit_conn* c, bool counts, bool vec = false) {
  MvPlan p{};
  if (c->block > 0 && c->block <= kTileMax && c->n_post > c->block) {
    p.tile = c->block;  // one block per tile: every generated target lands in the tile
  } else if (c->n_post <= kTileMax) {
    p.tile = c->n_post > 0 ? c->n_post : 1;
  } else {
    p.tile = kTileMax;  // whole-row sequences regenerated up to each tile
  }
  p.n_tiles = (int32_t)(((int64_t)c->n_post + p.tile - 1) / p.tile);
  if (p.n_tiles < 1) p.n_tiles = 1;
  set_chunks(p, c->n_pre, counts, c->n_post, false, vec);
  return p;
}

// Batched product: the single-vector plan, kMatCols columns of X per
// workgroup while the LDS tile holds them (tile * mg <= kTileMax), column
// groups on blockIdx.y, row chunks sized for tiles x groups workgroups.
static MvPlan plan_jit_mat(const bp_jit_conn* c, int32_t m, int32_t* mg, int32_t* groups) {
  MvPlan p = plan_jit(c, false, true);
  *mg = max(1, min(min(kMatCols, kTileMax / p.tile), m));
  *groups = (m + *mg - 1) / *mg;
  const int32_t nt = p.n_tiles;
  p.n_tiles = nt * *groups;
  set_chunks(p, c->n_pre, false, c->n_post, false, true);
  p.n_tiles = nt;
  p.ws = p.chunks > 1 ? (size_t)p.chunks * c->n_post * m * sizeof(float) : 0;
  return p;
}

// Batched spike products: up to kMatCols vectors per workgroup (group on
// blockIdx.y) while the LDS tile holds them: counts take one 32-bit word per
// column and pair of vectors, sums one float per column and vector.  Tiles
// are the single-vector ones when they leave room for at least two vectors,
// else narrower (CSR: equal tiles found by the in-kernel row search, or the
// caller's tile index when its width fits; JIT: the tile is still one block
// when the block fits, else equal tiles).  Partials are [chunks][batch][n_post].
static int32_t batch_group(int32_t tile, bool counts, int32_t batch) {
  const int32_t words = kTileMax / max(tile, 1);  // LDS words per column
  const int32_t per = counts ? 2 * words : words;
  return max(1, min(min(kMatCols, per), batch));
}

static MvPlan plan_csr_batch(const bp_csr* m, int32_t batch, int32_t* mb, int32_t* groups) {
  MvPlan p{};
  const bool counts = m->data == nullptr;
  const int32_t cap = counts ? kTileMax / (kMatCols / 2) : kTileMax / kMatCols;  // room for 8 vectors
  if (m->n_post <= cap) {
    p.tile = m->n_post > 0 ? m->n_post : 1;
    p.n_tiles = 1;
  } else if (m->tile_ptr && m->tile_width > 0 && m->tile_width <= kTileMax / (counts ? 1 : 2)) {
    p.tile = m->tile_width;  // the caller's index, at least two vectors per group
    p.n_tiles = (int32_t)(((int64_t)m->n_post + p.tile - 1) / p.tile);
  } else {
    const int32_t nt = (int32_t)(((int64_t)m->n_post + cap - 1) / cap);
    p.tile = (int32_t)(((int64_t)m->n_post + nt - 1) / nt);
    p.n_tiles = (int32_t)(((int64_t)m->n_post + p.tile - 1) / p.tile);
  }
  *mb = batch_group(p.tile, counts, batch);
  *groups = (batch + *mb - 1) / *mb;
  const int32_t nt = p.n_tiles;
  p.n_tiles = nt * *groups;
  set_chunks(p, m->n_pre, counts, m->n_post, counts);
  p.n_tiles = nt;
  p.ws = p.chunks > 1 ? (size_t)p.chunks * batch * m->n_post * (counts ? 2 : 4) : 0;
  return p;
}

static MvPlan plan_jit_batch(const bp_jit_conn* c, int32_t batch, int32_t* mb, int32_t* groups) {
  const bool counts = c->wkind == kWHomo;
  MvPlan p{};
  const int32_t cap = counts ? kTileMax / (kMatCols / 2) : kTileMax / kMatCols;
  if (c->block > 0 && c->block <= kTileMax / (counts ? 1 : 2) && c->n_post > c->block) {
    p.tile = c->block;  // one block per tile, at least two vectors per group
  } else if (c->n_post <= cap) {
    p.tile = c->n_post > 0 ? c->n_post : 1;
  } else {
    const int32_t nt = (int32_t)(((int64_t)c->n_post + cap - 1) / cap);
    p.tile = (int32_t)(((int64_t)c->n_post + nt - 1) / nt);
  }
  p.n_tiles = (int32_t)(((int64_t)c->n_post + p.tile - 1) / p.tile);
  if (p.n_tiles < 1) p.n_tiles = 1;
  *mb = batch_group(p.tile, counts, batch);
  *groups = (batch + *mb - 1) / *mb;
  const int32_t nt = p.n_tiles;
  p.n_tiles = nt * *groups;
  set_chunks(p, c->n_pre, counts, c->n_post, counts);
  p.n_tiles = nt;
  p.ws = p.chunks > 1 ? (size_t)p.chunks * batch * c->n_post * (counts ? 2 : 4) : 0;
  return p;
}

static bp_status finish_batch(const MvPlan& p, bool counts, const void* ws, int32_t batch, int32_t n_post, float w,
                              float* y, int64_t y_stride, hipStream_t st) {
  if (p.chunks <= 1 || n_post == 0) return BP_OK;
  const dim3 g((unsigned)((n_post + 511) / 512), (unsigned)batch);
  if (counts) mv_reduce_batch_k<true><<<g, 256, 0, st>>>(ws, p.chunks, batch, n_post, w, y, y_stride);
  else mv_reduce_batch_k<false><<<g, 256, 0, st>>>(ws, p.chunks, batch, n_post, w, y, y_stride);
  BP_LAUNCHED("mv_reduce_batch_k");
  return BP_OK;
}

static bp_status check_csr(const bp_csr* m) {
  BP_REQUIRE(m != nullptr, "null CSR descriptor");
  BP_REQUIRE(m->n_pre >= 0 && m->n_post >= 0, "negative size");
  BP_REQUIRE(m->indptr != nullptr, "null indptr");
  return BP_OK;
}

template <int MODE>
static bp_status launch_scatter(const MvArgs& a, const MvPlan& p, hipStream_t st) {
  mv_scatter_k<MODE><<<p.n_tiles * p.chunks, kMvThreads, 0, st>>>(a);
  BP_LAUNCHED("mv_scatter_k");
  return BP_OK;
}

static bp_status finish_partials(const MvPlan& p, bool homo, void* ws, int32_t n_post, float w, float* y,
                                 hipStream_t st) {
  if (p.chunks <= 1 || n_post == 0) return BP_OK;
  if (p.chunks >= kRedMinChunks && (n_post & 7) == 0 &&
      ((reinterpret_cast<uintptr_t>(ws) | reinterpret_cast<uintptr_t>(y)) & 15) == 0) {
    const int g = p.n_tiles * reduce_slices(p.tile);
    if (homo) mv_reduce_wide_k<true><<<g, kRedThreads, 0, st>>>(ws, p.chunks, n_post, w, y, p.tile, p.n_tiles);
    else mv_reduce_wide_k<false><<<g, kRedThreads, 0, st>>>(ws, p.chunks, n_post, w, y, p.tile, p.n_tiles);
    BP_LAUNCHED("mv_reduce_wide_k");
    return BP_OK;
  }
  const int g = p.n_tiles * ((p.tile + 511) / 512);
  if (homo) mv_reduce_counts_k<<<g, 256, 0, st>>>((const uint16_t*)ws, p.chunks, n_post, w, y, p.tile, p.n_tiles);
  else mv_reduce_f32_k<<<g, 256, 0, st>>>((const float*)ws, p.chunks, n_post, y, p.tile, p.n_tiles);
  BP_LAUNCHED("mv_reduce_k");
  return BP_OK;
}

// ---------------------------------------------------------------- static scratch
// The scratch of the allocation-free entry point: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends).
// In host code its name is only a host-side stand-in; the device address of
// each GPU's copy comes from hipGetSymbolAddress with that GPU current, is
// kept per device, and is the only way host code refers to the array.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
static_assert(kStaticScratchBytes == BP_STATIC_SCRATCH_BYTES, "static scratch size");
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the static scratch on the GPU that runs `st`, looked up
// once per device (with that device current) and cached.
static bp_status static_scratch(hipStream_t st, void** out) {
  int dev = 0;
  if (st) {
    BP_HIP(hipStreamGetDevice(st, &dev));
  } else {
    BP_HIP(hipGetDevice(&dev));
  }
  if (dev < 0 || dev >= kMaxDevices) return set_error(BP_EUNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    BP_HIP(hipGetDevice(&cur));
    if (cur != dev) BP_HIP(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) BP_HIP(hipSetDevice(cur));
    if (e != hipSuccess || ptr == nullptr)
      return set_error(BP_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BP_OK;
}

static bp_status event_csr_run(const bp_csr* m, const MvPlan& p, const uint8_t* events, float* y, void* ws,
                               hipStream_t st);

}  // namespace bp

using namespace bp;

extern "C" {

size_t bp_event_csr_ws_bytes(const bp_csr* m) {
  if (!m) return 0;
  return plan_csr(m).ws;
}

bp_status bp_csr_tile_index(const int32_t* indptr, const int32_t* indices, int32_t n_pre, int32_t n_post,
                            int32_t tile_width, int32_t* tile_ptr, bp_stream stream) {
  BP_REQUIRE(indptr && tile_ptr, "null pointer");
  BP_REQUIRE(n_pre >= 0 && n_post >= 0, "negative size");
  BP_REQUIRE(tile_width > 0 && tile_width <= kTileMax, "tile_width must be in [1, %d]", kTileMax);
  if (n_pre == 0) return BP_OK;
  const int32_t n_tiles = (int32_t)(((int64_t)n_post + tile_width - 1) / tile_width);
  return launch_tile_index(indptr, indices, n_pre, tile_width, n_tiles > 0 ? n_tiles : 1, tile_ptr,
                           as_stream(stream));
}

bp_status bp_event_csr_matvec(const bp_csr* m, const uint8_t* events, float* y, void* ws, size_t ws_bytes,
                              bp_stream stream) {
  bp_status s = check_csr(m);
  if (s) return s;
  if (m->n_post == 0) return BP_OK;
  BP_REQUIRE(y != nullptr, "null y");
  BP_REQUIRE(m->n_pre == 0 || events != nullptr, "null events");
  const MvPlan p = plan_csr(m);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  return event_csr_run(m, p, events, y, ws, as_stream(stream));
}

bp_status bp_event_csr_matvec_noalloc(const bp_csr* m, const uint8_t* events, float* y, bp_stream stream) {
  bp_status s = check_csr(m);
  if (s) return s;
  if (m->n_post == 0) return BP_OK;
  BP_REQUIRE(y != nullptr, "null y");
  BP_REQUIRE(m->n_pre == 0 || events != nullptr, "null events");
  const MvPlan p = plan_csr(m);
  BP_REQUIRE(p.ws <= kStaticScratchBytes, "scratch of %zu bytes needed, the static array holds %zu", p.ws,
             kStaticScratchBytes);
  hipStream_t st = as_stream(stream);
  void* ws = nullptr;
  if (p.ws > 0) {
    s = static_scratch(st, &ws);
    if (s) return s;
  }
  return event_csr_run(m, p, events, y, ws, st);
}

}  // extern "C"

namespace bp {

static bp_status event_csr_run(const bp_csr* m, const MvPlan& p, const uint8_t* events, float* y, void* ws,
                               hipStream_t st) {
  bp_status s = BP_OK;
  const bool homo = m->data == nullptr;
  if (p.atomic_path) {
    uint32_t* acc = (uint32_t*)ws;
    const int g = (m->n_post + 255) / 256;
    mv_zero_k<<<g, 256, 0, st>>>(acc, m->n_post);
    BP_LAUNCHED("mv_zero_k");
    MvArgs a{};
    a.indptr = m->indptr; a.indices = m->indices; a.data = m->data; a.events = events; a.n_pre = m->n_pre;
    a.n_post = m->n_post;
    if (m->n_pre > 0) {
      if (homo) mv_atomic_k<true><<<1024, 256, 0, st>>>(a, acc);
      else mv_atomic_k<false><<<1024, 256, 0, st>>>(a, acc);
      BP_LAUNCHED("mv_atomic_k");
    }
    if (homo) {
      mv_counts_to_y_k<<<g, 256, 0, st>>>(acc, m->n_post, m->w, y);
      BP_LAUNCHED("mv_counts_to_y_k");
    } else {
      BP_HIP(hipMemcpyAsync(y, acc, (size_t)m->n_post * 4, hipMemcpyDeviceToDevice, st));
    }
    return BP_OK;
  }
  MvArgs a{};
  a.indptr = m->indptr; a.indices = m->indices; a.data = m->data;
  a.tile_ptr = p.n_tiles > 1 && m->tile_ptr && p.tile == m->tile_width ? m->tile_ptr : nullptr;
  a.search = p.n_tiles > 1 && a.tile_ptr == nullptr;
  a.events = events; a.out = p.chunks > 1 ? ws : (void*)y; a.w = m->w;
  a.n_pre = m->n_pre; a.n_post = m->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  s = homo ? launch_scatter<kCsrHomo>(a, p, st) : launch_scatter<kCsrData>(a, p, st);
  if (s) return s;
  return finish_partials(p, homo, ws, m->n_post, m->w, y, st);
}

}  // namespace bp

extern "C" {

size_t bp_csr_matvec_dense_ws_bytes(const bp_csr* m) {
  if (!m) return 0;
  return plan_csr(m, true).ws;
}

bp_status bp_csr_matvec_dense(const bp_csr* m, const float* v, float* y, void* ws, size_t ws_bytes,
                              bp_stream stream) {
  bp_status s = check_csr(m);
  if (s) return s;
  if (m->n_post == 0) return BP_OK;
  BP_REQUIRE(y != nullptr, "null y");
  BP_REQUIRE(m->n_pre == 0 || v != nullptr, "null v");
  const MvPlan p = plan_csr(m, true);
  if (p.unsupported)
    return set_error(BP_EUNSUPPORTED, "float-vector products of unsorted rows need n_post <= %d", kTileMax);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  hipStream_t st = as_stream(stream);
  MvArgs a{};
  a.indptr = m->indptr; a.indices = m->indices; a.data = m->data; a.vec = v;
  a.tile_ptr = p.n_tiles > 1 && m->tile_ptr && p.tile == m->tile_width ? m->tile_ptr : nullptr;
  a.search = p.n_tiles > 1 && a.tile_ptr == nullptr;
  a.out = p.chunks > 1 ? ws : (void*)y; a.w = m->w;
  a.n_pre = m->n_pre; a.n_post = m->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  s = launch_scatter<kCsrVec>(a, p, st);
  if (s) return s;
  return finish_partials(p, false, ws, m->n_post, m->w, y, st);
}

size_t bp_event_csr_matmat_ws_bytes(const bp_csr* m, int32_t batch) {
  if (!m || batch <= 0) return 0;
  int32_t mb, groups;
  return plan_csr_batch(m, batch, &mb, &groups).ws;
}

// Shared argument checks of the batched spike products.
static bp_status check_batch(int32_t batch, int64_t ev_stride, int64_t y_stride, int32_t n_pre, int32_t n_post,
                             const uint8_t* events, const float* y) {
  BP_REQUIRE(batch >= 0, "negative batch");
  BP_REQUIRE(n_pre < (1 << 24), "batched products take n_pre < 2^24 (got %d)", n_pre);
  BP_REQUIRE(ev_stride >= n_pre && y_stride >= n_post, "strides below the vector lengths");
  BP_REQUIRE(batch == 0 || n_post == 0 || y != nullptr, "null y");
  BP_REQUIRE(batch == 0 || n_pre == 0 || events != nullptr, "null events");
  return BP_OK;
}

bp_status bp_event_csr_matmat(const bp_csr* m, const uint8_t* events, int32_t batch, int64_t ev_stride, float* y,
                              int64_t y_stride, void* ws, size_t ws_bytes, bp_stream stream) {
  bp_status s = check_csr(m);
  if (s) return s;
  s = check_batch(batch, ev_stride, y_stride, m->n_pre, m->n_post, events, y);
  if (s) return s;
  if (batch == 0 || m->n_post == 0) return BP_OK;
  if (!m->sorted) return set_error(BP_EUNSUPPORTED, "batched CSR products need strictly increasing rows");
  int32_t mb, groups;
  const MvPlan p = plan_csr_batch(m, batch, &mb, &groups);
  BP_REQUIRE(groups <= 65535, "too many vector groups (%d)", groups);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  const bool counts = m->data == nullptr;
  hipStream_t st = as_stream(stream);
  MvArgs a{};
  a.indptr = m->indptr; a.indices = m->indices; a.data = m->data;
  a.tile_ptr = p.n_tiles > 1 && m->tile_ptr && p.tile == m->tile_width ? m->tile_ptr : nullptr;
  a.search = p.n_tiles > 1 && a.tile_ptr == nullptr;
  a.events = events; a.out = p.chunks > 1 ? ws : (void*)y; a.w = m->w;
  a.batch = batch; a.mb = mb; a.ev_stride = ev_stride; a.y_stride = y_stride;
  a.n_pre = m->n_pre; a.n_post = m->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  const dim3 grid((unsigned)(p.n_tiles * p.chunks), (unsigned)groups);
  if (counts) mv_scatter_k<kCsrHomoB><<<grid, kMvThreads, 0, st>>>(a);
  else mv_scatter_k<kCsrDataB><<<grid, kMvThreads, 0, st>>>(a);
  BP_LAUNCHED("mv_scatter_k");
  return finish_batch(p, counts, ws, batch, m->n_post, m->w, y, y_stride, st);
}

size_t bp_jit_conn_matmat_ws_bytes(const bp_jit_conn* c, int32_t batch) {
  if (!c || batch <= 0) return 0;
  int32_t mb, groups;
  return plan_jit_batch(c, batch, &mb, &groups).ws;
}

bp_status bp_jit_conn_matmat(const bp_jit_conn* c, const uint8_t* events, int32_t batch, int64_t ev_stride, float* y,
                             int64_t y_stride, void* ws, size_t ws_bytes, bp_stream stream) {
  bp_status s = check_conn(c, true);
  if (s) return s;
  s = check_batch(batch, ev_stride, y_stride, c->n_pre, c->n_post, events, y);
  if (s) return s;
  if (batch == 0 || c->n_post == 0) return BP_OK;
  int32_t mb, groups;
  const MvPlan p = plan_jit_batch(c, batch, &mb, &groups);
  BP_REQUIRE(groups <= 65535, "too many vector groups (%d)", groups);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  const bool counts = c->wkind == kWHomo;
  hipStream_t st = as_stream(stream);
  MvArgs a{};
  a.jit = *c; a.events = events; a.out = p.chunks > 1 ? ws : (void*)y; a.w = c->w0;
  a.batch = batch; a.mb = mb; a.ev_stride = ev_stride; a.y_stride = y_stride;
  a.n_pre = c->n_pre; a.n_post = c->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  const dim3 grid((unsigned)(p.n_tiles * p.chunks), (unsigned)groups);
  if (counts) mv_scatter_k<kJitHomoB><<<grid, kMvThreads, 0, st>>>(a);
  else mv_scatter_k<kJitWeightedB><<<grid, kMvThreads, 0, st>>>(a);
  BP_LAUNCHED("mv_scatter_k");
  return finish_batch(p, counts, ws, batch, c->n_post, c->w0, y, y_stride, st);
}

size_t bp_jit_ws_bytes(const bp_jit_conn* c) {
  if (!c) return 0;
  return plan_jit(c, c->wkind == kWHomo).ws;
}

bp_status bp_jit_conn_matvec(const bp_jit_conn* c, const uint8_t* events, float* y, void* ws, size_t ws_bytes,
                             bp_stream stream) {
  bp_status s = check_conn(c, true);
  if (s) return s;
  if (c->n_post == 0) return BP_OK;
  BP_REQUIRE(y != nullptr, "null y");
  BP_REQUIRE(c->n_pre == 0 || events != nullptr, "null events");
  hipStream_t st = as_stream(stream);
  const bool homo = c->wkind == kWHomo;
  const MvPlan p = plan_jit(c, homo);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  MvArgs a{};
  a.jit = *c; a.events = events; a.out = p.chunks > 1 ? ws : (void*)y; a.w = c->w0;
  a.n_pre = c->n_pre; a.n_post = c->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  s = homo ? launch_scatter<kJitHomo>(a, p, st) : launch_scatter<kJitWeighted>(a, p, st);
  if (s) return s;
  return finish_partials(p, homo, ws, c->n_post, c->w0, y, st);
}

size_t bp_jit_dense_ws_bytes(const bp_jit_conn* c) {
  if (!c) return 0;
  return plan_jit(c, false, true).ws;
}

bp_status bp_jit_conn_matvec_dense(const bp_jit_conn* c, const float* v, float* y, void* ws, size_t ws_bytes,
                                   bp_stream stream) {
  bp_status s = check_conn(c, true);
  if (s) return s;
  if (c->n_post == 0) return BP_OK;
  BP_REQUIRE(y != nullptr, "null y");
  BP_REQUIRE(c->n_pre == 0 || v != nullptr, "null v");
  hipStream_t st = as_stream(stream);
  const MvPlan p = plan_jit(c, false, true);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  MvArgs a{};
  a.jit = *c; a.vec = v; a.out = p.chunks > 1 ? ws : (void*)y; a.w = c->w0;
  a.n_pre = c->n_pre; a.n_post = c->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  s = launch_scatter<kJitVec>(a, p, st);
  if (s) return s;
  return finish_partials(p, false, ws, c->n_post, c->w0, y, st);
}

size_t bp_jit_matmat_ws_bytes(const bp_jit_conn* c, int32_t m) {
  if (!c || m <= 0) return 0;
  int32_t mg, groups;
  return plan_jit_mat(c, m, &mg, &groups).ws;
}

bp_status bp_jit_conn_matmat_dense(const bp_jit_conn* c, const float* X, int32_t m, float* Y, void* ws,
                                   size_t ws_bytes, bp_stream stream) {
  bp_status s = check_conn(c, true);
  if (s) return s;
  BP_REQUIRE(m >= 0, "negative m");
  if (c->n_post == 0 || m == 0) return BP_OK;
  BP_REQUIRE((int64_t)c->n_post * m <= INT32_MAX, "n_post * m exceeds 2^31 - 1");
  BP_REQUIRE(Y != nullptr, "null Y");
  BP_REQUIRE(c->n_pre == 0 || X != nullptr, "null X");
  hipStream_t st = as_stream(stream);
  int32_t mg, groups;
  const MvPlan p = plan_jit_mat(c, m, &mg, &groups);
  BP_REQUIRE(groups <= 65535, "too many column groups (%d)", groups);
  BP_REQUIRE(ws_bytes >= p.ws && (p.ws == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, p.ws);
  MvArgs a{};
  a.jit = *c; a.x = X; a.m = m; a.mg = mg; a.out = p.chunks > 1 ? ws : (void*)Y;
  a.n_pre = c->n_pre; a.n_post = c->n_post; a.tile = p.tile; a.n_tiles = p.n_tiles;
  a.chunks = p.chunks; a.chunk_rows = p.chunk_rows;
  mv_scatter_k<kJitMat><<<dim3(p.n_tiles * p.chunks, groups), kMvThreads, 0, st>>>(a);
  BP_LAUNCHED("mv_scatter_k");
  MvPlan flat = p;  // the partials are [chunk][n_post * m]: tiles of tile * m floats
  flat.tile = p.tile * m;
  return finish_partials(flat, false, ws, c->n_post * m, c->w0, Y, st);
}

bp_status bp_event_csr_backward(const bp_csr* m, const uint8_t* events, const float* dy, float* d_events,
                                float* d_data, float* d_w, bp_stream stream) {
  bp_status s = check_csr(m);
  if (s) return s;
  hipStream_t st = as_stream(stream);
  if (d_w) {
    zero_f32_k<<<1, 64, 0, st>>>(d_w, 1);
    BP_LAUNCHED("zero_f32_k");
  }
  if (m->n_pre == 0) return BP_OK;
  BP_REQUIRE(events && dy, "null events or dy");
  const int64_t waves = m->n_pre;
  const int64_t want = (waves + 3) / 4;
  const int blocks = (int)(want < 4096 ? want : 4096);
  csr_backward_k<<<blocks, 256, 0, st>>>(*m, events, dy, d_events, d_data, d_w);
  BP_LAUNCHED("csr_backward_k");
  return BP_OK;
}

bp_status bp_jit_conn_backward(const bp_jit_conn* c, const uint8_t* events, const float* dy, float* d_events,
                               float* d_w, bp_stream stream) {
  bp_status s = check_conn(c, true);
  if (s) return s;
  hipStream_t st = as_stream(stream);
  if (d_w) {
    zero_f32_k<<<1, 64, 0, st>>>(d_w, 2);
    BP_LAUNCHED("zero_f32_k");
  }
  if (c->n_pre == 0) return BP_OK;
  BP_REQUIRE(events && dy, "null events or dy");
  // lanes per row: one per post block (rounded up to a power of two), 64 for
  // exactly fixed out-degree (one per target), 1 for a single block
  const int32_t nb = c->block > 0 ? (int32_t)(((int64_t)c->n_post + c->block - 1) / c->block) : 1;
  int lpr = 1;
  if (c->rule == kRuleFixedDegree) lpr = 64;
  else
    while (lpr < nb && lpr < 64) lpr *= 2;
  const int64_t threads = (int64_t)c->n_pre * lpr;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  switch (lpr) {
    case 1: jit_backward_k<1><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    case 2: jit_backward_k<2><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    case 4: jit_backward_k<4><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    case 8: jit_backward_k<8><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    case 16: jit_backward_k<16><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    case 32: jit_backward_k<32><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
    default: jit_backward_k<64><<<grid, 256, 0, st>>>(*c, events, dy, d_events, d_w); break;
  }
  BP_LAUNCHED("jit_backward_k");
  return BP_OK;
}

bp_status bp_backward(int32_t op, const void* args, const uint8_t* events, const float* dy, float* d_events,
                      float* d_data, float* d_w, bp_stream stream) {
  BP_REQUIRE(args != nullptr, "null args");
  if (op == 0) return bp_event_csr_backward((const bp_csr*)args, events, dy, d_events, d_data, d_w, stream);
  if (op == 1) return bp_jit_conn_backward((const bp_jit_conn*)args, events, dy, d_events, d_w, stream);
  return set_error(BP_EINVAL, "unknown op %d", op);
}

}  // extern "C"
