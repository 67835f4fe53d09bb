// Spike compaction: ascending ids of the non-zero bytes of a spike vector
// (the event set that event-driven work iterates over, Appendix B).
// Two passes over tiles of 4096 bytes: per-tile counts, then each tile adds
// the counts of the tiles before it and writes its ids in order.
#include "bp_device.h"
#include "bp_host.h"

namespace bp {

constexpr int kCompactThreads = 256;
constexpr int kCompactPer = 16;  // bytes per thread
constexpr int kCompactTile = kCompactThreads * kCompactPer;

__device__ __forceinline__ int load_bits16(const uint8_t* s, int64_t base, int64_t n, uint32_t* bits) {
  uint32_t m = 0;
  if (base + kCompactPer <= n && ((uintptr_t)(s + base) & 15u) == 0) {
    const uint4 v = *reinterpret_cast<const uint4*>(s + base);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if ((w[q >> 2] >> (8 * (q & 3))) & 0xFFu) m |= 1u << q;
  } else {
    for (int q = 0; q < kCompactPer; ++q)
      if (base + q < n && s[base + q]) m |= 1u << q;
  }
  *bits = m;
  return __popc(m);
}

__global__ void __launch_bounds__(kCompactThreads) compact_count_k(const uint8_t* __restrict__ s, int64_t n,
                                                                     int32_t* __restrict__ tile_counts) {
  __shared__ int red[kCompactThreads / kWave];
  uint32_t bits;
  const int c = load_bits16(s, (int64_t)blockIdx.x * kCompactTile + threadIdx.x * kCompactPer, n, &bits);
  const int ws = wave_sum(c);
  if (lane_id() == 0) red[threadIdx.x / kWave] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kCompactThreads / kWave; ++w) t += red[w];
    tile_counts[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kCompactThreads) compact_write_k(const uint8_t* __restrict__ s, int64_t n,
                                                                     const int32_t* __restrict__ tile_counts,
                                                                     int32_t ntiles, int32_t* __restrict__ ids,
                                                                     int32_t* __restrict__ count) {
  __shared__ int scratch[kCompactThreads / kWave + 1];
  __shared__ int base_s;
  // sum of the counts of earlier tiles
  int acc = 0;
  for (int t = threadIdx.x; t < (int)blockIdx.x; t += kCompactThreads) acc += tile_counts[t];
  int tot;
  block_excl_scan(acc, scratch, &tot);
  if (threadIdx.x == 0) base_s = tot;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kCompactTile + threadIdx.x * kCompactPer;
  uint32_t bits;
  const int c = load_bits16(s, base, n, &bits);
  int tile_tot;
  int off = base_s + block_excl_scan(c, scratch, &tile_tot);
  while (bits) {
    const int q = __ffs(bits) - 1;
    bits &= bits - 1;
    if (off < n) ids[off] = (int32_t)(base + q);
    ++off;
  }
  if (blockIdx.x == (unsigned)(ntiles - 1) && threadIdx.x == 0) *count = base_s + tile_tot;
}

}  // namespace bp

using namespace bp;

extern "C" {

size_t bp_compact_ws_bytes(int32_t n) {
  const int64_t nt = n > 0 ? ((int64_t)n + kCompactTile - 1) / kCompactTile : 1;
  return (size_t)nt * sizeof(int32_t);
}

__global__ void bp_zero_int_k(int32_t* p) { *p = 0; }

bp_status bp_compact(const uint8_t* s, int32_t n, int32_t* ids, int32_t* count, void* ws, size_t ws_bytes,
                     bp_stream stream) {
  BP_REQUIRE(n >= 0, "negative n");
  BP_REQUIRE(count != nullptr, "null count");
  hipStream_t st = as_stream(stream);
  if (n == 0) {
    bp_zero_int_k<<<1, 1, 0, st>>>(count);
    BP_LAUNCHED("bp_zero_int_k");
    return BP_OK;
  }
  BP_REQUIRE(s && ids && ws, "null pointer");
  BP_REQUIRE(ws_bytes >= bp_compact_ws_bytes(n), "workspace too small (%zu < %zu)", ws_bytes, bp_compact_ws_bytes(n));
  const int32_t nt = (int32_t)(((int64_t)n + kCompactTile - 1) / kCompactTile);
  compact_count_k<<<nt, kCompactThreads, 0, st>>>(s, n, (int32_t*)ws);
  BP_LAUNCHED("compact_count_k");
  compact_write_k<<<nt, kCompactThreads, 0, st>>>(s, n, (const int32_t*)ws, nt, ids, count);
  BP_LAUNCHED("compact_write_k");
  return BP_OK;
}

}  // extern "C"
