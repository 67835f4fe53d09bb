// Counter-based hash entry point, maximum-gap rule and the seeded CSR build
// (Appendix C matrix stored in the Appendix B format).
#include <math.h>
#include <string.h>

#include "bp_device.h"
#include "bp_host.h"

namespace bp {

static thread_local char g_err[512] = "";

bp_status set_error(bp_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

__global__ void hash_k(uint64_t seed, uint32_t stream, const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                       const uint32_t* __restrict__ k, uint32_t* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = hash_word(seed, stream, a[i], b[i], k[i]);
}

// One thread per row: number of targets of row j (all blocks) -> rowlen[j].
__global__ void csr_rowlen_k(bp_jit_conn c, int32_t* __restrict__ rowlen) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c.n_pre) return;
  if (c.rule == kRuleFixedDegree) {  // exactly min(degree, n_post) targets
    rowlen[j] = c.degree < c.n_post ? c.degree : c.n_post;
    return;
  }
  const ConnGen G = conn_gen(c);
  const int32_t nb = c.block > 0 ? (int32_t)(((int64_t)c.n_post + c.block - 1) / c.block) : 1;
  int32_t cnt = 0;
  for (int32_t b = 0; b < nb; ++b) gen_block(G, (uint32_t)j, (uint32_t)b, 0, c.n_post, [&](int32_t, uint32_t) { ++cnt; });
  rowlen[j] = cnt;
}

// In-place inclusive scan of a[1..n] by one workgroup (a[0] = 0 on exit), so
// that a becomes the row-pointer array.  A total above INT32_MAX is reported
// by writing -1 to a[n].
__global__ void __launch_bounds__(1024) scan_rowptr_k(int32_t* a, int32_t n) {
  __shared__ int scratch[1024 / kWave + 1];
  __shared__ long long carry_s;
  if (threadIdx.x == 0) { carry_s = 0; a[0] = 0; }
  __syncthreads();
  for (int32_t base = 1; base <= n; base += blockDim.x) {
    const int32_t i = base + threadIdx.x;
    const int v = (i <= n) ? a[i] : 0;
    int tot;
    const int ex = block_excl_scan(v, scratch, &tot);
    const long long carry = carry_s;
    if (i <= n) {
      const long long r = carry + ex + v;
      a[i] = r > 2147483647LL ? -1 : (int32_t)r;
    }
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && carry_s > 2147483647LL) a[n] = -1;
}

__global__ void csr_fill_k(bp_jit_conn c, const int32_t* __restrict__ indptr, int32_t* __restrict__ indices) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c.n_pre) return;
  const int32_t nb = c.block > 0 ? (int32_t)(((int64_t)c.n_post + c.block - 1) / c.block) : 1;
  int32_t* out = indices + indptr[j];
  const int32_t cap = indptr[j + 1] - indptr[j];
  const ConnGen G = conn_gen(c);
  int32_t cnt = 0;
  for (int32_t b = 0; b < nb; ++b)
    gen_block(G, (uint32_t)j, (uint32_t)b, 0, c.n_post, [&](int32_t pos, uint32_t) {
      if (cnt < cap) out[cnt] = pos;
      ++cnt;
    });
  if (c.rule == kRuleFixedDegree) {
    // the targets come in permutation order: heapsort the row in place so
    // that stored rows are strictly increasing like the other rules'
    const int32_t n = cnt < cap ? cnt : cap;
    auto sift = [&](int32_t root, int32_t end) {
      const int32_t v = out[root];
      while (2 * root + 1 < end) {
        int32_t ch = 2 * root + 1;
        if (ch + 1 < end && out[ch + 1] > out[ch]) ++ch;
        if (out[ch] <= v) break;
        out[root] = out[ch];
        root = ch;
      }
      out[root] = v;
    };
    for (int32_t r = n / 2 - 1; r >= 0; --r) sift(r, n);
    for (int32_t e = n - 1; e > 0; --e) {
      const int32_t t = out[0];
      out[0] = out[e];
      out[e] = t;
      sift(0, e);
    }
  }
}

// Tile index of a sorted CSR: tp[j][t] = first idx of row j with column >= t*P.
__global__ void csr_tile_index_k(const int32_t* __restrict__ indptr, const int32_t* __restrict__ indices, int32_t n_pre,
                                 int32_t tile, int32_t n_tiles, int32_t* __restrict__ tp) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_pre) return;
  const int32_t s = indptr[j], e = indptr[j + 1];
  int32_t* out = tp + (size_t)j * (n_tiles + 1);
  int32_t idx = s;
  for (int32_t t = 0; t <= n_tiles; ++t) {
    const int64_t bound = (int64_t)t * tile;
    // rows are sorted: advance by binary search from idx
    int32_t l = idx, h = e;
    while (l < h) {
      const int32_t mid = (l + h) >> 1;
      if (indices[mid] < bound) l = mid + 1; else h = mid;
    }
    idx = l;
    out[t] = (t == n_tiles) ? e : idx;
  }
}

bp_status launch_tile_index(const int32_t* indptr, const int32_t* indices, int32_t n_pre, int32_t tile,
                            int32_t n_tiles, int32_t* tp, hipStream_t st) {
  if (n_pre <= 0) return BP_OK;
  csr_tile_index_k<<<(n_pre + 255) / 256, 256, 0, st>>>(indptr, indices, n_pre, tile, n_tiles, tp);
  BP_LAUNCHED("csr_tile_index_k");
  return BP_OK;
}

bp_status check_rule(int32_t rule, int32_t max_gap, float inv_rate, int32_t degree, int32_t block) {
  BP_REQUIRE(rule == kRuleUniform || rule == kRuleGeometric || rule == kRuleFixedDegree, "unknown rule %d", rule);
  if (rule == kRuleUniform) BP_REQUIRE(max_gap >= 1, "max_gap must be >= 1 (got %d)", max_gap);
  if (rule == kRuleGeometric)
    BP_REQUIRE(inv_rate >= 0.f && inv_rate < 1e30f, "geo_inv_rate must be finite and >= 0 (got %g)", inv_rate);
  if (rule == kRuleFixedDegree) {
    BP_REQUIRE(degree >= 0, "degree must be >= 0 (got %d)", degree);
    BP_REQUIRE(block == 0, "fixed out-degree rows take one post block (block 0, got %d)", block);
  }
  return BP_OK;
}

bp_status check_conn(const bp_jit_conn* c, bool weights) {
  BP_REQUIRE(c != nullptr, "null connectivity descriptor");
  BP_REQUIRE(c->n_pre >= 0 && c->n_post >= 0, "negative size (n_pre %d, n_post %d)", c->n_pre, c->n_post);
  BP_REQUIRE(c->block >= 0, "block must be >= 0 (got %d)", c->block);
  bp_status s = check_rule(c->rule, c->max_gap, c->geo_inv_rate, c->degree, c->block);
  if (s) return s;
  if (weights)
    BP_REQUIRE(c->wkind == kWHomo || c->wkind == kWNormal || c->wkind == kWUniform, "unknown weight kind %d",
               c->wkind);
  return BP_OK;
}

}  // namespace bp

using namespace bp;

extern "C" {

const char* bp_last_error(void) { return bp::g_err; }
const char* bp_version(void) { return "bpmi 0.1 gfx950"; }

float bp_geo_inv_rate(double p) {
  if (!(p > 0.0) || !(p < 1.0)) return 0.0f;
  return (float)(1.0 / -log1p(-p));
}

int32_t bp_max_gap(double p) {
  if (!(p > 0.0) || p > 1.0) return -1;
  const double x = 2.0 / p - 1.0;
  const double r = floor(x + 0.5);
  double K = (fabs(x - r) <= 1e-9 * x) ? r : floor(x);
  if (K < 1.0) K = 1.0;
  if (K > 2147483646.0) return -1;
  return (int32_t)K;
}

bp_status bp_hash(uint64_t seed, uint32_t rng_stream, const uint32_t* a, const uint32_t* b, const uint32_t* k,
                  uint32_t* out, int64_t n, bp_stream stream) {
  BP_REQUIRE(n >= 0, "negative n");
  if (n == 0) return BP_OK;
  BP_REQUIRE(a && b && k && out, "null pointer");
  const int64_t blocks = (n + 255) / 256;
  hash_k<<<(unsigned)(blocks < 65536 ? blocks : 65536), 256, 0, as_stream(stream)>>>(seed, rng_stream, a, b, k, out, n);
  BP_LAUNCHED("hash_k");
  return BP_OK;
}

bp_status bp_csr_count(const bp_jit_conn* c, int32_t* indptr, bp_stream stream) {
  bp_status s = check_conn(c, false);
  if (s) return s;
  BP_REQUIRE(indptr != nullptr, "null indptr");
  hipStream_t st = as_stream(stream);
  if (c->n_pre > 0) {
    csr_rowlen_k<<<(c->n_pre + 255) / 256, 256, 0, st>>>(*c, indptr + 1);
    BP_LAUNCHED("csr_rowlen_k");
  }
  scan_rowptr_k<<<1, 1024, 0, st>>>(indptr, c->n_pre);
  BP_LAUNCHED("scan_rowptr_k");
  return BP_OK;
}

bp_status bp_csr_fill(const bp_jit_conn* c, const int32_t* indptr, int32_t* indices, bp_stream stream) {
  bp_status s = check_conn(c, false);
  if (s) return s;
  BP_REQUIRE(indptr != nullptr, "null indptr");
  if (c->n_pre == 0) return BP_OK;
  BP_REQUIRE(indices != nullptr, "null indices");
  csr_fill_k<<<(c->n_pre + 255) / 256, 256, 0, as_stream(stream)>>>(*c, indptr, indices);
  BP_LAUNCHED("csr_fill_k");
  return BP_OK;
}

}  // extern "C"
