// Synaptic projections with multi-step spike delays (Section 4.3,
// Appendix D; Appendix F's synaptic delays) built on the event-driven and
// float-vector products.
//
// A delay line is a ring of spike vectors in device memory, [depth][n]
// bytes, slot t mod depth holding the spikes of step t (zeroed by the caller
// before step 0, so steps before 0 read as silent).  A projection step reads
// the spikes of step t - delay from it:
//   AlignPost: y = M^T s (event product: integer counts for homogeneous
//              weights), then g <- g d + y elementwise;
//   AlignPre:  x <- x d + s (or the saturating x <- x d + u (1 - x d) on a
//              spike), one trace per presynaptic neuron, then g = M^T x (the
//              float-vector product over the rows with x != 0).
// Every FP32 operation of the state updates is rounded on its own in the
// order written (the library is built without contraction), which the
// oracle's FP32 recursion mirrors.
#include "bp_device.h"
#include "bp_host.h"

namespace bp {

__global__ void proj_zero_k(float* __restrict__ p, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// g[k] = g[k] * d + y[k]
__global__ void exp_accum_k(float* __restrict__ g, const float* __restrict__ y, float d, int32_t n) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const float gd = g[k] * d;
    g[k] = gd + y[k];
  }
}

// x[j] <- x[j] d, then + 1 (exponential) or + u (1 - x) (saturating) where
// the delayed spike is set; s may be null (no spikes yet).
__global__ void trace_k(float* __restrict__ x, const uint8_t* __restrict__ s, float d, float u, int32_t sat,
                        int32_t n) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float xp = x[j] * d;
  float v = xp;
  if (s && s[j]) {
    if (sat) {
      const float r = 1.0f - xp;
      const float inc = u * r;
      v = xp + inc;
    } else {
      v = xp + 1.0f;
    }
  }
  x[j] = v;
}

static bp_status check_proj(const bp_proj* p, int32_t* n_pre, int32_t* n_post) {
  BP_REQUIRE(p != nullptr, "null projection");
  BP_REQUIRE(p->align == BP_ALIGN_POST || p->align == BP_ALIGN_PRE, "unknown alignment %d", p->align);
  BP_REQUIRE(p->syn == BP_SYN_EXP || (p->syn == BP_SYN_SAT && p->align == BP_ALIGN_PRE),
             "synapse model %d (the saturating synapse needs AlignPre)", p->syn);
  BP_REQUIRE(p->delay >= 0, "negative delay");
  if (p->conn == BP_CONN_CSR) {
    BP_REQUIRE(p->csr != nullptr, "null CSR");
    *n_pre = p->csr->n_pre;
    *n_post = p->csr->n_post;
  } else if (p->conn == BP_CONN_JIT) {
    BP_REQUIRE(p->jit != nullptr, "null JIT descriptor");
    bp_status s = check_conn(p->jit, true);
    if (s) return s;
    *n_pre = p->jit->n_pre;
    *n_post = p->jit->n_post;
  } else {
    return set_error(BP_EINVAL, "unknown connectivity %d", p->conn);
  }
  return BP_OK;
}

// Scratch of the product the projection runs.
static size_t product_ws(const bp_proj* p) {
  if (p->conn == BP_CONN_CSR)
    return p->align == BP_ALIGN_POST ? bp_event_csr_ws_bytes(p->csr) : bp_csr_matvec_dense_ws_bytes(p->csr);
  return p->align == BP_ALIGN_POST ? bp_jit_ws_bytes(p->jit) : bp_jit_dense_ws_bytes(p->jit);
}

}  // namespace bp

using namespace bp;

extern "C" {

bp_status bp_delay_push(uint8_t* ring, int32_t depth, int32_t n, int64_t t, const uint8_t* spikes,
                        bp_stream stream) {
  BP_REQUIRE(depth >= 1 && n >= 0 && t >= 0, "bad delay line (depth %d, n %d, step %lld)", depth, n, (long long)t);
  if (n == 0) return BP_OK;
  BP_REQUIRE(ring && spikes, "null pointer");
  BP_HIP(hipMemcpyAsync(ring + (size_t)(t % depth) * n, spikes, (size_t)n, hipMemcpyDeviceToDevice,
                        as_stream(stream)));
  return BP_OK;
}

size_t bp_proj_ws_bytes(const bp_proj* p) {
  int32_t n_pre = 0, n_post = 0;
  if (!p || check_proj(p, &n_pre, &n_post)) return 0;
  const size_t y = p->align == BP_ALIGN_POST ? align_up((size_t)n_post * 4, 256) : 0;
  return y + product_ws(p);
}

bp_status bp_proj_step(const bp_proj* p, const uint8_t* ring, int32_t depth, int64_t t, float* state, float* g,
                       void* ws, size_t ws_bytes, bp_stream stream) {
  int32_t n_pre = 0, n_post = 0;
  bp_status s = check_proj(p, &n_pre, &n_post);
  if (s) return s;
  BP_REQUIRE(depth >= 1 && p->delay < depth, "delay %d needs a ring deeper than %d", p->delay, depth);
  BP_REQUIRE(t >= 0, "negative step");
  BP_REQUIRE(n_pre == 0 || ring != nullptr, "null ring");
  BP_REQUIRE(state != nullptr || (p->align == BP_ALIGN_POST ? n_post : n_pre) == 0, "null state");
  BP_REQUIRE(g != nullptr || n_post == 0 || p->align == BP_ALIGN_POST, "null g");
  const size_t need = bp_proj_ws_bytes(p);
  BP_REQUIRE(ws_bytes >= need && (need == 0 || ws != nullptr), "workspace too small (%zu < %zu)", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  // the spikes of step t - delay (none before step 0)
  const uint8_t* sd = t - p->delay >= 0 && n_pre > 0 ? ring + (size_t)((t - p->delay) % depth) * n_pre : nullptr;
  if (p->align == BP_ALIGN_POST) {
    if (n_post == 0) return BP_OK;
    float* y = (float*)ws;
    void* pws = (char*)ws + align_up((size_t)n_post * 4, 256);
    const size_t pwb = ws_bytes - align_up((size_t)n_post * 4, 256);
    if (sd) {
      s = p->conn == BP_CONN_CSR ? bp_event_csr_matvec(p->csr, sd, y, pws, pwb, stream)
                                 : bp_jit_conn_matvec(p->jit, sd, y, pws, pwb, stream);
      if (s) return s;
    } else {
      proj_zero_k<<<(n_post + 255) / 256, 256, 0, st>>>(y, n_post);
      BP_LAUNCHED("proj_zero_k");
    }
    exp_accum_k<<<(n_post + 255) / 256, 256, 0, st>>>(state, y, p->decay, n_post);
    BP_LAUNCHED("exp_accum_k");
    if (g && g != state) BP_HIP(hipMemcpyAsync(g, state, (size_t)n_post * 4, hipMemcpyDeviceToDevice, st));
    return BP_OK;
  }
  if (n_pre > 0) {
    trace_k<<<(n_pre + 255) / 256, 256, 0, st>>>(state, sd, p->decay, p->u, p->syn == BP_SYN_SAT, n_pre);
    BP_LAUNCHED("trace_k");
  }
  if (n_post == 0) return BP_OK;
  return p->conn == BP_CONN_CSR ? bp_csr_matvec_dense(p->csr, state, g, ws, ws_bytes, stream)
                                : bp_jit_conn_matvec_dense(p->jit, state, g, ws, ws_bytes, stream);
}

bp_status bp_proj_run(const bp_proj* p, const uint8_t* raster, int32_t T, uint8_t* ring, int32_t depth, int64_t t0,
                      float* state, float* g_out, void* ws, size_t ws_bytes, bp_stream stream) {
  int32_t n_pre = 0, n_post = 0;
  bp_status s = check_proj(p, &n_pre, &n_post);
  if (s) return s;
  BP_REQUIRE(T >= 0, "negative T");
  BP_REQUIRE(T == 0 || n_pre == 0 || raster != nullptr, "null raster");
  BP_REQUIRE(g_out != nullptr || n_post == 0 || T == 0, "null g_out");
  for (int32_t i = 0; i < T; ++i) {
    const int64_t t = t0 + i;
    if ((s = bp_delay_push(ring, depth, n_pre, t, raster + (size_t)i * n_pre, stream))) return s;
    if ((s = bp_proj_step(p, ring, depth, t, state, g_out + (size_t)i * n_post, ws, ws_bytes, stream))) return s;
  }
  return BP_OK;
}

}  // extern "C"
