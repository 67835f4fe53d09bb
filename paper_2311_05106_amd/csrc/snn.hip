// Recurrent LIF network trained by backpropagation through time with a
// surrogate spike derivative (Section 5.3; Appendix I; every operator has a
// reverse mode, Section 4.1).
//
// One workgroup per sample, one thread per neuron.  Forward step t:
//   I = alpha I + sum over firing input channels (ascending) of W_in[c, k]
//             + sum over firing presynaptic neurons j (ascending) of w_jk
//   V = beta V (1 - z_prev) + (1 - beta) I ;  z = [V > theta]
// The recurrent sum is event-driven: the rows of the neurons that fired are
// pushed into an LDS accumulator, row after row in ascending order, each wave
// adding the entries that fall in its 64 columns (a row holds a column at
// most once), so each neuron adds its inputs in a fixed order and the
// forward pass and its recomputation inside the reverse pass give identical
// spikes.
// The forward stores the state before every ckpt_every-th step; the reverse
// pass walks the segments from the last, recomputes each one, and runs the
// recurrence backward through it.  Weight gradients are accumulated per
// sample by the thread that owns each entry, then summed over samples in
// sample order.
#include <math.h>

#include "bp_device.h"
#include "bp_host.h"

namespace bp {

constexpr int kSnnMaxN = 1024;
constexpr int kSnnMaxC = 4096;
constexpr int kSnnMaxO = 64;

struct SnnLayout {
  int32_t nck;
  size_t off_I, off_V, off_z, off_zsum, ck_total;
  size_t off_segV, off_segz, off_pin, off_prec, off_dlog, off_elli, off_ellw, ws_total;
};

static SnnLayout snn_layout(const bp_snn* m) {
  SnnLayout L{};
  const size_t BN = (size_t)m->B * m->N;
  L.nck = (m->T + m->ckpt_every - 1) / m->ckpt_every;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_I = take(L.nck * BN * 4);
  L.off_V = take(L.nck * BN * 4);
  L.off_z = take(L.nck * BN);
  L.off_zsum = take(BN * 4);
  L.ck_total = o;
  o = 0;
  L.off_segV = take((size_t)m->B * m->ckpt_every * m->N * 4);
  L.off_segz = take((size_t)m->B * m->ckpt_every * m->N);
  L.off_pin = take((size_t)m->B * m->C * m->N * 4);
  L.off_prec = take((size_t)m->B * (m->nnz > 0 ? m->nnz : 1) * 4);
  L.off_dlog = take((size_t)m->B * m->O * 4);
  // the recurrent rows transposed: entry i of row k at [i][k] (rows of at
  // most N entries)
  L.off_elli = take((size_t)m->N * m->N * 4);
  L.off_ellw = take((size_t)m->N * m->N * 4);
  L.ws_total = o;
  return L;
}

struct SnnDev {
  int32_t B, C, N, O, T, nnz, surrogate, detach, E, nck;
  float alpha, beta, omb, theta, slope, relu_a, relu_w;
  const uint8_t* x;
  const int32_t* labels;
  const float* W_in;
  const int32_t* indptr;
  const int32_t* indices;
  const float* w_rec;
  const float* W_out;
  const float* b_out;
  float* ckI;
  float* ckV;
  uint8_t* ckz;
  float* zsum;
};

struct SnnShared {
  uint8_t zprev[kSnnMaxN];
  int ch[kSnnMaxC];
  int sp[kSnnMaxN];     // neurons that fired at the previous step, ascending
  int rlo[kSnnMaxN];    // their rows in the recurrent CSR: [rlo, rhi)
  int rhi[kSnnMaxN];
  float acc[kSnnMaxN];  // input current being accumulated
  int scratch[2 * (1024 / kWave + 1)];
  int nch, nsp;
  float red[kSnnMaxO][1024 / kWave];
};

// Input bytes of one step held by wave 0 (up to 256 channels), loaded one
// step ahead of their use.
struct XPre {
  int t;
  bool on[4];
};

// Ascending lists of the firing input channels of sample b at step t (wave
// 0) and of the neurons with sh.zprev set (the last wave), by wave ballots;
// ends with a barrier.  Wave 0 also loads the input bytes of step t_next
// (-1: none) into xp.
__device__ __forceinline__ void stage_lists(const SnnDev& m, int b, int t, SnnShared& sh, XPre& xp, int t_next) {
  const int wv = threadIdx.x / kWave, l = lane_id(), last = blockDim.x / kWave - 1;
  if (wv == 0 && m.C <= 4 * kWave) {
    bool on[4];
    const uint8_t* xt = m.x + ((size_t)t * m.B + b) * m.C;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int c = g * kWave + l;
      on[g] = xp.t == t ? xp.on[g] : (c < m.C && xt[c]);
    }
    xp.t = t_next;
    if (t_next >= 0) {
      const uint8_t* xn = m.x + ((size_t)t_next * m.B + b) * m.C;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int c = g * kWave + l;
        xp.on[g] = c < m.C && xn[c];
      }
    }
    int base = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint64_t msk = __ballot(on[g]);
      if (on[g]) sh.ch[base + mask_rank(msk)] = g * kWave + l;
      base += __popcll(msk);
    }
    if (l == 0) sh.nch = base;
  } else if (wv == 0) {
    const uint8_t* xt = m.x + ((size_t)t * m.B + b) * m.C;
    int base = 0;
    for (int c0 = 0; c0 < m.C; c0 += 4 * kWave) {
      // four 64-channel groups loaded together, then compacted in order
      bool on[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int c = c0 + g * kWave + l;
        on[g] = c < m.C && xt[c];
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint64_t msk = __ballot(on[g]);
        if (on[g]) sh.ch[base + mask_rank(msk)] = c0 + g * kWave + l;
        base += __popcll(msk);
      }
    }
    if (l == 0) sh.nch = base;
  }
  if (wv == last) {
    int base = 0;
    for (int k0 = 0; k0 < m.N; k0 += kWave) {
      const int k = k0 + l;
      const bool on = k < m.N && sh.zprev[k];
      const uint64_t msk = __ballot(on);
      if (on) sh.sp[base + mask_rank(msk)] = k;
      base += __popcll(msk);
    }
    if (l == 0) sh.nsp = base;
    // row bounds of the listed neurons, all loads in flight together
    for (int r = l; r < base; r += kWave) {
      const int j = sh.sp[r];
      sh.rlo[r] = m.indptr[j];
      sh.rhi[r] = m.indptr[j + 1];
    }
  }
  __syncthreads();
}

// One forward step for neuron k given the lists of stage_lists; returns z.
// Contains two barriers (every thread of the block must call it).
__device__ __forceinline__ bool fwd_step(const SnnDev& m, int k, bool valid, float& I, float& V, SnnShared& sh) {
  if (valid) {
    // input channels in list order, eight loads in flight at a time
    float acc = m.alpha * I;
    const int nch = sh.nch;
    for (int q0 = 0; q0 < nch; q0 += 8) {
      float wv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wv[u] = q0 + u < nch ? m.W_in[(size_t)sh.ch[q0 + u] * m.N + k] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < nch) acc = acc + wv[u];
    }
    sh.acc[k] = acc;
  }
  __syncthreads();
  // recurrent input: rows of the fired neurons, ascending; wave w adds the
  // entries of columns [64 w, 64 w + 64).  The first 64 entries of four rows
  // are loaded together, then added row by row (the same order per column).
  const int klo = (int)(threadIdx.x / kWave) * kWave, l = lane_id();
  const int nsp = sh.nsp;
  for (int r0 = 0; r0 < nsp; r0 += 4) {
    int kk[4];
    float wr[4];
    int rl[4], rh[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // r0 + u < kSnnMaxN: unguarded LDS reads, masked below
      rl[u] = sh.rlo[r0 + u];
      rh[u] = sh.rhi[r0 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      kk[u] = -1;
      wr[u] = 0.f;
      const int e = rl[u] + l;
      if (r0 + u < nsp && e < rh[u]) {
        kk[u] = m.indices[e];
        wr[u] = m.w_rec[e];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (r0 + u < nsp) {
        if (kk[u] >= klo && kk[u] < klo + kWave && kk[u] < m.N) sh.acc[kk[u]] = sh.acc[kk[u]] + wr[u];
        for (int e = rl[u] + kWave + l; e < rh[u]; e += kWave) {  // rows longer than 64
          const int c = m.indices[e];
          if (c >= klo && c < klo + kWave && c < m.N) sh.acc[c] = sh.acc[c] + m.w_rec[e];
        }
      }
    }
  }
  __syncthreads();
  if (!valid) return false;
  I = sh.acc[k];
  const float vp = sh.zprev[k] ? 0.0f : V;
  V = m.beta * vp + m.omb * I;
  return V > m.theta;
}

__global__ void __launch_bounds__(1024) snn_forward_k(SnnDev m, float* logits, uint8_t* raster) {
  __shared__ SnnShared sh;
  const int b = blockIdx.x, k = threadIdx.x;
  const bool valid = k < m.N;
  float I = 0.f, V = 0.f, zs = 0.f;
  XPre xp{-1, {false, false, false, false}};
  if (valid) sh.zprev[k] = 0;
  __syncthreads();
  for (int t = 0; t < m.T; ++t) {
    if (t % m.E == 0 && valid) {
      const size_t o = ((size_t)(t / m.E) * m.B + b) * m.N + k;
      m.ckI[o] = I;
      m.ckV[o] = V;
      m.ckz[o] = sh.zprev[k];
    }
    stage_lists(m, b, t, sh, xp, t + 1 < m.T ? t + 1 : -1);
    const bool z = fwd_step(m, k, valid, I, V, sh);
    if (valid) {
      sh.zprev[k] = z ? 1 : 0;
      zs += z ? 1.f : 0.f;
      if (raster) raster[((size_t)t * m.B + b) * m.N + k] = z ? 1 : 0;
    }
    __syncthreads();
  }
  if (valid) m.zsum[(size_t)b * m.N + k] = zs;
  // logits[b, o] = b_out[o] + sum_k zsum[k] / T * W_out[k, o]
  const int nw = blockDim.x / kWave, wv = threadIdx.x / kWave;
  for (int o = 0; o < m.O; ++o) {
    float p = valid ? zs / (float)m.T * m.W_out[(size_t)k * m.O + o] : 0.f;
    p = wave_sum_f(p);
    if (lane_id() == 0) sh.red[o][wv] = p;
  }
  __syncthreads();
  if (threadIdx.x < m.O) {
    float s = m.b_out[threadIdx.x];
    for (int w = 0; w < nw; ++w) s += sh.red[threadIdx.x][w];
    logits[(size_t)b * m.O + threadIdx.x] = s;
  }
}

// loss = mean over samples of logsumexp(logits) - logits[label];
// dlog[b, o] = (softmax(logits_b)[o] - [o == label]) / B.  One thread per sample.
__global__ void snn_loss_k(SnnDev m, const float* logits, float* loss, float* dlog) {
  __shared__ float part[1024];
  float acc = 0.f;
  for (int b = threadIdx.x; b < m.B; b += blockDim.x) {
    const float* lg = logits + (size_t)b * m.O;
    float mx = lg[0];
    for (int o = 1; o < m.O; ++o) mx = fmaxf(mx, lg[o]);
    float se = 0.f;
    for (int o = 0; o < m.O; ++o) se += expf(lg[o] - mx);
    const float lse = mx + logf(se);
    acc += lse - lg[m.labels[b]];
    if (dlog)
      for (int o = 0; o < m.O; ++o)
        dlog[(size_t)b * m.O + o] = (expf(lg[o] - lse) - (o == m.labels[b] ? 1.f : 0.f)) / (float)m.B;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int i = 0; i < (int)blockDim.x; ++i) s += part[i];
    *loss = s / (float)m.B;
  }
}

__device__ __forceinline__ float surrogate(const SnnDev& m, float v) {
  const float x = v - m.theta;
  if (m.surrogate == 1) return fmaxf(0.f, m.relu_a * (m.relu_w - fabsf(x)));
  const float s = 1.f / (1.f + expf(-m.slope * x));
  return m.slope * s * (1.f - s);
}

// Copies the recurrent rows into the transposed layout read by the backward
// gather (entry i of row k at [i * N + k]: lanes of a wave, one row each,
// read consecutive words).  One thread per row.
__global__ void snn_ell_k(SnnDev m, int32_t* elli, float* ellw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.N) return;
  const int e0 = m.indptr[k], len = m.indptr[k + 1] - e0;
  for (int i = 0; i < len; ++i) {
    elli[(size_t)i * m.N + k] = m.indices[e0 + i];
    ellw[(size_t)i * m.N + k] = m.w_rec[e0 + i];
  }
}

struct SnnBwdShared {
  SnnShared f;
  float dI[kSnnMaxN];
  float dlog[kSnnMaxO];
};

__global__ void __launch_bounds__(1024) snn_backward_k(SnnDev m, const float* dlog_all, float* segV, uint8_t* segz,
                                                       float* pin, float* prec, const int32_t* elli,
                                                       const float* ellw) {
  __shared__ SnnBwdShared sh;
  const int b = blockIdx.x, k = threadIdx.x;
  const bool valid = k < m.N;
  float* pin_b = pin + (size_t)b * m.C * m.N;
  float* prec_b = prec + (size_t)b * m.nnz;
  for (size_t i = threadIdx.x; i < (size_t)m.C * m.N; i += blockDim.x) pin_b[i] = 0.f;
  for (int i = threadIdx.x; i < m.nnz; i += blockDim.x) prec_b[i] = 0.f;
  if (threadIdx.x < m.O) sh.dlog[threadIdx.x] = dlog_all[(size_t)b * m.O + threadIdx.x];
  if (valid) sh.dI[k] = 0.f;
  __syncthreads();
  float gd = 0.f;
  if (valid) {
    for (int o = 0; o < m.O; ++o) gd += m.W_out[(size_t)k * m.O + o] * sh.dlog[o];
    gd = gd / (float)m.T;
  }
  float dVn = 0.f;
  XPre xp{-1, {false, false, false, false}};
  const int re0 = valid ? m.indptr[k] : 0, re1 = valid ? m.indptr[k + 1] : 0;  // own row
  float* sV = segV + (size_t)b * m.E * m.N;
  uint8_t* sz = segz + (size_t)b * m.E * m.N;
  for (int seg = m.nck - 1; seg >= 0; --seg) {
    const int t0 = seg * m.E, t1 = min(t0 + m.E, m.T);
    // recompute the segment from its checkpoint
    float I = 0.f, V = 0.f;
    uint8_t z_start = 0;
    if (valid) {
      const size_t o = ((size_t)seg * m.B + b) * m.N + k;
      I = m.ckI[o];
      V = m.ckV[o];
      z_start = m.ckz[o];
      sh.f.zprev[k] = z_start;
    }
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
      stage_lists(m, b, t, sh.f, xp, t + 1 < t1 ? t + 1 : -1);
      const bool z = fwd_step(m, k, valid, I, V, sh.f);
      if (valid) {
        sh.f.zprev[k] = z ? 1 : 0;
        sV[(size_t)(t - t0) * m.N + k] = V;
        sz[(size_t)(t - t0) * m.N + k] = z ? 1 : 0;
      }
      __syncthreads();
    }
    // reverse through the segment; V_t and z_{t-1} of the next step are
    // loaded one step ahead (z_t is the previous step's z_{t-1})
    float Vn = 0.f;
    uint8_t zc = 0, zp = 0;
    if (valid) {
      const int i = t1 - 1 - t0;
      Vn = sV[(size_t)i * m.N + k];
      zc = sz[(size_t)i * m.N + k];
      zp = i > 0 ? sz[(size_t)(i - 1) * m.N + k] : z_start;
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const bool last = (t + 1 >= m.T);
      const float Vt = Vn;
      const bool zt = zc != 0;
      const uint8_t zprev_t = zp;
      uint8_t zp_next = 0;
      if (valid && t > t0) {
        const int i = t - 1 - t0;
        Vn = sV[(size_t)i * m.N + k];
        zp_next = i > 0 ? sz[(size_t)(i - 1) * m.N + k] : z_start;
      }
      float dI = 0.f;
      if (valid) {
        float dz = gd;
        if (!last) {
          // own row, entries in order
          float g = 0.f;
          // (transposed copy: entry i at [i * N + k], consecutive across lanes)
          const int len = re1 - re0;
          int i = 0;
          for (; i + 16 <= len; i += 16) {
            int c[16];
            float wv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              c[u] = elli[(size_t)(i + u) * m.N + k];
              wv[u] = ellw[(size_t)(i + u) * m.N + k];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) g += wv[u] * sh.dI[c[u]];
          }
          for (; i + 4 <= len; i += 4) {
            int c[4];
            float wv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              c[u] = elli[(size_t)(i + u) * m.N + k];
              wv[u] = ellw[(size_t)(i + u) * m.N + k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) g += wv[u] * sh.dI[c[u]];
          }
          for (; i < len; ++i) g += ellw[(size_t)i * m.N + k] * sh.dI[elli[(size_t)i * m.N + k]];
          dz += g;
          if (!m.detach) dz += dVn * (-m.beta * Vt);
        }
        float dV = dz * surrogate(m, Vt);
        if (!last) dV += dVn * m.beta * (zt ? 0.f : 1.f);
        dI = dV * m.omb;
        if (!last) dI += sh.dI[k] * m.alpha;
        dVn = dV;
      }
      __syncthreads();
      if (valid) {
        sh.dI[k] = dI;
        sh.f.zprev[k] = zprev_t;  // z_{t-1}: from the segment scratch or the checkpoint
      }
      zc = zprev_t;
      zp = zp_next;
      __syncthreads();
      stage_lists(m, b, t, sh.f, xp, t > t0 ? t - 1 : -1);  // ends with a barrier
      if (valid) {
        // the listed channels are distinct: eight read-modify-writes in flight
        const int nch = sh.f.nch;
        for (int q0 = 0; q0 < nch; q0 += 8) {
          float pv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) pv[u] = q0 + u < nch ? pin_b[(size_t)sh.f.ch[q0 + u] * m.N + k] : 0.f;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (q0 + u < nch) pin_b[(size_t)sh.f.ch[q0 + u] * m.N + k] = pv[u] + dI;
        }
      }
      // rows of the neurons that fired at t - 1 (the staged list and row
      // bounds): wave w takes rows w, w + waves, ..., lanes over the entries;
      // every entry is updated once per step
      if (t > 0) {
        const int nwv = blockDim.x / kWave, l = lane_id();
        for (int r = (int)(threadIdx.x / kWave); r < sh.f.nsp; r += nwv) {
          const int e1 = sh.f.rhi[r];
          for (int idx = sh.f.rlo[r] + l; idx < e1; idx += kWave) prec_b[idx] += sh.dI[m.indices[idx]];
        }
      }
      // (no barrier here: the next step's first barrier orders these reads
      // of sh before its writes)
    }
  }
}

__global__ void snn_reduce_k(const float* part, int B, size_t n, float* out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  // samples in order, eight loads in flight
  float s = 0.f;
  int b = 0;
  for (; b + 8 <= B; b += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(b + u) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < B; ++b) s += part[(size_t)b * n + i];
  out[i] = s;
}

// dW_out[k, o] = sum_b zsum[b, k] / T * dlog[b, o];  db_out[o] = sum_b dlog[b, o]
__global__ void snn_readout_grad_k(SnnDev m, const float* dlog, float* dW_out, float* db_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (dW_out && i < m.N * m.O) {
    const int k = i / m.O, o = i % m.O;
    float s = 0.f;
    int b = 0;
    for (; b + 8 <= m.B; b += 8) {  // samples in order, eight loads in flight
      float zv[8], dv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        zv[u] = m.zsum[(size_t)(b + u) * m.N + k];
        dv[u] = dlog[(size_t)(b + u) * m.O + o];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += zv[u] / (float)m.T * dv[u];
    }
    for (; b < m.B; ++b) s += m.zsum[(size_t)b * m.N + k] / (float)m.T * dlog[(size_t)b * m.O + o];
    dW_out[i] = s;
  }
  if (db_out && i < m.O) {
    float s = 0.f;
    for (int b = 0; b < m.B; ++b) s += dlog[(size_t)b * m.O + i];
    db_out[i] = s;
  }
}

static bp_status check_snn(const bp_snn* m) {
  BP_REQUIRE(m != nullptr, "null descriptor");
  BP_REQUIRE(m->B > 0 && m->C > 0 && m->N > 0 && m->O > 0 && m->T > 0, "sizes must be positive");
  BP_REQUIRE(m->N <= kSnnMaxN, "N must be <= %d", kSnnMaxN);
  BP_REQUIRE(m->C <= kSnnMaxC, "C must be <= %d", kSnnMaxC);
  BP_REQUIRE(m->O <= kSnnMaxO, "O must be <= %d", kSnnMaxO);
  BP_REQUIRE(m->nnz >= 0, "nnz must be >= 0");
  BP_REQUIRE(m->ckpt_every > 0, "ckpt_every must be > 0");
  BP_REQUIRE(m->surrogate == 0 || m->surrogate == 1, "surrogate must be 0 or 1");
  BP_REQUIRE(m->x && m->labels && m->W_in && m->indptr && m->W_out && m->b_out, "null input");
  BP_REQUIRE(m->nnz == 0 || (m->indices && m->w_rec), "null recurrent weights");
  return BP_OK;
}

static SnnDev snn_dev(const bp_snn* m, void* ckpt) {
  const SnnLayout L = snn_layout(m);
  SnnDev d{};
  d.B = m->B; d.C = m->C; d.N = m->N; d.O = m->O; d.T = m->T; d.nnz = m->nnz;
  d.surrogate = m->surrogate; d.detach = m->detach_reset; d.E = m->ckpt_every; d.nck = L.nck;
  d.alpha = m->alpha; d.beta = m->beta; d.omb = 1.0f - m->beta; d.theta = m->theta; d.slope = m->slope;
  d.relu_a = m->relu_a; d.relu_w = m->relu_width;
  d.x = m->x; d.labels = m->labels; d.W_in = m->W_in; d.indptr = m->indptr; d.indices = m->indices;
  d.w_rec = m->w_rec; d.W_out = m->W_out; d.b_out = m->b_out;
  char* c = (char*)ckpt;
  d.ckI = (float*)(c + L.off_I);
  d.ckV = (float*)(c + L.off_V);
  d.ckz = (uint8_t*)(c + L.off_z);
  d.zsum = (float*)(c + L.off_zsum);
  return d;
}

static int snn_threads(int N) { return ((N + kWave - 1) / kWave) * kWave; }

}  // namespace bp

using namespace bp;

extern "C" {

size_t bp_snn_ckpt_bytes(const bp_snn* m) {
  if (check_snn(m)) return 0;
  return snn_layout(m).ck_total;
}

size_t bp_snn_ws_bytes(const bp_snn* m) {
  if (check_snn(m)) return 0;
  return snn_layout(m).ws_total;
}

bp_status bp_snn_forward(const bp_snn* m, void* ckpt, float* logits, float* loss, uint8_t* raster, bp_stream stream) {
  bp_status s = check_snn(m);
  if (s) return s;
  BP_REQUIRE(ckpt && logits, "null output");
  hipStream_t st = as_stream(stream);
  const SnnDev d = snn_dev(m, ckpt);
  snn_forward_k<<<m->B, snn_threads(m->N), 0, st>>>(d, logits, raster);
  BP_LAUNCHED("snn_forward_k");
  if (loss) {
    snn_loss_k<<<1, 1024, 0, st>>>(d, logits, loss, nullptr);
    BP_LAUNCHED("snn_loss_k");
  }
  return BP_OK;
}

bp_status bp_snn_backward(const bp_snn* m, const void* ckpt, const float* logits, float* dW_in, float* dw_rec,
                          float* dW_out, float* db_out, void* ws, size_t ws_bytes, bp_stream stream) {
  bp_status s = check_snn(m);
  if (s) return s;
  BP_REQUIRE(ckpt && logits && ws, "null pointer");
  const SnnLayout L = snn_layout(m);
  BP_REQUIRE(ws_bytes >= L.ws_total, "workspace too small (%zu < %zu)", ws_bytes, L.ws_total);
  hipStream_t st = as_stream(stream);
  const SnnDev d = snn_dev(m, const_cast<void*>(ckpt));
  char* w = (char*)ws;
  float* dlog = (float*)(w + L.off_dlog);
  snn_loss_k<<<1, 1024, 0, st>>>(d, logits, nullptr, dlog);
  BP_LAUNCHED("snn_loss_k");
  float* pin = (float*)(w + L.off_pin);
  float* prec = (float*)(w + L.off_prec);
  int32_t* elli = (int32_t*)(w + L.off_elli);
  float* ellw = (float*)(w + L.off_ellw);
  snn_ell_k<<<(m->N + 255) / 256, 256, 0, st>>>(d, elli, ellw);
  BP_LAUNCHED("snn_ell_k");
  snn_backward_k<<<m->B, snn_threads(m->N), 0, st>>>(d, dlog, (float*)(w + L.off_segV), (uint8_t*)(w + L.off_segz),
                                                      pin, prec, elli, ellw);
  BP_LAUNCHED("snn_backward_k");
  if (dW_in) {
    const size_t n = (size_t)m->C * m->N;
    snn_reduce_k<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(pin, m->B, n, dW_in);
    BP_LAUNCHED("snn_reduce_k");
  }
  if (dw_rec && m->nnz > 0) {
    snn_reduce_k<<<(unsigned)((m->nnz + 255) / 256), 256, 0, st>>>(prec, m->B, (size_t)m->nnz, dw_rec);
    BP_LAUNCHED("snn_reduce_k");
  }
  if (dW_out || db_out) {
    const int n = m->N * m->O > m->O ? m->N * m->O : m->O;
    snn_readout_grad_k<<<(n + 255) / 256, 256, 0, st>>>(d, dlog, dW_out, db_out);
    BP_LAUNCHED("snn_readout_grad_k");
  }
  return BP_OK;
}

}  // extern "C"
