/*
 * proj.c -- plain CPU reference for synaptic projections with multi-step
 * delays (Section 4.3 and Appendix D: AlignPre and AlignPost projections;
 * Appendix E: the exponential synapse; Appendix F: synaptic delays).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): shares nothing with the GPU
 * library.
 *
 * A projection carries the spikes of a presynaptic group to a postsynaptic
 * group through a connectivity matrix M (rows presynaptic), `delay` steps
 * late: at step t it reads the presynaptic spikes s of step t - delay (none
 * before step 0).  Two exact forms:
 *   AlignPost: the synaptic variable lives on the postsynaptic side (n_post
 *     values): g <- g d + M^T s.  Exact for synapses whose dynamics are
 *     linear with one exponential (Appendix E: every arriving spike adds one
 *     to g, whichever neuron sent it).
 *   AlignPre: the synaptic variable lives on the presynaptic side (n_pre
 *     values), one trace per presynaptic neuron shared by all its synapses
 *     (Appendix D: homogeneous synapses driven by the same spike train have
 *     the same dynamics), and the postsynaptic input is g = M^T x.  Exact for
 *     any per-synapse dynamics; here the exponential synapse (x <- x d + s)
 *     and a saturating one (x <- x d, then x <- x + u (1 - x) on a spike).
 * For the exponential synapse the two coincide exactly (the map is linear):
 * that identity is one of the pins.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* out = the spikes of step t - delay, all zero before step 0. */
static const uint8_t* delayed(const uint8_t* raster, int32_t n_pre, int32_t t, int32_t delay) {
  return t - delay >= 0 ? raster + (size_t)(t - delay) * n_pre : NULL;
}

/* y[k] = sum over rows j with weight factor f[j] != 0 of M[j, k] f[j]
 * (M[j, k] = data or w), FP64. */
static void csr_tmul(const int32_t* indptr, const int32_t* indices, const float* data, double w, int32_t n_pre,
                     int32_t n_post, const double* f, double* y) {
  for (int32_t k = 0; k < n_post; ++k) y[k] = 0.0;
  for (int32_t j = 0; j < n_pre; ++j) {
    if (f[j] == 0.0) continue;
    for (int32_t e = indptr[j]; e < indptr[j + 1]; ++e) y[indices[e]] += (data ? (double)data[e] : w) * f[j];
  }
}

/* T steps of one projection driven by a presynaptic raster [T][n_pre] (FP64).
 * align 0 = AlignPost (state: g[n_post]), 1 = AlignPre (state: x[n_pre]);
 * syn 0 = exponential, 1 = saturating with increment u (AlignPre only).
 * g_out[t][k] receives the postsynaptic input of step t. */
void or_proj_run_f64(const int32_t* indptr, const int32_t* indices, const float* data, double w, int32_t n_pre,
                     int32_t n_post, int32_t align, int32_t syn, double decay, double u, int32_t delay, int32_t T,
                     const uint8_t* raster, double* state, double* g_out) {
  double* f = (double*)malloc(sizeof(double) * (size_t)(n_pre > 0 ? n_pre : 1));
  double* y = (double*)malloc(sizeof(double) * (size_t)(n_post > 0 ? n_post : 1));
  for (int32_t t = 0; t < T; ++t) {
    const uint8_t* s = delayed(raster, n_pre, t, delay);
    double* g = g_out + (size_t)t * n_post;
    if (align == 0) {
      for (int32_t j = 0; j < n_pre; ++j) f[j] = (s && s[j]) ? 1.0 : 0.0;
      csr_tmul(indptr, indices, data, w, n_pre, n_post, f, y);
      for (int32_t k = 0; k < n_post; ++k) state[k] = state[k] * decay + y[k];
      memcpy(g, state, sizeof(double) * (size_t)n_post);
    } else {
      for (int32_t j = 0; j < n_pre; ++j) {
        const int on = s && s[j];
        const double xp = state[j] * decay;
        state[j] = syn == 0 ? xp + (on ? 1.0 : 0.0) : (on ? xp + u * (1.0 - xp) : xp);
      }
      csr_tmul(indptr, indices, data, w, n_pre, n_post, state, g);
    }
  }
  free(f);
  free(y);
}

/* The same in FP32 with the library's order of operations for the state:
 *   AlignPost, homogeneous weights: y = (float)count * w, g = g * d + y;
 *   AlignPre: xp = x * d; x = xp + 1 (exponential) or xp + u * (1 - xp)
 *   (saturating) on a spike, else xp.
 * The FP32 state is what the library must reproduce bit for bit
 * (homogeneous AlignPost g, AlignPre x); g of AlignPre and of weighted
 * AlignPost is a sum of FP32 terms in an unspecified order (FP64 here). */
void or_proj_run_f32(const int32_t* indptr, const int32_t* indices, const float* data, float w, int32_t n_pre,
                     int32_t n_post, int32_t align, int32_t syn, float decay, float u, int32_t delay, int32_t T,
                     const uint8_t* raster, float* state, double* g_out) {
  double* f = (double*)malloc(sizeof(double) * (size_t)(n_pre > 0 ? n_pre : 1));
  double* y = (double*)malloc(sizeof(double) * (size_t)(n_post > 0 ? n_post : 1));
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_post > 0 ? n_post : 1));
  for (int32_t t = 0; t < T; ++t) {
    const uint8_t* s = delayed(raster, n_pre, t, delay);
    double* g = g_out + (size_t)t * n_post;
    if (align == 0) {
      if (!data) {
        for (int32_t k = 0; k < n_post; ++k) cnt[k] = 0;
        for (int32_t j = 0; j < n_pre; ++j)
          if (s && s[j])
            for (int32_t e = indptr[j]; e < indptr[j + 1]; ++e) cnt[indices[e]] += 1;
        for (int32_t k = 0; k < n_post; ++k) {
          const float yk = (float)cnt[k] * w;
          const float gd = state[k] * decay;
          state[k] = gd + yk;
        }
      } else {
        for (int32_t j = 0; j < n_pre; ++j) f[j] = (s && s[j]) ? 1.0 : 0.0;
        csr_tmul(indptr, indices, data, w, n_pre, n_post, f, y);
        for (int32_t k = 0; k < n_post; ++k) {
          const float gd = state[k] * decay;
          state[k] = gd + (float)y[k];
        }
      }
      for (int32_t k = 0; k < n_post; ++k) g[k] = state[k];
    } else {
      for (int32_t j = 0; j < n_pre; ++j) {
        const int on = s && s[j];
        const float xp = state[j] * decay;
        if (!on) {
          state[j] = xp;
        } else if (syn == 0) {
          state[j] = xp + 1.0f;
        } else {
          const float r = 1.0f - xp;
          const float inc = u * r;
          state[j] = xp + inc;
        }
        f[j] = (double)state[j];
      }
      csr_tmul(indptr, indices, data, w, n_pre, n_post, f, g);
    }
  }
  free(f);
  free(y);
  free(cnt);
}
