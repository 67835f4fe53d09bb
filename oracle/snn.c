/*
 * snn.c -- plain FP64 reference for the differentiable recurrent LIF network
 * trained by backpropagation through time with a surrogate spike derivative
 * (paper Section 4.1: every dedicated operator has a reverse mode; Section
 * 5.3 and Appendix I: BPTT with a surrogate gradient; the recurrent product
 * is the event-driven CSR operator of Appendix B).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Full-storage BPTT: every state of
 * every step is kept, no checkpointing, straightforward loops.
 *
 * Model, per sample b, t = 0..T-1, zero initial state:
 *   I_t = alpha I_{t-1} + x_t W_in + z_{t-1} W_rec      (W_rec: CSR rows = pre)
 *   V_t = beta V_{t-1} (1 - z_{t-1}) + (1 - beta) I_t
 *   z_t = H(V_t - theta)                    (smooth mode: S(V_t - theta), S the
 *                                            antiderivative of the surrogate)
 *   logits = (1/T) sum_t z_t W_out + b_out
 *   loss = (1/B) sum_b [ logsumexp(logits_b) - logits_b[label_b] ]
 * Surrogate dz/dV: sigmoid kind  s sig(s x)(1 - sig(s x)),  x = V - theta;
 *                  relu kind     max(0, a (width - |x|))      (Appendix I).
 * detach_reset = 1 treats the factor (1 - z_{t-1}) as a constant in the
 * reverse pass; 0 differentiates through it.
 *
 * Smooth mode makes the forward pass the function whose exact derivative the
 * surrogate is, so finite differences of the loss pin the reverse pass:
 *   sigmoid kind: S(x) = sig(s x), S'(x) = s sig(s x)(1 - sig(s x));
 *   relu kind:    S(x) = 0 for x <= -w, a (x + w)^2 / 2 for -w < x <= 0,
 *                 a w^2 - a (w - x)^2 / 2 for 0 < x <= w, a w^2 for x > w,
 *                 whose derivative is max(0, a (w - |x|)) (C^1, piecewise
 *                 quadratic).
 * A frozen reset (reset_in given) replaces the factor (1 - z_{t-1}) of step
 * t by reset_in[t]: the forward pass is then a function in which the reset
 * does not depend on the parameters, and its exact gradient is the
 * detached-reset gradient when reset_in holds the free run's factors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t B, C, N, O, T;
  int32_t surrogate;     /* 0 sigmoid, 1 relu */
  int32_t smooth;        /* 1: forward uses S, the surrogate's antiderivative */
  int32_t detach_reset;
  double alpha, beta, theta, slope, relu_a, relu_width;
} or_snn;

static double sig(double x) { return 1.0 / (1.0 + exp(-x)); }

/* S(x), the smooth spike function whose derivative is the surrogate. */
static double smooth_spike(const or_snn* P, double v) {
  double x = v - P->theta;
  if (P->surrogate == 1) {
    double a = P->relu_a, w = P->relu_width;
    if (x <= -w) return 0.0;
    if (x <= 0.0) return 0.5 * a * (x + w) * (x + w);
    if (x <= w) return a * w * w - 0.5 * a * (w - x) * (w - x);
    return a * w * w;
  }
  return sig(P->slope * x);
}

static double surrogate(const or_snn* P, double v) {
  double x = v - P->theta;
  if (P->surrogate == 1) {
    double r = P->relu_a * (P->relu_width - fabs(x));
    return r > 0.0 ? r : 0.0;
  }
  double s = sig(P->slope * x);
  return P->slope * s * (1.0 - s);
}

/* The smooth spike function S and the surrogate derivative at n membrane
 * values (for the tests of their shapes). */
void or_snn_spike_fns(const or_snn* P, const double* v, int64_t n, double* s_out, double* ds_out) {
  for (int64_t i = 0; i < n; ++i) {
    if (s_out) s_out[i] = smooth_spike(P, v[i]);
    if (ds_out) ds_out[i] = surrogate(P, v[i]);
  }
}

/*
 * x: uint8 [T, B, C]; labels: int32 [B]; W_in: [C, N]; CSR (indptr [N+1],
 * indices, w_rec [nnz]); W_out: [N, O]; b_out: [O].
 * z_force (nullable, uint8 [T, B, N]): when given, the spikes of the forward
 * pass are taken from it instead of from the threshold (teacher forcing with
 * another implementation's spike decisions; states are still recomputed).
 * reset_in (nullable, [T, B, N]): frozen reset factors (see above); entry t
 * multiplies V_{t-1} at step t (entry 0 is unused).
 * Outputs: loss, logits [B, O], z_out (nullable, [T, B, N] of the spikes used,
 * thresholded in hard mode), vmargin (nullable, [T, B, N]: V_t - theta, to
 * check another implementation's spike decisions), zval_out (nullable,
 * [T, B, N]: the spike values z_t themselves, fractional in smooth mode),
 * gradients (each nullable) with the shapes of the parameters.  Returns 0,
 * or -1 on allocation failure.
 */
int or_snn_grad(const or_snn* P, const uint8_t* x, const int32_t* labels, const double* W_in,
                const int32_t* indptr, const int32_t* indices, const double* w_rec,
                const double* W_out, const double* b_out, const uint8_t* z_force,
                const double* reset_in, double* loss, double* logits, uint8_t* z_out, double* vmargin,
                double* zval_out, double* dW_in, double* dw_rec, double* dW_out, double* db_out) {
  const int32_t B = P->B, C = P->C, N = P->N, O = P->O, T = P->T;
  const size_t TBN = (size_t)T * B * N;
  int32_t nnz = indptr[N];
  double* I = (double*)calloc(TBN, sizeof(double));
  double* V = (double*)calloc(TBN, sizeof(double));
  double* Z = (double*)calloc(TBN, sizeof(double));
  double* R = (double*)calloc(TBN, sizeof(double)); /* reset factor applied at step t */
  double* dI_next = (double*)calloc((size_t)B * N, sizeof(double));
  double* dV_next = (double*)calloc((size_t)B * N, sizeof(double));
  double* dI = (double*)calloc((size_t)B * N, sizeof(double));
  double* dV = (double*)calloc((size_t)B * N, sizeof(double));
  double* dz = (double*)calloc((size_t)B * N, sizeof(double));
  double* dlog = (double*)calloc((size_t)B * O, sizeof(double));
  double* zsum = (double*)calloc((size_t)B * N, sizeof(double));
  if (!I || !V || !Z || !R || !dI_next || !dV_next || !dI || !dV || !dz || !dlog || !zsum) return -1;

  /* forward */
  for (int32_t t = 0; t < T; ++t) {
    for (int32_t b = 0; b < B; ++b) {
      double* It = I + ((size_t)t * B + b) * N;
      double* Vt = V + ((size_t)t * B + b) * N;
      double* Zt = Z + ((size_t)t * B + b) * N;
      const double* Ip = t ? I + ((size_t)(t - 1) * B + b) * N : NULL;
      const double* Vp = t ? V + ((size_t)(t - 1) * B + b) * N : NULL;
      const double* Zp = t ? Z + ((size_t)(t - 1) * B + b) * N : NULL;
      const uint8_t* xt = x + ((size_t)t * B + b) * C;
      for (int32_t k = 0; k < N; ++k) It[k] = Ip ? P->alpha * Ip[k] : 0.0;
      for (int32_t c = 0; c < C; ++c)
        if (xt[c])
          for (int32_t k = 0; k < N; ++k) It[k] += W_in[(size_t)c * N + k];
      if (Zp)
        for (int32_t j = 0; j < N; ++j)
          if (Zp[j] != 0.0)
            for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx)
              It[indices[idx]] += Zp[j] * w_rec[idx];
      double* Rt = R + ((size_t)t * B + b) * N;
      for (int32_t k = 0; k < N; ++k) {
        if (Vp) Rt[k] = reset_in ? reset_in[((size_t)t * B + b) * N + k] : 1.0 - Zp[k];
        double vprev = Vp ? Vp[k] * Rt[k] : 0.0;
        Vt[k] = P->beta * vprev + (1.0 - P->beta) * It[k];
        double z;
        if (z_force) z = z_force[((size_t)t * B + b) * N + k] ? 1.0 : 0.0;
        else if (P->smooth) z = smooth_spike(P, Vt[k]);
        else z = Vt[k] > P->theta ? 1.0 : 0.0;
        Zt[k] = z;
        if (vmargin) vmargin[((size_t)t * B + b) * N + k] = Vt[k] - P->theta;
        if (zval_out) zval_out[((size_t)t * B + b) * N + k] = z;
        zsum[(size_t)b * N + k] += z;
        if (z_out) z_out[((size_t)t * B + b) * N + k] = (uint8_t)(z > 0.5);
      }
    }
  }
  /* readout and loss */
  double L = 0.0;
  for (int32_t b = 0; b < B; ++b) {
    double* lg = logits + (size_t)b * O;
    for (int32_t o = 0; o < O; ++o) {
      double acc = b_out[o];
      for (int32_t k = 0; k < N; ++k) acc += zsum[(size_t)b * N + k] / T * W_out[(size_t)k * O + o];
      lg[o] = acc;
    }
    double mx = lg[0];
    for (int32_t o = 1; o < O; ++o) if (lg[o] > mx) mx = lg[o];
    double se = 0.0;
    for (int32_t o = 0; o < O; ++o) se += exp(lg[o] - mx);
    double lse = mx + log(se);
    L += lse - lg[labels[b]];
    for (int32_t o = 0; o < O; ++o)
      dlog[(size_t)b * O + o] = (exp(lg[o] - lse) - (o == labels[b] ? 1.0 : 0.0)) / B;
  }
  *loss = L / B;

  if (dW_in) memset(dW_in, 0, sizeof(double) * (size_t)C * N);
  if (dw_rec) memset(dw_rec, 0, sizeof(double) * (size_t)nnz);
  if (dW_out) {
    for (int32_t k = 0; k < N; ++k)
      for (int32_t o = 0; o < O; ++o) {
        double acc = 0.0;
        for (int32_t b = 0; b < B; ++b) acc += zsum[(size_t)b * N + k] / T * dlog[(size_t)b * O + o];
        dW_out[(size_t)k * O + o] = acc;
      }
  }
  if (db_out)
    for (int32_t o = 0; o < O; ++o) {
      double acc = 0.0;
      for (int32_t b = 0; b < B; ++b) acc += dlog[(size_t)b * O + o];
      db_out[o] = acc;
    }

  /* reverse pass; dI_next / dV_next hold dL/dI_{t+1}, dL/dV_{t+1} */
  for (int32_t t = T - 1; t >= 0; --t) {
    for (int32_t b = 0; b < B; ++b) {
      const double* Vt = V + ((size_t)t * B + b) * N;
      const double* Rn = (t + 1 < T) ? R + ((size_t)(t + 1) * B + b) * N : NULL;
      double* dIn = dI_next + (size_t)b * N;
      double* dVn = dV_next + (size_t)b * N;
      double* dIt = dI + (size_t)b * N;
      double* dVt = dV + (size_t)b * N;
      double* dzt = dz + (size_t)b * N;
      /* dL/dz_t: readout + recurrent product into I_{t+1} + reset factor of V_{t+1} */
      for (int32_t j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int32_t o = 0; o < O; ++o) acc += W_out[(size_t)j * O + o] * dlog[(size_t)b * O + o];
        acc /= T;
        if (t + 1 < T) {
          for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) acc += w_rec[idx] * dIn[indices[idx]];
          if (!P->detach_reset) acc += dVn[j] * (-P->beta * Vt[j]);
        }
        dzt[j] = acc;
      }
      for (int32_t k = 0; k < N; ++k) {
        double g = dzt[k] * surrogate(P, Vt[k]);
        if (t + 1 < T) g += dVn[k] * P->beta * Rn[k];
        dVt[k] = g;
        dIt[k] = g * (1.0 - P->beta) + (t + 1 < T ? dIn[k] * P->alpha : 0.0);
      }
      /* parameter gradients of step t */
      const uint8_t* xt = x + ((size_t)t * B + b) * C;
      if (dW_in)
        for (int32_t c = 0; c < C; ++c)
          if (xt[c])
            for (int32_t k = 0; k < N; ++k) dW_in[(size_t)c * N + k] += dIt[k];
      if (dw_rec && t > 0) {
        const double* Zp = Z + ((size_t)(t - 1) * B + b) * N;
        for (int32_t j = 0; j < N; ++j)
          if (Zp[j] != 0.0)
            for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx)
              dw_rec[idx] += Zp[j] * dIt[indices[idx]];
      }
    }
    memcpy(dI_next, dI, sizeof(double) * (size_t)B * N);
    memcpy(dV_next, dV, sizeof(double) * (size_t)B * N);
  }
  free(I); free(V); free(Z); free(R); free(dI_next); free(dV_next); free(dI); free(dV); free(dz);
  free(dlog); free(zsum);
  return 0;
}

/*
 * Magnitude companion of or_snn_grad's reverse pass (a running error bound):
 * the same recursion with every sum replaced by the sum of the absolute
 * values of its terms, so that each output entry is the sum of |terms| that
 * reach that gradient entry through every path of the reverse pass.  An
 * implementation that carries the reverse pass in FP32 with the same spikes
 * differs from the FP64 gradient by a small multiple of its unit roundoff
 * times this sum per entry (the reverse recursion is contracting, alpha and
 * beta below one), which is what the per-entry parity tolerance is stated
 * against.  Spikes are taken from z_force (required); the outputs are
 * [C, N], [nnz], [N, O], [O] like the gradients.
 */
int or_snn_grad_abs(const or_snn* P, const uint8_t* x, const int32_t* labels, const double* W_in,
                    const int32_t* indptr, const int32_t* indices, const double* w_rec, const double* W_out,
                    const double* b_out, const uint8_t* z_force, double* aW_in, double* aw_rec, double* aW_out,
                    double* ab_out) {
  const int32_t B = P->B, C = P->C, N = P->N, O = P->O, T = P->T;
  const size_t TBN = (size_t)T * B * N;
  const int32_t nnz = indptr[N];
  double* I = (double*)calloc(TBN, sizeof(double));
  double* V = (double*)calloc(TBN, sizeof(double));
  double* Z = (double*)calloc(TBN, sizeof(double));
  double* dIn = (double*)calloc((size_t)B * N, sizeof(double));
  double* dVn = (double*)calloc((size_t)B * N, sizeof(double));
  double* dI = (double*)calloc((size_t)B * N, sizeof(double));
  double* dV = (double*)calloc((size_t)B * N, sizeof(double));
  double* dlog = (double*)calloc((size_t)B * O, sizeof(double));
  double* zsum = (double*)calloc((size_t)B * N, sizeof(double));
  if (!I || !V || !Z || !dIn || !dVn || !dI || !dV || !dlog || !zsum || !z_force) return -1;
  /* forward with the given spikes (the reset factor is 1 - z_{t-1}) */
  for (int32_t t = 0; t < T; ++t)
    for (int32_t b = 0; b < B; ++b) {
      double* It = I + ((size_t)t * B + b) * N;
      double* Vt = V + ((size_t)t * B + b) * N;
      double* Zt = Z + ((size_t)t * B + b) * N;
      const double* Ip = t ? I + ((size_t)(t - 1) * B + b) * N : NULL;
      const double* Vp = t ? V + ((size_t)(t - 1) * B + b) * N : NULL;
      const double* Zp = t ? Z + ((size_t)(t - 1) * B + b) * N : NULL;
      const uint8_t* xt = x + ((size_t)t * B + b) * C;
      for (int32_t k = 0; k < N; ++k) It[k] = Ip ? P->alpha * Ip[k] : 0.0;
      for (int32_t c = 0; c < C; ++c)
        if (xt[c])
          for (int32_t k = 0; k < N; ++k) It[k] += W_in[(size_t)c * N + k];
      if (Zp)
        for (int32_t j = 0; j < N; ++j)
          if (Zp[j] != 0.0)
            for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) It[indices[idx]] += w_rec[idx];
      for (int32_t k = 0; k < N; ++k) {
        const double vprev = Vp ? Vp[k] * (1.0 - Zp[k]) : 0.0;
        Vt[k] = P->beta * vprev + (1.0 - P->beta) * It[k];
        Zt[k] = z_force[((size_t)t * B + b) * N + k] ? 1.0 : 0.0;
        zsum[(size_t)b * N + k] += Zt[k];
      }
    }
  for (int32_t b = 0; b < B; ++b) {
    double lg[1024];
    double mx = -1e300;
    for (int32_t o = 0; o < O; ++o) {
      double acc = b_out[o];
      for (int32_t k = 0; k < N; ++k) acc += zsum[(size_t)b * N + k] / T * W_out[(size_t)k * O + o];
      lg[o] = acc;
      if (acc > mx) mx = acc;
    }
    double se = 0.0;
    for (int32_t o = 0; o < O; ++o) se += exp(lg[o] - mx);
    for (int32_t o = 0; o < O; ++o)
      dlog[(size_t)b * O + o] = fabs((exp(lg[o] - mx) / se - (o == labels[b] ? 1.0 : 0.0)) / B);
  }
  memset(aW_in, 0, sizeof(double) * (size_t)C * N);
  memset(aw_rec, 0, sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  for (int32_t k = 0; k < N; ++k)
    for (int32_t o = 0; o < O; ++o) {
      double acc = 0.0;
      for (int32_t b = 0; b < B; ++b) acc += zsum[(size_t)b * N + k] / T * dlog[(size_t)b * O + o];
      aW_out[(size_t)k * O + o] = acc;
    }
  for (int32_t o = 0; o < O; ++o) {
    double acc = 0.0;
    for (int32_t b = 0; b < B; ++b) acc += dlog[(size_t)b * O + o];
    ab_out[o] = acc;
  }
  for (int32_t t = T - 1; t >= 0; --t) {
    for (int32_t b = 0; b < B; ++b) {
      const double* Vt = V + ((size_t)t * B + b) * N;
      const double* Zt = Z + ((size_t)t * B + b) * N;
      double* dInb = dIn + (size_t)b * N;
      double* dVnb = dVn + (size_t)b * N;
      double* dIt = dI + (size_t)b * N;
      double* dVt = dV + (size_t)b * N;
      for (int32_t j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int32_t o = 0; o < O; ++o) acc += fabs(W_out[(size_t)j * O + o]) * dlog[(size_t)b * O + o];
        acc /= T;
        if (t + 1 < T) {
          for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) acc += fabs(w_rec[idx]) * dInb[indices[idx]];
          if (!P->detach_reset) acc += dVnb[j] * P->beta * fabs(Vt[j]);
        }
        const double g = acc * fabs(surrogate(P, Vt[j])) + (t + 1 < T ? dVnb[j] * P->beta * (1.0 - Zt[j]) : 0.0);
        dVt[j] = g;
        dIt[j] = g * (1.0 - P->beta) + (t + 1 < T ? dInb[j] * P->alpha : 0.0);
      }
      const uint8_t* xt = x + ((size_t)t * B + b) * C;
      for (int32_t c = 0; c < C; ++c)
        if (xt[c])
          for (int32_t k = 0; k < N; ++k) aW_in[(size_t)c * N + k] += dIt[k];
      if (t > 0) {
        const double* Zp = Z + ((size_t)(t - 1) * B + b) * N;
        for (int32_t j = 0; j < N; ++j)
          if (Zp[j] != 0.0)
            for (int32_t idx = indptr[j]; idx < indptr[j + 1]; ++idx) aw_rec[idx] += dIt[indices[idx]];
      }
    }
    memcpy(dIn, dI, sizeof(double) * (size_t)B * N);
    memcpy(dVn, dV, sizeof(double) * (size_t)B * N);
  }
  free(I); free(V); free(Z); free(dIn); free(dVn); free(dI); free(dV); free(dlog); free(zsum);
  return 0;
}
