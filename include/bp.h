/*
 * bp.h -- C ABI of the MI355X (gfx950) event-driven spiking-network library.
 *
 * The operations follow "A differentiable brain simulator bridging brain
 * simulation and brain-inspired computing" (BrainPy, ICLR 2024):
 *   - event-driven CSR matrix-vector product       (Appendix B; Section 4.1)
 *   - just-in-time (JIT) connectivity matvec        (Appendix C; Sections 4.2, 5.2)
 *   - reverse mode of both operators                (Section 4.1)
 *   - the E/I balanced LIF network with conductance (COBA) or current (CUBA)
 *     synapses, exponential synapses merged per postsynaptic neuron
 *     (AlignPost) and a one-step spike delay       (Appendices E, F, N; Section 4.3)
 *   - a recurrent LIF network trained by BPTT with a surrogate spike
 *     derivative                                    (Section 5.3; Appendix I)
 *
 * Conventions for every call:
 *   - Pointers documented "device" are HIP device memory owned by the caller;
 *     the library never frees or retains them beyond the call, except that a
 *     network (bp_net) keeps using the workspace given to bp_create_net until
 *     bp_destroy_net.  Pointers documented "host" are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on that stream unless it says it synchronizes.
 *   - Return value: BP_OK (0) or a negative bp_status; bp_last_error() gives a
 *     thread-local message for the last failure.  No exception crosses the ABI.
 *     Argument errors are detected on the host before any launch.
 *   - Connectivity matrices have presynaptic rows and postsynaptic columns:
 *     shape (n_pre, n_post); the products compute y = M^T e (y has n_post
 *     entries).  Event vectors are uint8, any non-zero byte is a spike.
 */
#ifndef BP_H
#define BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bp_status;
#define BP_OK 0
#define BP_EINVAL (-1)       /* invalid argument (null pointer, bad size, p outside (0,1], ...) */
#define BP_ENOMEM (-2)       /* caller's workspace too small */
#define BP_EDEVICE (-3)      /* HIP runtime error (message holds hipGetErrorString) */
#define BP_ESTATE (-4)       /* object used in a wrong state (destroyed net, stalled kernel) */
#define BP_EUNSUPPORTED (-5) /* valid request the library does not support */

typedef void* bp_stream; /* hipStream_t */

const char* bp_last_error(void);
const char* bp_version(void);

/* ------------------------------------------------------------------------ */
/* Random source and connectivity rule                                      */
/* ------------------------------------------------------------------------ */

/* Weight kinds of a JIT matrix (Section 5.2 describes the matrix by four
 * scalars: probability, weight parameters and seed). */
#define BP_W_HOMO 0    /* every connection has weight w0 */
#define BP_W_NORMAL 1  /* w0 + w1 z, z standard normal (Box-Muller) */
#define BP_W_UNIFORM 2 /* w0 + (w1 - w0) u, u uniform on [0, 1) */

/* Random streams (the `stream` word of the Philox counter). */
#define BP_STREAM_CONN 1 /* connection positions */
#define BP_STREAM_W 2    /* JIT weights */
#define BP_STREAM_V0 3   /* initial membrane potentials */

/* K, the largest gap of the connectivity sampler (Appendix C: gaps uniform on
 * [1, floor(2/p - 1)] have mean 1/p).  Computed in FP64; a value within 1e-9
 * relative of an integer counts as that integer.  Returns K >= 1, or -1 for p
 * outside (0, 1]. */
int32_t bp_max_gap(double p);

/* out[i] = word (k[i] mod 4) of Philox-4x32-10 with key (seed low 32 bits,
 * seed high 32 bits) and counter (a[i], b[i], k[i] / 4, rng_stream): the
 * counter-based draw behind every random choice of the method, so that a
 * regenerated matrix is identical on every call (caption of the JIT listing,
 * Appendix C).  a, b, k, out: device arrays of n uint32.  n = 0 is a no-op. */
bp_status bp_hash(uint64_t seed, uint32_t rng_stream, const uint32_t* a, const uint32_t* b,
                  const uint32_t* k, uint32_t* out, int64_t n, bp_stream stream);

/* The fixed-probability connectivity of Appendix C, regenerated from a seed.
 * Row j, post block b (block width `block`; 0 = one block spanning the row):
 *   block == 0: first target = gap - 1, then one gap per further target,
 *               gaps uniform on [1, K], stop at n_post (the paper's sampler);
 *   block  > 0: restart at each block [b*block, min((b+1)*block, n_post));
 *               first target = block start + min(ra, rb), ra uniform on
 *               {0..K-1}, rb uniform on {0..K} (stationary start), then gaps.
 * Draw i of (j, b) is hash(seed, BP_STREAM_CONN, j, b, i). */
typedef struct {
  int32_t n_pre, n_post;
  int32_t max_gap; /* K from bp_max_gap(p), >= 1 (rule BP_RULE_UNIFORM) */
  int32_t block;   /* >= 0 */
  uint64_t seed;
  int32_t wkind;   /* BP_W_* (JIT products only) */
  float w0, w1;    /* weight parameters (see BP_W_*) */
  int32_t rule;    /* BP_RULE_*; 0 = the sampler above */
  float geo_inv_rate; /* BP_RULE_GEOMETRIC: bp_geo_inv_rate(p) */
  int32_t degree;  /* BP_RULE_FIXED_DEGREE: targets per row (block must be 0) */
} bp_jit_conn;

/* Exact-statistics alternatives to the uniform gaps (each defines its own
 * matrix for a seed; the products, the CSR build and the network treat every
 * rule alike):
 *   BP_RULE_GEOMETRIC: the exact Bernoulli(p) process named in Appendix C,
 *     gaps Geo[p] = 1 + floor(-ln(U) / -ln(1 - p)) with U = ((w >> 8) + 1)
 *     2^-24 from draw w of (j, b), the logarithm evaluated by a fixed
 *     sequence of FP32 operations (same gaps on every device); the first
 *     target of a block is its start plus gap - 1 (memoryless, so blocks keep
 *     the law), every later draw is one more gap.  Gaps are capped at 2^30.
 *   BP_RULE_FIXED_DEGREE: every row has exactly min(degree, n_post) distinct
 *     targets: target i is pi_j(i), pi_j a keyed permutation of [0, n_post)
 *     (four alternating Feistel rounds over the high b - b/2 and low b/2
 *     bits of [0, 2^b), 2^b the smallest power of two >= n_post (b >= 2),
 *     with MurmurHash3's 32-bit finalizer as round function, cycle-walked
 *     into [0, n_post); round keys the four words of Philox block
 *     (j, 0, 0, BP_STREAM_CONN)).  Targets are
 *     generated in index order; connection i of the JIT weight streams is
 *     target i.  One post block only (block == 0). */
#define BP_RULE_UNIFORM 0
#define BP_RULE_GEOMETRIC 1
#define BP_RULE_FIXED_DEGREE 2

/* 1 / (-ln(1 - p)) computed in FP64 and rounded once to FP32: the rate
 * parameter of BP_RULE_GEOMETRIC.  0 for p outside (0, 1) (p = 1: every
 * position is connected under a rate of 0). */
float bp_geo_inv_rate(double p);

/* ------------------------------------------------------------------------ */
/* Seeded CSR build (Appendix B storage of the Appendix C matrix)            */
/* ------------------------------------------------------------------------ */

/* indptr (device int32[n_pre + 1]) <- row pointers of the seeded matrix.
 * The caller reads indptr[n_pre] (= nnz, must stay below 2^31) to size
 * `indices`.  Rows come out strictly increasing, so each row adds at most one
 * to any column. */
bp_status bp_csr_count(const bp_jit_conn* c, int32_t* indptr, bp_stream stream);

/* indices (device int32[nnz]) <- column indices, given indptr from
 * bp_csr_count with the same descriptor. */
bp_status bp_csr_fill(const bp_jit_conn* c, const int32_t* indptr, int32_t* indices, bp_stream stream);

/* ------------------------------------------------------------------------ */
/* Spike compaction                                                          */
/* ------------------------------------------------------------------------ */

/* ids (device int32[n]) <- the positions j with s[j] != 0 in ascending order;
 * *count (device int32) <- how many.  Appendix B: event-driven work touches
 * only the rows whose event is true.  ws: device scratch of
 * bp_compact_ws_bytes(n) bytes. */
size_t bp_compact_ws_bytes(int32_t n);
bp_status bp_compact(const uint8_t* s, int32_t n, int32_t* ids, int32_t* count, void* ws, size_t ws_bytes,
                     bp_stream stream);

/* ------------------------------------------------------------------------ */
/* Event-driven CSR matvec (Appendix B) and its reverse mode (Section 4.1)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  const int32_t* indptr;  /* device int32[n_pre + 1] */
  const int32_t* indices; /* device int32[nnz], each in [0, n_post) */
  const float* data;      /* device float[nnz], or NULL: every entry is w */
  float w;                /* homogeneous weight (data == NULL) */
  int32_t n_pre, n_post;
  int32_t sorted;         /* 1 if every row's indices are strictly increasing
                             (true for bp_csr_fill output) */
  const int32_t* tile_ptr; /* optional device int32[n_pre][n_tiles + 1] from
                              bp_csr_tile_index, n_tiles = ceil(n_post /
                              tile_width): a speed hint for sorted rows with
                              n_post > 16384 (LDS tiles of tile_width columns,
                              each row's tile segment read from the index).
                              Without it sorted rows use equal tiles of at most
                              16384 columns and the kernel finds each row's
                              segment by a search of the row (same results).
                              Unsorted rows with n_post > 16384 (and unsorted
                              homogeneous rows split over several row chunks)
                              take a device-atomic kernel: integer counts stay
                              exact, FP32 sums are unordered as in every
                              weighted path. */
  int32_t tile_width;
} bp_csr;

/* Tile index of a sorted CSR: tile_ptr[j][t] = first position of row j whose
 * column is >= t * tile_width (tile_ptr[j][n_tiles] = end of row).
 * tile_width in [1, 16384]. */
bp_status bp_csr_tile_index(const int32_t* indptr, const int32_t* indices, int32_t n_pre, int32_t n_post,
                            int32_t tile_width, int32_t* tile_ptr, bp_stream stream);

/* y (device float[n_post], overwritten) = M^T e over the rows with a spike:
 * y[k] = sum over firing rows j of M[j, k].  Homogeneous weights are summed as
 * exact integer counts, then y[k] = w * count[k] (one FP32 rounding).
 * ws: device scratch of bp_event_csr_ws_bytes(m) bytes. */
size_t bp_event_csr_ws_bytes(const bp_csr* m);
bp_status bp_event_csr_matvec(const bp_csr* m, const uint8_t* events, float* y, void* ws, size_t ws_bytes,
                              bp_stream stream);

/* Batched form (Appendix B's product on a matrix of spike vectors, the
 * matrix-matrix member of the event-driven operator family of Section 4.2):
 * Y[b] = M^T E[b] for b < batch, E a device uint8 [batch][n_pre] with row
 * stride ev_stride >= n_pre bytes, Y a device float [batch][n_post] with row
 * stride y_stride >= n_post floats (rows overwritten; padding untouched).
 * Each firing row is streamed once per group of up to eight vectors and its
 * entries are added to every vector of the group that fires it, so a row
 * firing in several vectors costs one read.  Row b of Y equals
 * bp_event_csr_matvec of E[b] (homogeneous: exactly; data: up to FP32
 * summation order).  Rows must be strictly increasing (m->sorted;
 * BP_EUNSUPPORTED otherwise) and n_pre < 2^24.  A tile index whose width
 * leaves room for two vectors per group is used; otherwise tiles are found by
 * the in-kernel row search.  ws: bp_event_csr_matmat_ws_bytes(m, batch)
 * bytes of device scratch (0 when one row chunk covers the matrix).  Errors
 * (BP_EINVAL, before any launch): negative batch, strides below the vector
 * lengths, null E or Y with work to do, a short workspace.  batch == 0 is a
 * no-op. */
size_t bp_event_csr_matmat_ws_bytes(const bp_csr* m, int32_t batch);
bp_status bp_event_csr_matmat(const bp_csr* m, const uint8_t* events, int32_t batch, int64_t ev_stride, float* y,
                              int64_t y_stride, void* ws, size_t ws_bytes, bp_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bp_event_csr_matvec with no workspace argument, same kernels and results.
 * Its scratch (row-chunk partials, or the accumulators of the device-atomic
 * path) is a static device array of BP_STATIC_SCRATCH_BYTES inside the
 * library; each GPU the library runs on holds its own copy until the process
 * ends.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); the first call on a device looks up the array's address
 * there (with that device current) and caches it.  BP_EINVAL, before any
 * device work, when bp_event_csr_ws_bytes(m) exceeds BP_STATIC_SCRATCH_BYTES
 * (for sorted rows with a tile index, about n_post <= 60,000 x 32 row chunks
 * of FP32 partials; homogeneous weights need half).  Every call on one GPU
 * shares that GPU's array and leaves the last call's partials in it: calls
 * that overlap on one GPU (several streams or threads) race and must be
 * serialized by the caller.  Nothing in the array needs to start at zero. */
#define BP_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
bp_status bp_event_csr_matvec_noalloc(const bp_csr* m, const uint8_t* events, float* y, bp_stream stream);

/* Reverse mode of y = M^T e for an upstream gradient dy (device float[n_post]):
 *   d_events[j] = sum over row j of M[j,k] dy[k]            (every row)
 *   d_data[idx] = (e[j] != 0) * dy[indices[idx]]             (zero off firing rows)
 *   d_w[0]      = sum over firing rows of sum over the row of dy  (data == NULL)
 * Outputs (device) may each be NULL to skip; they are overwritten. */
bp_status bp_event_csr_backward(const bp_csr* m, const uint8_t* events, const float* dy, float* d_events,
                                float* d_data, float* d_w, bp_stream stream);

/* ------------------------------------------------------------------------ */
/* JIT connectivity matvec (Appendix C; Section 5.2) and reverse mode        */
/* ------------------------------------------------------------------------ */

/* y (device float[n_post], overwritten) = M^T e with M regenerated from
 * (seed, K, block, weights), never stored.  Homogeneous weights are summed as
 * exact integer counts.  ws: bp_jit_ws_bytes(c) bytes of device scratch. */
size_t bp_jit_ws_bytes(const bp_jit_conn* c);
bp_status bp_jit_conn_matvec(const bp_jit_conn* c, const uint8_t* events, float* y, void* ws, size_t ws_bytes,
                             bp_stream stream);

/* Batched JIT product on spike vectors: Y[b] = M^T E[b] with M regenerated
 * from (seed, K, block, weights), E and Y laid out as in bp_event_csr_matmat
 * (strided rows).  Each firing (row, block) is generated once per group of up
 * to eight vectors (fewer when weighted blocks are wider than 2048 columns or
 * homogeneous blocks wider than 4096) and its targets are added to every
 * vector of the group that fires the row.  Row b of Y equals
 * bp_jit_conn_matvec of E[b] (homogeneous: exactly; weighted: up to FP32
 * summation order).  n_pre < 2^24.  ws: bp_jit_conn_matmat_ws_bytes(c, batch)
 * bytes.  Errors as bp_event_csr_matmat. */
size_t bp_jit_conn_matmat_ws_bytes(const bp_jit_conn* c, int32_t batch);
bp_status bp_jit_conn_matmat(const bp_jit_conn* c, const uint8_t* events, int32_t batch, int64_t ev_stride, float* y,
                             int64_t y_stride, void* ws, size_t ws_bytes, bp_stream stream);

/* Float-vector form of the JIT product (Section 5.2's operator on a dense
 * vector): y (device float[n_post], overwritten) = J^T v, y[k] = sum over
 * rows j of v[j] * w_jk, for v a device float[n_pre] (16-byte aligned for the
 * vector loads; any alignment is accepted).  Rows with v[j] == 0 (either
 * sign) are skipped; NaN and infinities propagate.  The connectivity and
 * weights are those of bp_jit_conn_matvec for the same descriptor, so on a
 * 0/1 vector the two agree up to FP32 summation order.  Every product
 * v[j] * w_jk is rounded to FP32 and summed in FP32 in an unspecified order.
 * ws: bp_jit_dense_ws_bytes(c) bytes of device scratch (0 when one row chunk
 * covers the matrix).  Errors: BP_EINVAL on a null y, a null v with
 * n_pre > 0, a bad descriptor or a short workspace; nothing is launched. */
size_t bp_jit_dense_ws_bytes(const bp_jit_conn* c);
bp_status bp_jit_conn_matvec_dense(const bp_jit_conn* c, const float* v, float* y, void* ws, size_t ws_bytes,
                                   bp_stream stream);

/* Batched float-vector JIT product (Section 5.2's operator on m vectors at
 * once): Y = J^T X with X a device float[n_pre][m] and Y a device
 * float[n_post][m] (both row-major, Y overwritten); column c of Y is
 * bp_jit_conn_matvec_dense of column c of X up to FP32 summation order.
 * Every row is used (zero entries add zero); up to 8 columns of X share one
 * generation of each row.  n_post * m must fit in int32.  ws:
 * bp_jit_matmat_ws_bytes(c, m) bytes of device scratch.  Errors: BP_EINVAL
 * on a null Y, a null X with n_pre > 0, m < 0, a bad descriptor or a short
 * workspace; m == 0 launches nothing. */
size_t bp_jit_matmat_ws_bytes(const bp_jit_conn* c, int32_t m);
bp_status bp_jit_conn_matmat_dense(const bp_jit_conn* c, const float* X, int32_t m, float* Y, void* ws,
                                   size_t ws_bytes, bp_stream stream);

/* Stored CSR on a dense float vector: y (device float[n_post], overwritten)
 * = M^T v, y[k] = sum over rows j with v[j] != 0 of M[j, k] v[j] (M[j, k] =
 * data or w), each term rounded to FP32 and summed in an unspecified order
 * (the float-vector counterpart of bp_event_csr_matvec: the AlignPre
 * projection's product of its presynaptic traces, Appendix D).  Unsorted rows
 * need n_post <= 16384 (BP_EUNSUPPORTED otherwise).  ws:
 * bp_csr_matvec_dense_ws_bytes(m) bytes. */
size_t bp_csr_matvec_dense_ws_bytes(const bp_csr* m);
bp_status bp_csr_matvec_dense(const bp_csr* m, const float* v, float* y, void* ws, size_t ws_bytes,
                              bp_stream stream);

/* Reverse mode: d_events[j] = sum over row j of w_jk dy[k] (every row);
 * d_w (device float[2], nullable) = derivatives with respect to (w0, w1)
 * summed over firing rows: homogeneous (sum dy, 0); normal (sum dy, sum z dy);
 * uniform (sum (1-u) dy, sum u dy). */
bp_status bp_jit_conn_backward(const bp_jit_conn* c, const uint8_t* events, const float* dy, float* d_events,
                               float* d_w, bp_stream stream);

/* Generic form: op 0 = event CSR (args: const bp_csr*), op 1 = JIT
 * (args: const bp_jit_conn*; d_data unused). */
bp_status bp_backward(int32_t op, const void* args, const uint8_t* events, const float* dy, float* d_events,
                      float* d_data, float* d_w, bp_stream stream);

/* ------------------------------------------------------------------------ */
/* Projections with multi-step delays (Section 4.3; Appendices D, E, F)      */
/* ------------------------------------------------------------------------ */

/* A spike delay line: device uint8 [depth][n], slot t mod depth holds the
 * spikes of step t; the caller zeroes it before step 0 (steps before 0 then
 * read as silent).  bp_delay_push copies step t's spikes (device uint8[n])
 * into its slot (an asynchronous device copy). */
bp_status bp_delay_push(uint8_t* ring, int32_t depth, int32_t n, int64_t t, const uint8_t* spikes,
                        bp_stream stream);

#define BP_ALIGN_POST 0 /* synaptic variable per postsynaptic neuron: g <- g d + M^T s */
#define BP_ALIGN_PRE 1  /* trace per presynaptic neuron x, g = M^T x */
#define BP_SYN_EXP 0    /* x <- x d + s */
#define BP_SYN_SAT 1    /* x <- x d, then x <- x + u (1 - x) on a spike (AlignPre only) */

/* A projection from a presynaptic group (n_pre neurons, the rows of the
 * connectivity) to a postsynaptic group (n_post), reading the presynaptic
 * spikes `delay` steps late from a delay line.  AlignPost keeps n_post
 * synaptic variables (exact for the exponential synapse: every arriving
 * spike adds its weight, whichever neuron sent it, Appendix E); AlignPre
 * keeps one trace per presynaptic neuron, shared by all its synapses and by
 * every projection that reads it with the same delay and dynamics (Appendix
 * D), and is exact for any per-synapse dynamics.  For the exponential synapse
 * both give the same g. */
typedef struct {
  int32_t align;            /* BP_ALIGN_POST or BP_ALIGN_PRE */
  int32_t syn;              /* BP_SYN_EXP or BP_SYN_SAT */
  int32_t conn;             /* BP_CONN_CSR (csr) or BP_CONN_JIT (jit) */
  const bp_csr* csr;        /* stored connectivity: weight w or data */
  const bp_jit_conn* jit;   /* regenerated connectivity and weights */
  int32_t delay;            /* steps, 0 <= delay < depth of the delay line */
  float decay;              /* exp(-dt / tau), computed in FP64 and rounded once */
  float u;                  /* BP_SYN_SAT increment */
} bp_proj;

/* Device scratch of one step: n_post floats (AlignPost) plus the product's. */
size_t bp_proj_ws_bytes(const bp_proj* p);

/* Step t (>= 0) of the projection, reading ring slot (t - delay) mod depth
 * (nothing before step 0):
 *   AlignPost: state = g (device float[n_post]), g <- g d + M^T s, in FP32
 *     as fl(fl(g d) + y) with y the event product (homogeneous: (float)count
 *     * w, so g is bit-reproducible); `g` (nullable) receives a copy.
 *   AlignPre: state = x (device float[n_pre]), x <- fl(x d) (+ 1, or
 *     + fl(u fl(1 - fl(x d))) saturating) where the delayed spike is set; then
 *     g (device float[n_post], overwritten) = M^T x by the float-vector
 *     product (FP32 terms, unspecified order).
 * Errors: BP_EINVAL for a bad descriptor, a delay >= depth, null buffers or
 * a short workspace, before any launch. */
bp_status bp_proj_step(const bp_proj* p, const uint8_t* ring, int32_t depth, int64_t t, float* state, float* g,
                       void* ws, size_t ws_bytes, bp_stream stream);

/* T steps from step t0 driven by a presynaptic raster (device uint8
 * [T][n_pre]): for each step, bp_delay_push of its raster row, then
 * bp_proj_step writing g_out[i] (device float [T][n_post]). */
bp_status bp_proj_run(const bp_proj* p, const uint8_t* raster, int32_t T, uint8_t* ring, int32_t depth, int64_t t0,
                      float* state, float* g_out, void* ws, size_t ws_bytes, bp_stream stream);

/* ------------------------------------------------------------------------ */
/* E/I LIF network (Appendices E, F, N)                                       */
/* ------------------------------------------------------------------------ */

#define BP_COBA 0 /* I = ge (E_exc - V) + gi (E_inh - V) + I_ext */
#define BP_CUBA 1 /* I = ge + gi + I_ext */
#define BP_CONN_CSR 0 /* connectivity built once and stored */
#define BP_CONN_JIT 1 /* connectivity regenerated every step */

/* Neurons 0..n_exc-1 are excitatory, n_exc..n-1 inhibitory; one
 * fixed-probability matrix (bp_jit_conn rule with n_pre = n_post = n) connects
 * all of them.  Per step t, with the spikes s of step t-1 (one-step delay):
 *   ge = ge*exp(-dt/tau_e) + w_exc * #{firing excitatory rows reaching k}
 *   gi = gi*exp(-dt/tau_i) + w_inh * #{firing inhibitory rows reaching k}
 *   refractory neurons count down and do not spike; the others take one
 *   forward-Euler step V += (dt/tau_m)((v_rest - V) + r I) and spike when
 *   V > v_th (then V = v_reset, refractory for round(tau_ref/dt) steps).
 * All state arithmetic is FP32, each operation rounded in this order; the
 * decay and Euler constants are computed in FP64 and rounded once.
 * V0 = v0_lo + (v0_hi - v0_lo) u_k, u_k from hash(seed, BP_STREAM_V0, k, 0, 0). */
typedef struct {
  int32_t model;   /* BP_COBA or BP_CUBA */
  int32_t n, n_exc;
  int32_t conn;    /* BP_CONN_CSR or BP_CONN_JIT */
  int32_t max_gap; /* K */
  int32_t block;   /* generator block width (0 = whole row, the paper's
                      sequence).  Results do not depend on it beyond the
                      connectivity it defines; speed does: with JIT
                      connectivity and several workgroups, block 0 nets
                      exchange the targets of each spike, others the spike
                      ids (each reader regenerates its own blocks). */
  uint64_t seed;
  float w_exc, w_inh;
  float tau_m, tau_e, tau_i, tau_ref;
  float v_rest, v_th, v_reset, e_exc, e_inh, r, i_ext, dt;
  float v0_lo, v0_hi;
  int32_t max_wgs; /* upper bound on the workgroups the net runs on
                      (0 = default: one per compute unit, at most 160);
                      fewer lets more nets share the GPU in bp_run_batch */
  int32_t rule;    /* connectivity rule BP_RULE_* (as in bp_jit_conn) */
  float geo_inv_rate;
  int32_t degree;  /* BP_RULE_FIXED_DEGREE: exact out-degree (block 0) */
} bp_net_desc;

typedef struct bp_net_s* bp_net;

/* Workspace bytes a network needs (its admission cost in HBM).  For stored
 * connectivity this uses an upper bound on nnz (mean + 8 sd + 4096);
 * bp_create_net fails with BP_ENOMEM in the (improbable) case the real nnz
 * exceeds it. */
bp_status bp_net_bytes(const bp_net_desc* d, size_t* bytes);

/* Workgroups the network runs on (all of them resident at once during a
 * run; a batch of nets must fit the device together). */
bp_status bp_net_workgroups(const bp_net_desc* d, int32_t* n_wg);

/* Creates a network whose state, connectivity and scratch live in `ws`
 * (device, `bytes` >= bp_net_bytes; caller-owned, must outlive the net).
 * Builds the stored connectivity if any and the initial state.  Synchronizes
 * `stream` once (to read nnz).  *out receives a host handle. */
bp_status bp_create_net(const bp_net_desc* d, void* ws, size_t bytes, bp_stream stream, bp_net* out);

/* Advances the network by n_steps (>= 0) in one persistent-kernel launch.
 * i_ext_vec: device float[n] added to I_ext for these steps, or NULL.
 * raster: device uint8[n_steps * n] (row t = spikes of step t), or NULL.
 * counts: device int32[n_steps] (spikes per step), or NULL. */
bp_status bp_run(bp_net net, int64_t n_steps, const float* i_ext_vec, uint8_t* raster, int32_t* counts,
                 bp_stream stream);

/* One step; spikes (device uint8[n], nullable) receives its spikes. */
bp_status bp_step(bp_net net, const float* i_ext_vec, uint8_t* spikes, bp_stream stream);

/* Continuous batching: advances every net[i] by n_steps[i] (host int64,
 * >= 0) in one launch; nets run concurrently, each on its own workgroups,
 * results identical to bp_run per net.  counts (nullable, host array of
 * device pointers): counts[i] is int32[n_steps[i]] or NULL. */
bp_status bp_run_batch(const bp_net* nets, int32_t n_nets, const int64_t* n_steps, int32_t* const* counts,
                       bp_stream stream);

typedef struct {
  int32_t n, n_wg, wg_range; /* neurons, workgroups, neurons per workgroup */
  int64_t nnz;               /* stored synapses (0 for JIT) */
  int64_t step;              /* steps taken so far */
  size_t bytes_used;         /* workspace bytes in use */
  const uint64_t* events_dev; /* device uint64[n_wg]: synaptic events delivered
                                 by each workgroup since creation */
  const uint32_t* error_dev;  /* device word, non-zero if a kernel gave up waiting
                                 for another workgroup (the run stopped early) */
} bp_net_info;
bp_status bp_net_get_info(bp_net net, bp_net_info* info);

/* *dst (device uint64) <- synaptic events delivered since creation: the sum
 * over steps of the row lengths of the rows that fired the step before. */
bp_status bp_net_events(bp_net net, uint64_t* dst, bp_stream stream);

/* Checkpoint: the state is V, ge, gi (float[n] each), refractory counters
 * (int32[n]) and the last step's spikes (uint8[n]), packed in that order;
 * bp_state_bytes gives the size.  dst / src are device memory.  The step
 * counter is part of the host handle (bp_net_get_info / bp_set_state's step). */
size_t bp_state_bytes(bp_net net);
bp_status bp_get_state(bp_net net, void* dst, size_t bytes, bp_stream stream);
bp_status bp_set_state(bp_net net, const void* src, size_t bytes, int64_t step, bp_stream stream);

/* Releases the host handle (never the workspace).  The library keeps a table
 * of live handles: destroying a handle twice, or passing a destroyed or
 * foreign handle to any bp_* call, returns BP_ESTATE without reading the
 * freed handle.  Calls on one net must not race with its destruction. */
bp_status bp_destroy_net(bp_net net);

/* ------------------------------------------------------------------------ */
/* Recurrent LIF network trained by BPTT (Section 5.3; Appendix I)            */
/* ------------------------------------------------------------------------ */

/* Per sample b, t = 0..T-1, zero initial state:
 *   I_t = alpha I_{t-1} + x_t W_in + z_{t-1} W_rec   (W_rec a CSR, rows = pre)
 *   V_t = beta V_{t-1} (1 - z_{t-1}) + (1 - beta) I_t
 *   z_t = [V_t > theta]
 *   logits = (1/T) sum_t z_t W_out + b_out; loss = mean cross-entropy.
 * The reverse pass replaces dz/dV by a surrogate: sigmoid
 * slope*sig(slope x)(1 - sig(slope x)) or the ReLU form
 * max(0, relu_a (relu_width - |x|)), x = V - theta; detach_reset = 1 treats
 * (1 - z_{t-1}) as a constant. */
typedef struct {
  int32_t B, C, N, O, T;  /* batch, input channels, neurons (<= 1024), classes (<= 64), steps */
  int32_t nnz;            /* recurrent synapses (indptr[N]) */
  int32_t surrogate;    /* 0 sigmoid, 1 relu */
  int32_t detach_reset;
  int32_t ckpt_every;   /* checkpoint interval of the forward pass (> 0) */
  float alpha, beta, theta, slope, relu_a, relu_width;
  const uint8_t* x;       /* device uint8[T, B, C] input spikes */
  const int32_t* labels;  /* device int32[B] */
  const float* W_in;      /* device float[C, N] */
  const int32_t* indptr;  /* device int32[N + 1] */
  const int32_t* indices; /* device int32[nnz], rows strictly increasing */
  const float* w_rec;     /* device float[nnz] */
  const float* W_out;     /* device float[N, O] */
  const float* b_out;     /* device float[O] */
} bp_snn;

/* Checkpoint buffer bytes: ceil(T / ckpt_every) checkpoints of (I, V)
 * float[B, N] and z uint8[B, N] (the state before each segment) and the
 * spike counts float[B, N].  Written by
 * bp_snn_forward, read by bp_snn_backward. */
size_t bp_snn_ckpt_bytes(const bp_snn* m);
/* Scratch of the reverse pass: one segment of (V, z) per sample,
 * per-sample gradient partials (reduced in sample order, so the result does
 * not depend on scheduling) and a transposed copy of the recurrent rows
 * (2 x N x N words, rebuilt by every bp_snn_backward call). */
size_t bp_snn_ws_bytes(const bp_snn* m);

/* Forward pass: logits (device float[B, O]), loss (device float[1]),
 * checkpoints into ckpt (device, bp_snn_ckpt_bytes).  raster (nullable,
 * device uint8[T, B, N]) receives the spikes.  The recurrent input of each
 * neuron is summed over its firing presynaptic neurons in ascending order
 * (deterministic, so the reverse pass recomputes identical spikes). */
bp_status bp_snn_forward(const bp_snn* m, void* ckpt, float* logits, float* loss, uint8_t* raster,
                         bp_stream stream);

/* Reverse pass from the checkpoints: recomputes each segment forward, then
 * walks it backward.  Gradients (device, overwritten, nullable):
 * dW_in float[C, N], dw_rec float[nnz], dW_out float[N, O], db_out float[O].
 * logits are the forward's output; ws: bp_snn_ws_bytes bytes. */
bp_status bp_snn_backward(const bp_snn* m, const void* ckpt, const float* logits, float* dW_in, float* dw_rec,
                          float* dW_out, float* db_out, void* ws, size_t ws_bytes, bp_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BP_H */
