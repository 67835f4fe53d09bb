// The E/I LIF network of Appendix N (LIF and conductance equations of
// Appendix F, exact exponential synapses of Appendix E merged per
// postsynaptic neuron as in the AlignPost projection of Section 4.3) with a
// one-step spike delay, run as one persistent kernel per call.
//
// Each workgroup owns a contiguous range of neurons: their V, ge, gi and
// refractory counters stay in registers for the whole launch.  One step:
//   1. gather the spikes of the previous step from every workgroup of the
//      net (see the record format below);
//   2. for every firing presynaptic row, accumulate the targets that fall in
//      the own range into LDS integer counters (excitatory and inhibitory
//      separately): stored CSR segments are streamed, JIT rows are
//      regenerated per post block from the seed;
//   3. update the own neurons (synaptic decay + input, COBA/CUBA current,
//      forward Euler, refractoriness, threshold, reset);
//   4. compact the own spikes (wave ballots, one LDS atomic per wave; the
//      list order carries no meaning) and publish them.
// Spike records: per workgroup and step parity an array of 64-bit slots,
// slot 0 = (tag, count), slot 1 + q = (tag, neuron id), tag = step + 1 in the
// high word; they hold the full lists (persistence, long lists).  The
// exchange itself goes through inboxes: every writer pushes a short line into
// a private inbox of every reader of the net, each 64-bit word tagged with
// the step (mod 16), so a reader accepts a word only when it carries the tag
// it waits for and the writer never waits for its stores to land.  Two lanes
// of the reader poll the two 16-byte halves of a line's first 32 bytes, so
// the payload arrives with the poll.  Spike-id lines carry the writer's spike
// count and its first 15 ids (longer lists are completed from the record).
// A one-workgroup net keeps its own list in LDS between steps.
// JIT nets of one post block (the paper's per-row sequence) exchange targets
// instead: the writer generates the whole row of each of its spikes (a wave
// per spike draws 256 gaps at once, one Philox call per lane, and places
// them by a wave prefix sum), sorts the targets by owning workgroup, and
// pushes up to 30 per line (13-bit entries, 14 in the polled 32 bytes); a
// line with more says so and the reader regenerates that writer's targets
// from its record.  Readers add the targets to their counters directly.
// Several nets run in one launch (continuous batching): the grid is the
// concatenation of their workgroup ranges and each net exchanges records only
// among its own workgroups.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <type_traits>
#include <unordered_set>

#include "bp_device.h"
#include "bp_host.h"

namespace bp {

constexpr int kNetThreads = 1024;
constexpr int kNetWaves = kNetThreads / kWave;
constexpr int kNPT = 4;                        // neurons per thread
constexpr int kRangeMax = kNetThreads * kNPT;  // neurons per workgroup
constexpr int kIdBatch = 4096;                 // firing rows staged per pass
constexpr int kMaxWgPerNet = 512;  // one gathering thread per source
constexpr int kTgtLine = 30;  // targets a line of the target exchange carries
constexpr int kInbox = 4;     // its polled words: 2 targets in word 0, 4 in each further word
constexpr int kExtra = 8;     // its further words: 2 targets each (targets 14..29)
constexpr int kLine = 4;      // words per inbox line of the spike-id exchange (32 bytes)
constexpr int kLineIds = 15;  // ids such a line carries: 3 in word 0, 4 in each of words 1..3
constexpr int kMaxBatch = 48;
constexpr int kDefaultWgs = 160;  // largest workgroup count of the default sizing (max_wgs == 0)
constexpr uint32_t kSpinLimit = 1u << 22;

struct NetDev {
  int32_t model, n, n_exc, conn, K, block, nb, ref_steps;
  uint64_t seed;
  int32_t rule, degree;  // connectivity rule (kRule*) and exact out-degree of rule 2
  float inv_rate;        // rule 1: 1 / -ln(1 - p)
  float w_exc, w_inh, de, di, a, v_rest, v_th, v_reset, e_exc, e_inh, r, i_ext;
  int32_t n_wg, range;
  int32_t push;  // several workgroups exchange targets (JIT, one post block), else spike ids
  int32_t ibw;   // words per inbox line: kInbox + kExtra (targets) or kLine (spike ids)
  float* V;
  float* ge;
  float* gi;
  int32_t* ref;
  const int32_t* indptr;
  const int32_t* indices;
  const int32_t* blkptr;  // [n][nb + 1] block index of the stored rows, or null
  uint64_t* rec;          // [2][n_wg][range + 1] spike records by step parity
  uint64_t* inbox;        // [2][n_wg dst][n_wg src][4] polled words of the lines pushed to each reader,
                          // then (target exchange) [2][n_wg dst][n_wg src][kExtra] further words
  unsigned long long* events;  // [n_wg] synaptic events delivered
  uint32_t* error;
};

struct NetLaunch {
  const NetDev* net;
  uint8_t* raster;
  int32_t* counts;
  const float* iext;
  int64_t t0;
  int32_t n_steps;
  int32_t wg_begin;
  int32_t n_wg;
  int32_t pad;
};

struct BatchArgs {
  int32_t n_nets;
  uint32_t spin_limit;
  NetLaunch e[kMaxBatch];
};

// input counters of the own neurons: excitatory at [k], inhibitory at
// [kRangeMax + k], so a target-line entry (12-bit local id, bit 12 set for an
// inhibitory source) is its own counter index
static_assert(kRangeMax == 0x1000, "target-line entries index the counters directly");
struct NetShared {
  uint32_t cnt[2 * kRangeMax];
  int ids[kIdBatch];
  int own[kRangeMax];  // own spikes of this step (order of the wave appends)
  int pref[kIdBatch + 1];
  int start[kIdBatch];
  int srcpref[kMaxWgPerNet + 1];
  int expref[kMaxWgPerNet + 1];
  int scan[2 * (kNetWaves + 1)];
  int ocnt[2];  // own spikes of the step, by step parity
  int abort_flag;
  // several workgroups: targets of the own spikes by destination workgroup
  uint16_t lst[kMaxWgPerNet][kTgtLine];  // local target id | 0x1000 if the source is inhibitory
  int dcnt[kMaxWgPerNet];
  int fb_src[kMaxWgPerNet];  // sources whose targets did not fit their inbox line
  int fb_cnt, fb_c, acnt;
  // neuron and synapse constants of the update, read from LDS there (as
  // scalars they would crowd the scalar registers of the whole step loop)
  alignas(16) float kc[12];
};

enum { kcWe, kcWi, kcDe, kcDi, kcIext, kcEe, kcEi, kcA, kcVrest, kcR, kcVth, kcVreset, kcCount };
static_assert(kcCount == 12, "the update reads the constants as three float4");

__device__ __forceinline__ uint64_t pack(uint32_t tag, uint32_t v) { return ((uint64_t)tag << 32) | v; }
__device__ __forceinline__ uint32_t tag_of(uint64_t s) { return (uint32_t)(s >> 32); }


__device__ __forceinline__ uint64_t* record(const NetDev& N, int par, int w) {
  return N.rec + ((size_t)par * N.n_wg + w) * (size_t)(N.range + 1);
}

// Word q of inbox line (par, dst, src): the 4 polled words of every line
// first (the lines a reader scans are contiguous), then the further words.
static_assert(kInbox == 4 && kLine == 4, "the polled part of a line is 4 words in both exchanges");
__device__ __forceinline__ uint64_t* iword(const NetDev& N, int par, int dst, int src, int q) {
  const size_t line = ((size_t)par * N.n_wg + dst) * N.n_wg + src;
  return q < 4 ? N.inbox + line * 4 + q : N.inbox + (size_t)2 * N.n_wg * N.n_wg * 4 + line * kExtra + (q - 4);
}

// Spike-id inbox line, 4 words of 64 bits, each written and read with its own
// tag so a reader can take the 16-byte halves as they land:
//   bits 63..60  tag: (step + 1) mod 16 of the step whose spikes it carries
//   bits 59..57  ids in this word
//   word 0: bits 56..44 the writer's spike count, bits 35..0 ids 0..2;
//   words 1..3: bits 47..0 ids 3..6, 7..10, 11..14
// Ids are local to the writer's range (12 bits; ranges hold at most 4096
// neurons) in the order of its record, which holds the ids beyond 15.
// Four-bit tags suffice: a reader waits for the tag of one step while the
// line holds that step's value or the one written two steps before.
__device__ __forceinline__ uint32_t tag4(uint64_t v) { return (uint32_t)(v >> 60); }
__device__ __forceinline__ int line_n(uint64_t v) { return (int)((v >> 57) & 7u); }
__device__ __forceinline__ int line_total(uint64_t v) { return (int)((v >> 44) & 0x1FFFu); }
__device__ __forceinline__ int line_first(int q) { return q == 0 ? 0 : 4 * q - 1; }
// Word q of a line; id(i) gives the writer's i-th spike (local id) and is
// called for every i < 15 whatever the count (it must stay in bounds).
template <class Id>
__device__ __forceinline__ uint64_t line_word(uint32_t tag, int q, int total, Id&& id) {
  const int first = line_first(q);
  const int n = max(0, min(min(total, kLineIds) - first, q == 0 ? 3 : 4));
  uint64_t v = ((uint64_t)(tag & 15u) << 60) | ((uint64_t)n << 57);
  if (q == 0) v |= (uint64_t)min(total, 0x1FFF) << 44;
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = (uint32_t)id(first + i);  // unconditional: the reads issue together
#pragma unroll
  for (int i = 0; i < 4; ++i)  // masked arithmetically, so no read moves into a branch
    v |= (uint64_t)(x[i] & (i < n ? 0xFFFu : 0u)) << (12 * i);
  return v;
}
// byte offset of the half h (words 2h, 2h + 1) of line (par, dst, src) in
// the first plane
__device__ __forceinline__ uint32_t line_off(const NetDev& N, int par, int dst, int src, int h) {
  return (uint32_t)(((((size_t)par * N.n_wg + dst) * N.n_wg + src) * kLine + 2 * h) * 8);
}
// Byte offset of further words 2 pq and 2 pq + 1 of target line (par, dst, src).
__device__ __forceinline__ uint32_t xline_off(const NetDev& N, int par, int dst, int src, int pq) {
  const size_t line = ((size_t)par * N.n_wg + dst) * N.n_wg + src;
  return (uint32_t)(((size_t)2 * N.n_wg * N.n_wg * 4 + line * kExtra + 2 * pq) * 8);
}
__device__ __forceinline__ uint32_t inbox_bytes(const NetDev& N) {
  return (uint32_t)(2 * (size_t)N.n_wg * N.n_wg * N.ibw * 8);
}

// Target inbox line (target exchange): 4 polled words, all written every step
// (two 16-byte halves), each carrying the 4-bit tag as above:
//   bits 63..60  tag, bits 59..57  entries in this word
//   word 0: bits 56..52 targets in the line (0..30; 31: more, the reader
//           regenerates them from the source's spike record), bits 51..39
//           the source's spike count, bits 25..0 entries 0..1;
//   words 1..3: bits 51..0 entries 4q - 2 .. 4q + 1 (targets up to 13);
// then up to kExtra further words, written only when the line needs them:
//   bits 63..32  the whole step tag, bits 27..26 entries in this word,
//   bits 25..0   entries 14 + 2 (q - 4) and the next.
// A further word can still hold a line of many steps earlier (it is not
// rewritten every step), so a 4-bit tag could match it before the new word
// lands; the whole tag cannot.
// An entry is 13 bits: local target id | 0x1000 if the source is inhibitory.
__device__ __forceinline__ int tline_tc(uint64_t v) { return (int)((v >> 52) & 31u); }
__device__ __forceinline__ int tline_spikes(uint64_t v) { return (int)((v >> 39) & 0x1FFFu); }
__device__ __forceinline__ int tline_first(int q) { return q == 0 ? 0 : 4 * q - 2; }
constexpr int kPolledTargets = 14;
// further words a line of ce targets needs
__device__ __forceinline__ int tline_extra(int ce) { return ce > kPolledTargets ? (ce - kPolledTargets + 1) / 2 : 0; }
constexpr uint64_t kNoTag = 0xFFFFFFFFull << 32;  // a further word no step can take
// Word q for c targets of which the line carries `ce` (c, or 0 if c > 30),
// from the entries x[i] = entry first(q) + i (unused ones may hold anything).
__device__ __forceinline__ uint64_t tline_pack(uint32_t tag, int q, int c, int ce, int spikes, const uint32_t (&x)[4]) {
  const int first = tline_first(q);
  const int n = max(0, min(ce - first, q == 0 ? 2 : 4));
  uint64_t v = ((uint64_t)(tag & 15u) << 60) | ((uint64_t)n << 57);
  if (q == 0) v |= ((uint64_t)(c > kTgtLine ? 31 : c) << 52) | ((uint64_t)min(spikes, 0x1FFF) << 39);
#pragma unroll
  for (int i = 0; i < 4; ++i) v |= (uint64_t)(x[i] & (i < n ? 0x1FFFu : 0u)) << (13 * i);
  return v;
}
// The same with the entries read through ent(i), called for i < 30 only.
template <class Ent>
__device__ __forceinline__ uint64_t tline_word(uint32_t tag, int q, int c, int ce, int spikes, Ent&& ent) {
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = ent(min(tline_first(q) + i, kTgtLine - 1));
  return tline_pack(tag, q, c, ce, spikes, x);
}

// Further word q (0-based) of a line of ce targets: entries 14 + 2q, 15 + 2q.
template <class Ent>
__device__ __forceinline__ uint64_t tline_xword(uint32_t tag, int q, int ce, Ent&& ent) {
  const int first = kPolledTargets + 2 * q;
  const int n = max(0, min(ce - first, 2));
  const uint32_t x0 = ent(min(first, kTgtLine - 1)) & (n > 0 ? 0x1FFFu : 0u);
  const uint32_t x1 = ent(min(first + 1, kTgtLine - 1)) & (n > 1 ? 0x1FFFu : 0u);
  return ((uint64_t)tag << 32) | ((uint64_t)n << 26) | ((uint64_t)x1 << 13) | x0;
}

// Load slot q of a record until it carries `tag` (bounded).
__device__ __forceinline__ uint64_t wait_slot(const uint64_t* r, int q, uint32_t tag, uint64_t first, uint32_t spin_limit,
                                              const NetDev& N, NetShared& sh) {
  uint64_t v = first;
  uint32_t spins = 0;
  while (tag_of(v) != tag) {
    if (++spins > spin_limit) {
      atomicOr(N.error, 1u);
      sh.abort_flag = 1;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    v = ld_coh64(&r[q]);
  }
  return v;
}

// Exclusive prefix sums of a and b over threads [0, nsrc) with one barrier
// (the other threads pass zeros and skip the wave scans); totals to all.
__device__ __forceinline__ void src_scan2(int a, int b, int nsrc, int* scratch, int* ea, int* eb, int* ta, int* tb) {
  const int l = lane_id(), w = threadIdx.x / kWave;
  const int nw = min((nsrc + kWave - 1) / kWave, kNetWaves);
  int ia = 0, ib = 0;
  if (w < nw) {
    ia = wave_incl_scan(a);
    ib = wave_incl_scan(b);
    if (l == kWave - 1) {
      scratch[w] = ia;
      scratch[kNetWaves + w] = ib;
    }
  }
  __syncthreads();
  // the (at most 16) wave sums in the first 16 lanes, scanned there (row
  // shifts), then read at the lanes of this wave and of the last wave
  int x = l < nw ? scratch[l] : 0, y = l < nw ? scratch[kNetWaves + l] : 0;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  y += __builtin_amdgcn_update_dpp(0, y, 0x111, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  y += __builtin_amdgcn_update_dpp(0, y, 0x112, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  y += __builtin_amdgcn_update_dpp(0, y, 0x114, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  y += __builtin_amdgcn_update_dpp(0, y, 0x118, 0xf, 0xf, false);
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int pa = wu > 0 ? __builtin_amdgcn_readlane(x, wu - 1) : 0;
  const int pb = wu > 0 ? __builtin_amdgcn_readlane(y, wu - 1) : 0;
  const int sa = __builtin_amdgcn_readlane(x, kNetWaves - 1), sb = __builtin_amdgcn_readlane(y, kNetWaves - 1);
  *ea = pa + ia - a;
  *eb = pb + ib - b;
  *ta = sa;
  *tb = sb;
}

// Gathers the spikes of the previous step (tagged `tag`, parity `par`) into
// sh.ids, in passes of kIdBatch; returns the total, calls `process(n)` for
// every pass of n ids.  Several workgroups: two lanes per source poll the
// two 16-byte halves of the source's line in the own inbox, which carry the
// spike count and the first 15 ids; longer lists are completed from the
// source's record.  One workgroup: the ids come from its own record.
template <class Process>
__device__ __forceinline__ int gather_and_process(const NetDev& N, int self, int par, uint32_t tag,
                                                  uint32_t spin_limit, NetShared& sh, Process&& process) {
  const int tid = threadIdx.x;
  const bool multi = N.n_wg > 1;
  const int src = multi ? tid >> 1 : 0, half = tid & 1;
  const bool poller = multi ? tid < 2 * N.n_wg : tid == 0;
  const bool carrier = poller && (!multi || half == 0);  // the lane that holds the source's count
  uint64_t wa = 0, wb = 0;
  int tot = 0;
  if (multi) {
    const __amdgpu_buffer_rsrc_t rs = coh_rsrc(N.inbox, inbox_bytes(N));
    const uint32_t t4 = tag & 15u;
    if (poller) {
      const uint32_t off = line_off(N, par, self, src, half);
      uint32_t spins = 0;
      while (true) {
        ld_coh128(rs, off, &wa, &wb);
        if (tag4(wa) == t4 && tag4(wb) == t4) break;
        if (++spins > spin_limit) {
          atomicOr(N.error, 1u);
          sh.abort_flag = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        __asm__ volatile("" ::: "memory");  // reload every pass
      }
      if (tag4(wa) != t4 || tag4(wb) != t4) wa = wb = 0;
      if (half == 0) tot = min(line_total(wa), N.range);
    }
  } else if (poller) {
    const uint64_t* r = record(N, par, 0);
    const uint64_t h = wait_slot(r, 0, tag, ld_coh64(&r[0]), spin_limit, N, sh);
    if (tag_of(h) == tag) tot = min((int)(uint32_t)h, N.range);
  }
  const int fx = multi ? kLineIds : 0;  // ids a source's line carries
  const int extra = max(0, tot - fx);
  int cpos, epos, A, E;
  src_scan2(tot, extra, multi ? 2 * N.n_wg : 1, sh.scan, &cpos, &epos, &A, &E);
  // the second lane of a pair: its prefix includes the first lane's count
  const int pair_tot = __builtin_amdgcn_update_dpp(0, tot, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  if (multi && half == 1) cpos -= pair_tot;
  if (sh.abort_flag) return -1;
  if (E > 0) {  // some list is longer than its line: per-source offsets for the record loads
    if (carrier) {
      sh.srcpref[src] = cpos;
      sh.expref[src] = epos;
    }
    if (tid == 0) {
      sh.srcpref[N.n_wg] = A;
      sh.expref[N.n_wg] = E;
    }
    __syncthreads();
  }
  const int32_t base = src * N.range;
  const int qa = half ? 7 : 0, qb = half ? 11 : 3;  // list positions of the lane's two words
  const int na = line_n(wa), nb = line_n(wb);
  for (int q0 = 0; q0 < A; q0 += kIdBatch) {
    const int n = min(kIdBatch, A - q0);
    if (na > 0) {  // lanes without ids skip the staging
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pa = cpos + qa + i - q0, pb = cpos + qb + i - q0;
        if (i < na && pa >= 0 && pa < n) sh.ids[pa] = base + (int32_t)((wa >> (12 * i)) & 0xFFFu);
        if (i < nb && pb >= 0 && pb < n) sh.ids[pb] = base + (int32_t)((wb >> (12 * i)) & 0xFFFu);
      }
    }
    // ids beyond a source's line (from its record), spread over the workgroup
    for (int e = tid; e < E; e += kNetThreads) {
      int l = 0, hh = N.n_wg;  // largest l with expref[l] <= e
      while (hh - l > 1) {
        const int m = (l + hh) >> 1;
        if (sh.expref[m] <= e) l = m; else hh = m;
      }
      const int q = fx + (e - sh.expref[l]);
      const int pos = sh.srcpref[l] + q - q0;
      const int cnt_l = sh.srcpref[l + 1] - sh.srcpref[l];
      if (pos >= 0 && pos < n && q < cnt_l && q < N.range) {
        const uint64_t* rr = record(N, par, l);
        const uint64_t x = wait_slot(rr, 1 + q, tag, ld_coh64(&rr[1 + q]), spin_limit, N, sh);
        sh.ids[pos] = (int)(uint32_t)x;
      }
    }
    __syncthreads();
    if (sh.abort_flag) return -1;
    process(n);
  }
  return A;
}

// One workgroup's run of L.n_steps steps of net N (CONN: stored CSR = 0,
// JIT = 1; specialised so each path keeps its own values in registers).
// PUSH (JIT nets of one post block, i.e. the paper's per-row sequence, with
// several workgroups): the writer generates the targets of its own spikes
// and pushes them to the inbox of the workgroup that owns them; otherwise
// the spike ids themselves are pushed and every reader regenerates (or
// streams) the part of each firing row inside its own range.
// RULES: nets of any connectivity rule; without it only the paper's uniform
// gaps are compiled in (the other rules' generators enlarge the kernel and
// raise its register pressure, so rule-0 launches use the lean variant).
template <int CONN, bool PUSH, bool RULES>
__device__ __forceinline__ void net_body(const NetLaunch& L, const NetDev& N, int w, uint32_t spin_limit,
                                         NetShared& sh) {
  const int tid = threadIdx.x, wave = tid / kWave;
  const int32_t lo = w * N.range;
  const int32_t hi = min(lo + N.range, N.n);
  const int32_t R = hi - lo;

  float V[kNPT], ge[kNPT], gi[kNPT];
  int32_t ref[kNPT];
#pragma unroll
  for (int i = 0; i < kNPT; ++i) {
    const int k = i * kNetThreads + tid;
    V[i] = ge[i] = gi[i] = 0.f;
    ref[i] = 0;
    if (k < R) {
      V[i] = N.V[lo + k];
      ge[i] = N.ge[lo + k];
      gi[i] = N.gi[lo + k];
      ref[i] = N.ref[lo + k];
    }
  }
  for (int k = tid; k < R; k += kNetThreads) {
    sh.cnt[k] = 0u;
    sh.cnt[kRangeMax + k] = 0u;
  }
  // one workgroup with stored rows (n <= kRangeMax): the row pointers staged
  // in LDS for the whole launch (sh.pref serves only the several-workgroup
  // row scan otherwise), so a firing row's bounds cost an LDS read, not a
  // cache round trip, every step
  static_assert(kIdBatch + 1 >= kRangeMax + 1, "row pointers of a one-workgroup net fit sh.pref");
  if (CONN == 0 && N.n_wg == 1)
    for (int k = tid; k <= N.n; k += kNetThreads) sh.pref[k] = as_global(N.indptr)[k];
  if (tid == 0) {
    sh.abort_flag = 0;
    sh.ocnt[0] = sh.ocnt[1] = 0;
    sh.fb_cnt = 0;
    sh.acnt = 0;
    sh.kc[kcWe] = N.w_exc;
    sh.kc[kcWi] = N.w_inh;
    sh.kc[kcDe] = N.de;
    sh.kc[kcDi] = N.di;
    sh.kc[kcIext] = N.i_ext;
    sh.kc[kcEe] = N.e_exc;
    sh.kc[kcEi] = N.e_inh;
    sh.kc[kcA] = N.a;
    sh.kc[kcVrest] = N.v_rest;
    sh.kc[kcR] = N.r;
    sh.kc[kcVth] = N.v_th;
    sh.kc[kcVreset] = N.v_reset;
  }
  __syncthreads();

  const int32_t B = N.block;
  const int32_t b_lo = B > 0 ? lo / B : 0;
  const int32_t b_hi = B > 0 ? (hi - 1) / B : 0;
  const int32_t nbt = b_hi - b_lo + 1;
  const uint64_t seed = N.seed;
  const uint32_t K = (uint32_t)N.K;
  unsigned long long ev_local = 0;

  // accumulate the targets of the staged firing rows sh.ids[0, nact)
  auto propagate = [&](int nact) {
    if constexpr (CONN == 1) {
      const int items = nact * nbt;
      for (int it = tid; it < items; it += kNetThreads) {
        const int ai = it / nbt;
        const uint32_t b = (uint32_t)(b_lo + it % nbt);
        const uint32_t j = (uint32_t)sh.ids[ai];
        if (j >= (uint32_t)N.n) continue;
        uint32_t* cnt = sh.cnt + ((int32_t)j < N.n_exc ? 0 : kRangeMax);
        auto add = [&](int32_t pos, uint32_t) {
          atomicAdd(&cnt[pos - lo], 1u);
          ++ev_local;
        };
        if constexpr (RULES) gen_block(ConnGen{seed, K, N.n, B, N.rule, N.inv_rate, N.degree}, j, b, lo, hi, add);
        else gen_block_uniform(seed, K, N.n, B, j, b, lo, hi, add);
      }
    } else if (N.n_wg == 1) {
      // one workgroup (every column is its own): wave w streams rows w,
      // w + 16, ... of the listed neurons, its lanes over the entries, two
      // loads per lane in flight; no scan of the row lengths
      for (int r = wave; r < nact; r += kNetWaves) {
        const int32_t j = sh.ids[r];
        if ((uint32_t)j >= (uint32_t)N.n) continue;
        const int32_t st = sh.pref[j], en = sh.pref[j + 1];
        uint32_t* cnt = sh.cnt + (j < N.n_exc ? 0 : kRangeMax);
        for (int32_t e0 = st; e0 < en; e0 += 2 * kWave) {
          const int32_t ea = e0 + lane_id(), eb = ea + kWave;
          const int32_t ca = ea < en ? as_global(N.indices)[ea] : -1;
          const int32_t cb = eb < en ? as_global(N.indices)[eb] : -1;
          if (ca >= lo && ca < hi) {
            atomicAdd(&cnt[ca - lo], 1u);
            ++ev_local;
          }
          if (cb >= lo && cb < hi) {
            atomicAdd(&cnt[cb - lo], 1u);
            ++ev_local;
          }
        }
      }
    } else {
      int total = 0;
      for (int base = 0; base < nact; base += kNetThreads) {
        const int i = base + tid;
        int st = 0, len = 0;
        if (i < nact && (uint32_t)sh.ids[i] < (uint32_t)N.n) {
          const int32_t j = sh.ids[i];
          if (N.blkptr) {
            const auto* bp = as_global(N.blkptr) + (size_t)j * (N.nb + 1);
            st = bp[b_lo];
            len = bp[b_hi + 1] - st;
          } else {
            int32_t l = as_global(N.indptr)[j], h = as_global(N.indptr)[j + 1];
            while (l < h) {
              const int32_t m = (l + h) >> 1;
              if (as_global(N.indices)[m] < lo) l = m + 1; else h = m;
            }
            st = l;
            h = as_global(N.indptr)[j + 1];
            while (l < h) {
              const int32_t m = (l + h) >> 1;
              if (as_global(N.indices)[m] < hi) l = m + 1; else h = m;
            }
            len = l - st;
          }
        }
        int tot;
        const int ex = block_excl_scan(len, sh.scan, &tot);
        if (i < nact) {
          sh.pref[i] = total + ex;
          sh.start[i] = st;
        }
        total += tot;
      }
      if (tid == 0) sh.pref[nact] = total;
      __syncthreads();
      const int per = (total + kNetWaves - 1) / kNetWaves;
      const int e0 = wave * per, e1 = min(e0 + per, total);
      if (e0 < e1) {
        int l = 0, h = nact;
        while (h - l > 1) {
          const int m = (l + h) >> 1;
          if (sh.pref[m] <= e0) l = m; else h = m;
        }
        int r = l;
        for (int ee = e0 + lane_id(); ee - lane_id() < e1; ee += kWave) {
          if (ee < e1) {
            while (r + 1 < nact && sh.pref[r + 1] <= ee) ++r;
            const int32_t col = as_global(N.indices)[sh.start[r] + (ee - sh.pref[r])];
            if (col >= lo && col < hi) {
              atomicAdd(&sh.cnt[(sh.ids[r] < N.n_exc ? 0 : kRangeMax) + col - lo], 1u);
              ++ev_local;
            }
          }
        }
      }
    }
    __syncthreads();
  };

  // ---- several workgroups: spikes travel as their targets ----
  // Reader: thread src polls the header of source src's inbox line, then
  // loads its target slots and adds them to the LDS counters at once; a
  // source with more targets than the line holds is handled afterwards from
  // its spike record (propagate over the own range).  Returns the spikes of
  // the previous step over all sources, -1 if a wait gave up.
  auto push_gather = [&](int par, uint32_t tag) -> int {
    const uint32_t t4 = tag & 15u;
    int sp = 0;  // spikes of the polled source (lanes h == 0)
    // add the entries of one target-line word to the counters (the writer
    // puts only targets inside the reader's range into its line; an entry
    // is at most 0x1FFF, inside the counters whatever it holds)
    auto apply = [&](uint64_t v, int nmax) {
      const int n = min(line_n(v), nmax);
      ev_local += (uint32_t)n;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < n) atomicAdd(&sh.cnt[(uint32_t)(v >> (13 * i)) & 0x1FFFu], 1u);
    };
    // add the entries of a further word
    auto apply_x = [&](uint64_t x) {
      const int n = (int)((x >> 26) & 3u);
      ev_local += (uint32_t)n;
      if (n > 0) atomicAdd(&sh.cnt[(uint32_t)x & 0x1FFFu], 1u);
      if (n > 1) atomicAdd(&sh.cnt[(uint32_t)(x >> 13) & 0x1FFFu], 1u);
    };
    if (tid < 2 * N.n_wg) {
      // two lanes per source: the two 16-byte halves of the polled words 0..3
      const int src = tid >> 1, h = tid & 1;
      const __amdgpu_buffer_rsrc_t rs = coh_rsrc(N.inbox, inbox_bytes(N));
      const uint32_t off = line_off(N, par, w, src, h);
      uint64_t wa = 0, wb = 0;
      uint32_t spins = 0;
      while (true) {
        ld_coh128(rs, off, &wa, &wb);
        if (tag4(wa) == t4 && tag4(wb) == t4) break;
        if (++spins > spin_limit) {
          atomicOr(N.error, 1u);
          sh.abort_flag = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        __asm__ volatile("" ::: "memory");  // reload every pass
      }
      if (tag4(wa) == t4 && tag4(wb) == t4) {
        apply(wa, h == 0 ? 2 : 4);
        apply(wb, 4);
        if (h == 0) {
          const int tc = tline_tc(wa);
          sp = tline_spikes(wa);
          if (tc == 31) {
            sh.fb_src[atomicAdd(&sh.fb_cnt, 1)] = src;
          } else if (tc > kPolledTargets) {  // the further words, each with the whole tag, in 16-byte pairs
            const int nx = tline_extra(tc), np = (nx + 1) / 2;
            uint64_t u[kExtra];
#pragma unroll
            for (int pq = 0; pq < kExtra / 2; ++pq) {
              u[2 * pq] = u[2 * pq + 1] = 0;
              if (pq < np) ld_coh128(rs, xline_off(N, par, w, src, pq), &u[2 * pq], &u[2 * pq + 1]);
            }
#pragma unroll
            for (int pq = 0; pq < kExtra / 2; ++pq) {
              if (pq < np) {
                uint64_t a = u[2 * pq], b = u[2 * pq + 1];
                const bool two = 2 * pq + 1 < nx;
                for (uint32_t spin = 0; (tag_of(a) != tag || (two && tag_of(b) != tag)) && spin <= spin_limit; ++spin) {
                  __builtin_amdgcn_s_sleep(1);
                  __asm__ volatile("" ::: "memory");  // reload every pass
                  ld_coh128(rs, xline_off(N, par, w, src, pq), &a, &b);
                }
                if (tag_of(a) == tag && (!two || tag_of(b) == tag)) {
                  apply_x(a);
                  if (two) apply_x(b);
                } else {
                  atomicOr(N.error, 1u);
                  sh.abort_flag = 1;
                }
              }
            }
          }
        }
      }
    }
    // the step's spike count is reported by workgroup 0 only: one LDS atomic
    // per wave after a DPP sum (no same-address atomics across the lanes)
    if (w == 0 && L.counts) {
      const int tot = wave_incl_scan(sp);
      if (lane_id() == kWave - 1 && tot != 0) atomicAdd(&sh.acnt, tot);
    }
    __syncthreads();
    if (sh.abort_flag) return -1;
    const int A = sh.acnt;
    const int fb = sh.fb_cnt;
    for (int f = 0; f < fb; ++f) {
      const int src = sh.fb_src[f];
      const uint64_t* rr = record(N, par, src);
      if (tid == 0) {
        const uint64_t hh = wait_slot(rr, 0, tag, ld_coh64(&rr[0]), spin_limit, N, sh);
        sh.fb_c = tag_of(hh) == tag ? min((int)(uint32_t)hh, N.range) : 0;
      }
      __syncthreads();
      if (sh.abort_flag) return -1;
      const int c = sh.fb_c;
      for (int q0 = 0; q0 < c; q0 += kIdBatch) {
        const int n = min(kIdBatch, c - q0);
        for (int q = tid; q < n; q += kNetThreads) {
          const uint64_t x = wait_slot(rr, 1 + q0 + q, tag, ld_coh64(&rr[1 + q0 + q]), spin_limit, N, sh);
          sh.ids[q] = tag_of(x) == tag ? (int)(uint32_t)x : -1;
        }
        __syncthreads();
        if (sh.abort_flag) return -1;
        propagate(n);
      }
      __syncthreads();
    }
    return A;
  };

  // Writer: the targets of the own spikes sh.own[0, total), sorted into
  // per-destination lists (LDS).  JIT rows are generated whole: with one
  // block (the paper's sequence) one wave per spike draws 256 gaps per pass
  // (a Philox call per lane) and places them by a wave prefix sum; with post
  // blocks one lane per (spike, block).  Stored rows are streamed by a wave.
  const float inv_range = 1.0f / (float)N.range;
  auto emit = [&](int32_t pos, uint32_t inh) {
    if ((uint32_t)pos >= (uint32_t)N.n) return;
    // the FP32 quotient is off by at most one workgroup; corrected by selects
    int d = (int)((float)pos * inv_range);
    int loc = pos - d * N.range;
    d = loc < 0 ? d - 1 : (loc >= N.range ? d + 1 : d);
    loc = loc < 0 ? loc + N.range : (loc >= N.range ? loc - N.range : loc);
    const int slot = atomicAdd(&sh.dcnt[d], 1);
    if (slot < kTgtLine) sh.lst[d][slot] = (uint16_t)((uint32_t)loc | inh);
  };
  // The same for a lane's four consecutive targets of a gap walk: the four
  // destination counters are incremented back to back (one LDS round trip
  // instead of four), then the entries stored.
  auto emit4 = [&](int32_t p0, int32_t p1, int32_t p2, int32_t p3, uint32_t inh) {
    const int32_t pp[4] = {p0, p1, p2, p3};
    int dd[4], ll[4], ss[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int d = (int)((float)pp[u] * inv_range);
      int loc = pp[u] - d * N.range;
      dd[u] = loc < 0 ? d - 1 : (loc >= N.range ? d + 1 : d);
      ll[u] = loc < 0 ? loc + N.range : (loc >= N.range ? loc - N.range : loc);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) ss[u] = (uint32_t)pp[u] < (uint32_t)N.n ? atomicAdd(&sh.dcnt[dd[u]], 1) : kTgtLine;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ss[u] < kTgtLine) sh.lst[dd[u]][ss[u]] = (uint16_t)((uint32_t)ll[u] | inh);
  };
  auto push_generate = [&](int total) {
    const int lane = lane_id();
    if constexpr (CONN == 1) {
      if constexpr (!RULES) {
        if (B == 0) {
          const uint32_t cap = (uint32_t)N.n;
          for (int si = wave; si < total; si += kNetWaves) {
            const uint32_t j = (uint32_t)sh.own[si];
            const uint32_t inh = (int32_t)j >= N.n_exc ? 0x1000u : 0u;
            int32_t base = 0;
            for (uint32_t c = 0;; ++c) {
              const uint32_t blk = c * kWave + (uint32_t)lane;
              const Words4 q = philox10(j, 0u, blk, kStreamConn, (uint32_t)seed, (uint32_t)(seed >> 32));
              // draw 0 is the first position itself, later draws are gaps 1 + U[0, K);
              // a gap beyond n ends the row, so gaps are clipped to n
              const uint32_t g0 = min(below(q.x, K) + (blk != 0u ? 1u : 0u), cap);
              const uint32_t g1 = min(1u + below(q.y, K), cap);
              const uint32_t g2 = min(1u + below(q.z, K), cap);
              const uint32_t g3 = min(1u + below(q.w, K), cap);
              const int s4 = (int)(g0 + g1 + g2 + g3);
              const int incl = wave_incl_scan(s4);
              const int32_t p = base + incl - s4 + (int32_t)g0;
              emit4(p, p + (int32_t)g1, p + (int32_t)(g1 + g2), p + (int32_t)(g1 + g2 + g3), inh);
              base += __builtin_amdgcn_readlane(incl, kWave - 1);
              if (base >= N.n) break;
            }
          }
        } else {
          const int items = total * N.nb;
          for (int it = tid; it < items; it += kNetThreads) {
            const int si = it / N.nb;
            const uint32_t b = (uint32_t)(it - si * N.nb);
            const uint32_t j = (uint32_t)sh.own[si];
            const uint32_t inh = (int32_t)j >= N.n_exc ? 0x1000u : 0u;
            auto put = [&](int32_t pos, uint32_t) { emit(pos, inh); };
            gen_block_uniform(seed, K, N.n, B, j, b, 0, N.n, put);
          }
        }
      } else {
        if (B == 0 && N.rule == kRuleFixedDegree) {
          // exactly `degree` targets per spike: lane l computes targets
          // l, l + 64, ... of the row's permutation
          const uint32_t fb = fd_bits(N.n);
          const int32_t k = N.degree < N.n ? N.degree : N.n;
          for (int si = wave; si < total; si += kNetWaves) {
            const uint32_t j = (uint32_t)sh.own[si];
            const uint32_t inh = (int32_t)j >= N.n_exc ? 0x1000u : 0u;
            const Words4 key = fd_keys(seed, j);
            for (int32_t i = lane; i < k; i += kWave) emit((int32_t)fd_target(key, fb, N.n, (uint32_t)i), inh);
          }
        } else if (B == 0) {
          // one wave per spike, gaps uniform or geometric (the law chosen
          // outside the loop)
          const uint32_t cap = (uint32_t)N.n;
          const float inv_rate = N.inv_rate;
          auto rows = [&](auto geo_tag) {
            constexpr bool kGeo = decltype(geo_tag)::value;
            auto gap = [&](uint32_t w) { return kGeo ? geo_gap(w, inv_rate) : 1u + below(w, K); };
            for (int si = wave; si < total; si += kNetWaves) {
              const uint32_t j = (uint32_t)sh.own[si];
              const uint32_t inh = (int32_t)j >= N.n_exc ? 0x1000u : 0u;
              int32_t base = 0;
              for (uint32_t c = 0;; ++c) {
                const uint32_t blk = c * kWave + (uint32_t)lane;
                const Words4 q = philox10(j, 0u, blk, kStreamConn, (uint32_t)seed, (uint32_t)(seed >> 32));
                // draw 0 is the first position itself (gap - 1), later draws are
                // gaps; a gap beyond n ends the row, so gaps are clipped to n
                const uint32_t g0 = min(gap(q.x) - (blk == 0u ? 1u : 0u), cap);
                const uint32_t g1 = min(gap(q.y), cap);
                const uint32_t g2 = min(gap(q.z), cap);
                const uint32_t g3 = min(gap(q.w), cap);
                const int s4 = (int)(g0 + g1 + g2 + g3);
                const int incl = wave_incl_scan(s4);
                const int32_t p = base + incl - s4 + (int32_t)g0;
                emit4(p, p + (int32_t)g1, p + (int32_t)(g1 + g2), p + (int32_t)(g1 + g2 + g3), inh);
                base += __builtin_amdgcn_readlane(incl, kWave - 1);
                if (base >= N.n) break;
              }
            }
          };
          if (N.rule == kRuleGeometric) rows(std::true_type{});
          else rows(std::false_type{});
        } else {
          const int items = total * N.nb;
          for (int it = tid; it < items; it += kNetThreads) {
            const int si = it / N.nb;
            const uint32_t b = (uint32_t)(it - si * N.nb);
            const uint32_t j = (uint32_t)sh.own[si];
            const uint32_t inh = (int32_t)j >= N.n_exc ? 0x1000u : 0u;
            auto put = [&](int32_t pos, uint32_t) { emit(pos, inh); };
            gen_block(ConnGen{seed, K, N.n, B, N.rule, N.inv_rate, N.degree}, j, b, 0, N.n, put);
          }
        }
      }
    } else {
      for (int si = wave; si < total; si += kNetWaves) {
        const int32_t j = sh.own[si];
        const uint32_t inh = j >= N.n_exc ? 0x1000u : 0u;
        const int32_t e0 = as_global(N.indptr)[j], e1 = as_global(N.indptr)[j + 1];
        for (int32_t e = e0 + lane; e < e1; e += kWave) emit(as_global(N.indices)[e], inh);
      }
    }
  };

  // Writer: the two polled halves of every destination's inbox line (the
  // signal its reader polls; every word carries the tag), then the further
  // words of a line with more than 14 targets.
  auto push_publish = [&](int par, uint32_t tag, int total) {
    const __amdgpu_buffer_rsrc_t rs = coh_rsrc(N.inbox, inbox_bytes(N));
    for (int x = tid; x < 2 * N.n_wg; x += kNetThreads) {
      const int d = x >> 1, h = x & 1;
      // the half's entries read before the line's count (both LDS reads in
      // flight together; entries past the count are masked)
      uint32_t xa[4], xb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        xa[i] = sh.lst[d][tline_first(2 * h) + i];
        xb[i] = sh.lst[d][tline_first(2 * h + 1) + i];
      }
      const int c = sh.dcnt[d];
      const int ce = c > kTgtLine ? 0 : c;
      auto ent = [&](int i) { return (uint32_t)sh.lst[d][i]; };
      const uint64_t wa = tline_pack(tag, 2 * h, c, ce, total, xa);
      const uint64_t wb = tline_pack(tag, 2 * h + 1, c, ce, total, xb);
      st_coh128(rs, line_off(N, par, d, w, h), wa, wb);
      if (h == 0) {
        const int nx = tline_extra(ce);
        for (int pq = 0; 2 * pq < nx; ++pq)
          st_coh128(rs, xline_off(N, par, d, w, pq), tline_xword(tag, 2 * pq, ce, ent),
                    tline_xword(tag, 2 * pq + 1, ce, ent));
      }
    }
  };

  int nloc = -1;  // one workgroup: own spikes of the last step kept in sh.ids, -1 if not
  for (int32_t s = 0; s < L.n_steps; ++s) {
    const int64_t t = L.t0 + s;
    const int pin = (int)((t + 1) & 1);  // parity of step t-1
    const int pout = (int)(t & 1);
    int A;
    if constexpr (!PUSH) {
      // clear the own counters read by the last update (each thread its own
      // neurons; the gather below passes a barrier before any accumulation)
#pragma unroll
      for (int i = 0; i < kNPT; ++i) {
        const int k = i * kNetThreads + tid;
        if (k < R) {
          sh.cnt[k] = 0u;
          sh.cnt[kRangeMax + k] = 0u;
        }
      }
    }
    if (PUSH && N.n_wg > 1) {
      A = push_gather(pin, (uint32_t)t);
      if (A < 0) break;
      for (int d = tid; d < N.n_wg; d += kNetThreads) sh.dcnt[d] = 0;
    } else if (nloc >= 0) {
      A = nloc;  // own list of the last step, still in LDS
      __syncthreads();  // counters cleared
      if (A > 0) propagate(A);
    } else {
      A = gather_and_process(N, w, pin, (uint32_t)t, spin_limit, sh, propagate);
      if (A < 0) break;
    }
    // (every path above passed a barrier after the previous step's readers
    // of the next step's spike counter)
    if (tid == 0) sh.ocnt[(t + 1) & 1] = 0;
    if (w == 0 && tid == 0 && L.counts && s > 0) as_global(L.counts)[s - 1] = A;

    // neuron update: exactly the oracle's FP32 operation order
    uint32_t sbits = 0;
    const float* iext = L.iext;
    uint32_t ce[kNPT], ci[kNPT];
#pragma unroll
    for (int i = 0; i < kNPT; ++i) {
      const int k = i * kNetThreads + tid;
      // k < kRangeMax: always inside the arrays, so the accesses need no
      // guard (a guarded access is a branch and a wait of its own); values
      // for k >= R are never used
      if constexpr (PUSH) {  // read and clear in one LDS exchange (the next gather adds at once)
        ce[i] = atomicExch(&sh.cnt[k], 0u);
        ci[i] = atomicExch(&sh.cnt[kRangeMax + k], 0u);
      } else {  // cleared at the start of the next step
        ce[i] = sh.cnt[k];
        ci[i] = sh.cnt[kRangeMax + k];
      }
    }
    // (the model and the optional inputs and outputs are fixed for the whole
    // launch: the common case, COBA without external current or raster, is
    // compiled with them as constants)
    auto update = [&](auto coba, auto has_iext, auto has_raster) {
      // the constants read once per step, before the slots (read inside the
      // slots' conditional blocks they were reloaded in every slot, five LDS
      // round trips in sequence each)
      const float4 c0 = reinterpret_cast<const float4*>(sh.kc)[0];
      const float4 c1 = reinterpret_cast<const float4*>(sh.kc)[1];
      const float4 c2 = reinterpret_cast<const float4*>(sh.kc)[2];
      const float kWe = c0.x, kWi = c0.y, kDe = c0.z, kDi = c0.w, kIext = c1.x, kEe = c1.y, kEi = c1.z,
                  kA = c1.w, kVrest = c2.x, kR = c2.y, kVth = c2.z, kVreset = c2.w;
#pragma unroll
      for (int i = 0; i < kNPT; ++i) {
        const int k = i * kNetThreads + tid;
        if (k < R) {
          const float xe = (float)ce[i] * kWe;
          const float xi = (float)ci[i] * kWi;
          ge[i] = ge[i] * kDe + xe;
          gi[i] = gi[i] * kDi + xi;
          bool spk = false;
          if (ref[i] > 0) {
            ref[i] -= 1;
          } else {
            float ix = kIext;
            if (has_iext) ix = ix + as_global(iext)[lo + k];
            float I;
            if (coba) I = ge[i] * (kEe - V[i]) + gi[i] * (kEi - V[i]) + ix;
            else I = ge[i] + gi[i] + ix;
            float v = V[i] + kA * ((kVrest - V[i]) + kR * I);
            if (v > kVth) {
              spk = true;
              v = kVreset;
              ref[i] = N.ref_steps;
            }
            V[i] = v;
          }
          if (spk) sbits |= 1u << i;
          if (has_raster) as_global(L.raster)[(size_t)s * N.n + lo + k] = spk ? 1 : 0;
        }
      }
    };
    if (N.model == 0 && !iext && !L.raster) update(std::true_type{}, std::false_type{}, std::false_type{});
    else update(N.model == 0, iext != nullptr, L.raster != nullptr);
    // compaction of the own spikes: one LDS atomic per wave and neuron slot
    // reserves the wave's positions (the list order carries no meaning: every
    // reader accumulates integer counts)
#pragma unroll
    for (int i = 0; i < kNPT; ++i) {
      const uint64_t m = __ballot((sbits >> i) & 1u);
      if (m) {
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(&sh.ocnt[t & 1], (int)__popcll(m));
        base = __builtin_amdgcn_readfirstlane(base);
        if ((sbits >> i) & 1u) {
          const int pos = base + mask_rank(m);
          const int k = lo + i * kNetThreads + tid;
          if (pos < R) sh.own[pos] = k;
          if (N.n_wg == 1 && pos < kIdBatch) sh.ids[pos] = k;
        }
      }
    }
    __syncthreads();
    const uint32_t tag = (uint32_t)(t + 1);
    const int total = min(sh.ocnt[t & 1], R);
    nloc = (N.n_wg == 1 && total <= kIdBatch) ? total : -1;
    // full own record (persistence, long lists) ...
    uint64_t* out = record(N, pout, w);
    for (int q = tid; q < total; q += kNetThreads) st_coh64(&out[1 + q], pack(tag, (uint32_t)sh.own[q]));
    if (tid == 0) st_coh64(&out[0], pack(tag, (uint32_t)total));
    // ... and the targets, or the header + first ids, pushed to every
    // reader's inbox
    if (PUSH && N.n_wg > 1) {
      if (tid == 0) {  // last read before the barrier above
        sh.fb_cnt = 0;
        sh.acnt = 0;
      }
      push_generate(total);
      __syncthreads();
      push_publish(pout, tag, total);
    } else if (N.n_wg > 1) {
      // the same line to every reader; a thread writes one 16-byte half
      const __amdgpu_buffer_rsrc_t rs = coh_rsrc(N.inbox, inbox_bytes(N));
      const int h = tid & 1;
      auto id = [&](int q) { return sh.own[q] - lo; };
      const uint64_t wa = line_word(tag, 2 * h, total, id), wb = line_word(tag, 2 * h + 1, total, id);
      for (int x = tid; x < 2 * N.n_wg; x += kNetThreads) st_coh128(rs, line_off(N, pout, x >> 1, w, h), wa, wb);
    }
  }

#pragma unroll
  for (int i = 0; i < kNPT; ++i) {
    const int k = i * kNetThreads + tid;
    if (k < R) {
      N.V[lo + k] = V[i];
      N.ge[lo + k] = ge[i];
      N.gi[lo + k] = gi[i];
      N.ref[lo + k] = ref[i];
    }
  }
  // synaptic events delivered by this workgroup
  const unsigned long long ev = wave_sum_u64(ev_local);
  __shared__ unsigned long long ev_s[kNetWaves];
  if (lane_id() == 0) ev_s[wave] = ev;
  __syncthreads();
  if (tid == 0) {
    unsigned long long tot = 0;
    for (int q = 0; q < kNetWaves; ++q) tot += ev_s[q];
    N.events[w] += tot;
  }
  // spike count of the last step: the headers of every workgroup
  if (L.counts && L.n_steps > 0 && w == 0 && !sh.abort_flag) {
    const int64_t t_end = L.t0 + L.n_steps;
    const int par = (int)((t_end - 1) & 1);
    int c = 0;
    if (tid < N.n_wg) {
      if (N.n_wg > 1) {  // word 0 of the source's line in workgroup 0's inbox
        const uint64_t* r = iword(N, par, 0, tid, 0);
        const uint32_t t4 = (uint32_t)t_end & 15u;
        uint64_t hh = ld_coh64(&r[0]);
        for (uint32_t spins = 0; tag4(hh) != t4 && spins <= spin_limit; ++spins) {
          __builtin_amdgcn_s_sleep(1);
          hh = ld_coh64(&r[0]);
        }
        if (tag4(hh) == t4) c = PUSH ? tline_spikes(hh) : line_total(hh);
        else atomicOr(N.error, 1u);
      } else {
        const uint64_t* r = record(N, par, tid);
        const uint64_t hh = wait_slot(r, 0, (uint32_t)t_end, ld_coh64(&r[0]), spin_limit, N, sh);
        if (tag_of(hh) == (uint32_t)t_end) c = (int)(uint32_t)hh;
      }
    }
    int tot;
    block_excl_scan(c, sh.scan, &tot);
    if (tid == 0) as_global(L.counts)[L.n_steps - 1] = tot;
  }
}

template <bool RULES>
__global__ void __launch_bounds__(kNetThreads) net_run_k(BatchArgs args) {
  __shared__ NetShared sh;
  int e = 0;
  while (e < args.n_nets && (int)blockIdx.x >= args.e[e].wg_begin + args.e[e].n_wg) ++e;
  if (e >= args.n_nets) return;
  const NetLaunch L = args.e[e];
  const NetDev N = *L.net;
  const int w = (int)blockIdx.x - L.wg_begin;
  if (N.conn == 1) {
    if (N.push) net_body<1, true, RULES>(L, N, w, args.spin_limit, sh);
    else net_body<1, false, RULES>(L, N, w, args.spin_limit, sh);
  } else {
    // stored rows: the rule only decided how they were built
    net_body<0, false, false>(L, N, w, args.spin_limit, sh);
  }
}

// Launch of the kernel variant for nets of every connectivity rule.  It is
// instantiated in a translation unit of its own (net_rules.hip includes this
// file with BP_NET_RULES_TU defined): compiled beside the lean variant, the
// shared code was outlined differently and the lean kernel lost 2.5 % per
// step.
bp_status launch_net_rules(BatchArgs& args, int32_t wg, bool coop, hipStream_t st);

#ifdef BP_NET_RULES_TU
}  // namespace bp
#else

// Initial state: V0 from the hash (FP64 arithmetic, one rounding), zero
// conductances and counters; every record slot invalid, except the headers of
// the initial (empty) spike set of step -1, tagged 0 in parity 1.
__global__ void net_init_k(const NetDev* __restrict__ Np, float v0_lo, float v0_hi) {
  const NetDev N = *Np;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N.n) {
    const uint32_t wd = hash_word(N.seed, kStreamV0, (uint32_t)i, 0u, 0u);
    const double u = (double)(wd >> 8) * (1.0 / 16777216.0);
    N.V[i] = (float)((double)v0_lo + ((double)v0_hi - (double)v0_lo) * u);
    N.ge[i] = 0.f;
    N.gi[i] = 0.f;
    N.ref[i] = 0;
  }
  const int64_t per = (int64_t)N.range + 1;
  const int64_t slots = 2 * (int64_t)N.n_wg * per;
  if (i < slots) {
    const bool hdr1 = (i / per) >= N.n_wg && (i % per) == 0;
    N.rec[i] = hdr1 ? 0ull : (0xFFFFFFFFull << 32);
  }
  if (N.n_wg > 1) {
    const int64_t ib = 2 * (int64_t)N.n_wg * N.n_wg * N.ibw;
    const int64_t polled = 2 * (int64_t)N.n_wg * N.n_wg * 4;
    if (i < polled) {  // [2 parities][dst][src][4 words]
      const bool par1 = ((i / ((int64_t)N.n_wg * N.n_wg * 4)) & 1) == 1;
      N.inbox[i] = par1 ? 0ull : (15ull << 60);  // empty set of step -1; parity 0 as of step -2
    } else if (i < ib) {
      N.inbox[i] = kNoTag;
    }
  }
  if (i < N.n_wg) N.events[i] = 0ull;
  if (i == 0) *N.error = 0u;
}

// Checkpoint export by the owning workgroup: state and the spikes of the last
// step (records of parity par, tagged `tag`; ids in any order).
__global__ void __launch_bounds__(kNetThreads) net_get_state_k(const NetDev* __restrict__ Np, int par, uint32_t tag,
                                                                float* V, float* ge, float* gi, int32_t* ref,
                                                                uint8_t* s) {
  const NetDev N = *Np;
  const int w = blockIdx.x;
  const int32_t lo = w * N.range, hi = min(lo + N.range, N.n);
  for (int32_t i = lo + threadIdx.x; i < hi; i += kNetThreads) {
    V[i] = N.V[i];
    ge[i] = N.ge[i];
    gi[i] = N.gi[i];
    ref[i] = N.ref[i];
    s[i] = 0;
  }
  __syncthreads();
  const uint64_t* r = N.rec + ((size_t)par * N.n_wg + w) * (size_t)(N.range + 1);
  const uint64_t h = r[0];
  const int c = ((uint32_t)(h >> 32) == tag) ? min((int)(uint32_t)h, N.range) : 0;
  for (int q = threadIdx.x; q < c; q += kNetThreads) {
    const int32_t k = (int32_t)(uint32_t)r[1 + q];
    if (k >= lo && k < hi) s[k] = 1;
  }
}

// Checkpoint import by the owning workgroup: invalidates both record
// parities, then writes the spikes of step `step - 1` tagged `step`.
__global__ void __launch_bounds__(kNetThreads) net_set_state_k(const NetDev* __restrict__ Np, int par, uint32_t step,
                                                                const float* V, const float* ge, const float* gi,
                                                                const int32_t* ref, const uint8_t* s) {
  __shared__ int scan[kNetWaves + 1];
  __shared__ int base_s;
  const NetDev N = *Np;
  const int w = blockIdx.x;
  const int32_t lo = w * N.range, hi = min(lo + N.range, N.n);
  for (int p = 0; p < 2; ++p) {
    uint64_t* r = N.rec + ((size_t)p * N.n_wg + w) * (size_t)(N.range + 1);
    for (int q = threadIdx.x; q <= N.range; q += kNetThreads) r[q] = 0xFFFFFFFFull << 32;
    if (N.n_wg > 1)  // every line as of two steps before
      for (int x = threadIdx.x; x < N.n_wg * N.ibw; x += kNetThreads)
        *iword(N, p, x / N.ibw, w, x % N.ibw) = x % N.ibw < 4 ? (uint64_t)((step - 1u) & 15u) << 60 : kNoTag;
  }
  if (threadIdx.x == 0) base_s = 0;
  vm_drain();  // the invalidations land before the record is rewritten below
  __syncthreads();
  uint64_t* out = N.rec + ((size_t)par * N.n_wg + w) * (size_t)(N.range + 1);
  for (int32_t k0 = lo; k0 < hi; k0 += kNetThreads) {
    const int32_t k = k0 + threadIdx.x;
    int on = 0;
    if (k < hi) {
      N.V[k] = V[k];
      N.ge[k] = ge[k];
      N.gi[k] = gi[k];
      N.ref[k] = ref[k];
      on = s[k] != 0;
    }
    int tot;
    const int ex = block_excl_scan(on, scan, &tot);
    if (on) out[1 + base_s + ex] = ((uint64_t)step << 32) | (uint32_t)k;
    __syncthreads();
    if (threadIdx.x == 0) base_s += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = ((uint64_t)step << 32) | (uint32_t)base_s;
  vm_drain();
  __syncthreads();
  if (N.n_wg > 1 && N.push) {
    // target-pushing nets: "more than the line holds", so readers regenerate
    // the targets from the record
    auto none = [](int) { return 0u; };
    for (int x = threadIdx.x; x < N.n_wg * 4; x += kNetThreads)
      *iword(N, par, x / 4, w, x % 4) = tline_word(step, x % 4, kTgtLine + 1, 0, base_s, none);
  } else if (N.n_wg > 1) {
    auto id = [&](int q) { return (int32_t)(uint32_t)out[1 + q] - lo; };
    for (int x = threadIdx.x; x < N.n_wg * kLine; x += kNetThreads)
      *iword(N, par, x / kLine, w, x % kLine) = line_word(step, x % kLine, base_s, id);
  }
}

__global__ void net_events_k(const NetDev* __restrict__ Np, unsigned long long* dst) {
  const NetDev N = *Np;
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < N.n_wg; i += blockDim.x) s += N.events[i];
  s = wave_sum_u64(s);
  __shared__ unsigned long long red[16];
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) t += red[q];
    *dst = t;
  }
}

// ------------------------------------------------------------------ host side
struct Layout {
  int32_t n_wg, range, nb, push, ibw;
  int64_t nnz_cap;
  bool blk;
  size_t off_hdr, off_V, off_ge, off_gi, off_ref, off_rec, off_inbox, off_events, off_error,
      off_indptr, off_indices, off_blkptr, total;
};

static int64_t nnz_upper_bound(const bp_net_desc* d) {
  const double n = d->n;
  if (d->rule == kRuleFixedDegree) return (int64_t)d->n * (d->degree < d->n ? d->degree : d->n);
  // expected targets per row: 2 n / (K + 1) for uniform gaps, n p with
  // p = 1 - exp(-1 / inv_rate) for geometric gaps
  const double dens = d->rule == kRuleGeometric
                          ? (d->geo_inv_rate > 0.f ? -expm1(-1.0 / (double)d->geo_inv_rate) : 1.0)
                          : 2.0 / ((double)d->max_gap + 1.0);
  const double per_row = n * dens + 1.0;
  const double mean = n * per_row;
  return (int64_t)(mean + 8.0 * sqrt(n * (per_row + 1.0)) + 4096.0);
}

static bp_status make_layout(const bp_net_desc* d, Layout* L) {
  BP_REQUIRE(d != nullptr, "null descriptor");
  BP_REQUIRE(d->n > 0, "n must be > 0");
  BP_REQUIRE(d->n_exc >= 0 && d->n_exc <= d->n, "n_exc must be in [0, n]");
  BP_REQUIRE(d->model == BP_COBA || d->model == BP_CUBA, "unknown model %d", d->model);
  BP_REQUIRE(d->conn == BP_CONN_CSR || d->conn == BP_CONN_JIT, "unknown connectivity %d", d->conn);
  BP_REQUIRE(d->block >= 0, "block must be >= 0");
  bp_status rs = check_rule(d->rule, d->max_gap, d->geo_inv_rate, d->degree, d->block);
  if (rs) return rs;
  BP_REQUIRE(d->dt > 0.f && d->tau_m > 0.f && d->tau_e > 0.f && d->tau_i > 0.f && d->tau_ref >= 0.f,
             "time constants and dt must be positive");
  BP_REQUIRE(d->max_wgs >= 0, "max_wgs must be >= 0");
  const int32_t n = d->n;
  int32_t range, n_wg;
  if (n <= kRangeMax) {
    range = n;
    n_wg = 1;
  } else {
    // default sizing: at most kDefaultWgs workgroups (the exchange costs grow
    // with the square of the workgroup count: at 400k neurons 157 workgroups
    // beat 256 with either exchange), at least one neuron per thread
    const int32_t cap = d->max_wgs > 0 ? d->max_wgs : min(device_cu_count(), kDefaultWgs);
    int64_t r = (n + (int64_t)cap - 1) / cap;
    if (r < kNetThreads) r = kNetThreads;
    if (d->block > 0 && d->block <= kRangeMax) r = (r + d->block - 1) / d->block * d->block;
    if (r > kRangeMax) r = kRangeMax;
    range = (int32_t)r;
    n_wg = (int32_t)((n + r - 1) / r);
  }
  BP_REQUIRE(n_wg <= kMaxWgPerNet, "network too large: %d workgroups of %d neurons (max %d workgroups)", n_wg,
             range, kMaxWgPerNet);
  L->n_wg = n_wg;
  L->range = range;
  L->nb = d->block > 0 ? (int32_t)(((int64_t)n + d->block - 1) / d->block) : 1;
  L->nnz_cap = d->conn == BP_CONN_CSR ? nnz_upper_bound(d) : 0;
  L->blk = d->conn == BP_CONN_CSR && n_wg > 1 && d->block > 0;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L->off_hdr = take(sizeof(NetDev));
  L->off_V = take((size_t)n * 4);
  L->off_ge = take((size_t)n * 4);
  L->off_gi = take((size_t)n * 4);
  L->off_ref = take((size_t)n * 4);
  L->off_rec = take((size_t)2 * n_wg * (range + 1) * 8);
  L->push = n_wg > 1 && d->conn == BP_CONN_JIT && d->block == 0;
  L->ibw = L->push ? kInbox + kExtra : kLine;
  L->off_inbox = n_wg > 1 ? take((size_t)2 * n_wg * n_wg * L->ibw * 8) : 0;
  L->off_events = take((size_t)n_wg * 8);
  L->off_error = take(4);
  L->off_indptr = d->conn == BP_CONN_CSR ? take((size_t)(n + 1) * 4) : 0;
  L->off_indices = d->conn == BP_CONN_CSR ? take((size_t)L->nnz_cap * 4) : 0;
  L->off_blkptr = L->blk ? take((size_t)n * (L->nb + 1) * 4) : 0;
  L->total = o;
  return BP_OK;
}

}  // namespace bp

using namespace bp;

struct bp_net_s {
  NetDev host;
  NetDev* dev;
  bp_net_desc desc;
  Layout lay;
  int64_t step;
  int64_t nnz;
  uint32_t magic;
};

static constexpr uint32_t kNetMagic = 0xB1A1B1A1u;

// Live handles: a handle is dereferenced only after it is found here, so a
// destroyed (freed) or foreign handle is reported instead of read.
static std::mutex g_nets_mu;
static std::unordered_set<const bp_net_s*> g_nets;

static bp_status check_net(bp_net net) {
  bool live;
  {
    std::lock_guard<std::mutex> g(g_nets_mu);
    live = net != nullptr && g_nets.count(net) != 0;
  }
  if (!live || net->magic != kNetMagic) return set_error(BP_ESTATE, "invalid or destroyed network handle");
  return BP_OK;
}

static bp_status launch_batch(const bp_net* nets, int32_t n_nets, const int64_t* n_steps, int32_t* const* counts,
                              uint8_t* const* rasters, const float* const* iext, hipStream_t st) {
  BP_REQUIRE(n_nets >= 0 && n_nets <= kMaxBatch, "batch of %d nets (max %d)", n_nets, kMaxBatch);
  BatchArgs args{};
  args.spin_limit = kSpinLimit;
  int32_t wg = 0;
  bool coop = false, rules = false;  // rules: some regenerated net draws by another rule than rule 0
  for (int32_t i = 0; i < n_nets; ++i) {
    bp_status s = check_net(nets[i]);
    if (s) return s;
    if (nets[i]->desc.conn == BP_CONN_JIT && nets[i]->desc.rule != kRuleUniform) rules = true;
    BP_REQUIRE(n_steps[i] >= 0 && n_steps[i] <= INT32_MAX, "n_steps out of range");
    for (int32_t q = 0; q < i; ++q) BP_REQUIRE(nets[q] != nets[i], "a net appears twice in one batch");
    if (n_steps[i] == 0) continue;
    NetLaunch& L = args.e[args.n_nets++];
    L.net = nets[i]->dev;
    L.raster = rasters ? rasters[i] : nullptr;
    L.counts = counts ? counts[i] : nullptr;
    L.iext = iext ? iext[i] : nullptr;
    L.t0 = nets[i]->step;
    L.n_steps = (int32_t)n_steps[i];
    L.wg_begin = wg;
    L.n_wg = nets[i]->lay.n_wg;
    wg += L.n_wg;
    if (L.n_wg > 1) coop = true;
  }
  if (args.n_nets == 0) return BP_OK;
  if (rules) {
    bp_status s = launch_net_rules(args, wg, coop, st);
    if (s) return s;
  } else if (coop) {
    void* kargs[] = {&args};
    hipError_t e = hipLaunchCooperativeKernel((const void*)net_run_k<false>, dim3(wg), dim3(kNetThreads), kargs, 0,
                                              st);
    if (e != hipSuccess)
      return set_error(BP_EDEVICE, "cooperative launch of %d workgroups failed: %s", wg, hipGetErrorString(e));
  } else {
    net_run_k<false><<<wg, kNetThreads, 0, st>>>(args);
    BP_LAUNCHED("net_run_k");
  }
  for (int32_t i = 0; i < n_nets; ++i) nets[i]->step += n_steps[i];
  return BP_OK;
}

extern "C" {

bp_status bp_net_bytes(const bp_net_desc* d, size_t* bytes) {
  Layout L;
  bp_status s = make_layout(d, &L);
  if (s) return s;
  BP_REQUIRE(bytes != nullptr, "null bytes");
  *bytes = L.total;
  return BP_OK;
}

bp_status bp_net_workgroups(const bp_net_desc* d, int32_t* n_wg) {
  Layout L;
  bp_status s = make_layout(d, &L);
  if (s) return s;
  BP_REQUIRE(n_wg != nullptr, "null n_wg");
  *n_wg = L.n_wg;
  return BP_OK;
}

bp_status bp_create_net(const bp_net_desc* d, void* ws, size_t bytes, bp_stream stream, bp_net* out) {
  Layout L;
  bp_status s = make_layout(d, &L);
  if (s) return s;
  BP_REQUIRE(out != nullptr && ws != nullptr, "null pointer");
  if (bytes < L.total) return set_error(BP_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, L.total);
  hipStream_t st = as_stream(stream);
  bp_net net = new (std::nothrow) bp_net_s();
  if (!net) return set_error(BP_ENOMEM, "host allocation failed");
  char* base = (char*)ws;
  NetDev& H = net->host;
  H.model = d->model;
  H.n = d->n;
  H.n_exc = d->n_exc;
  H.conn = d->conn;
  H.K = d->max_gap;
  H.block = d->block;
  H.rule = d->rule;
  H.degree = d->degree;
  H.inv_rate = d->geo_inv_rate;
  H.nb = L.nb;
  H.ref_steps = (int32_t)floor((double)d->tau_ref / (double)d->dt + 0.5);
  H.seed = d->seed;
  H.w_exc = d->w_exc;
  H.w_inh = d->w_inh;
  H.de = (float)exp(-(double)d->dt / (double)d->tau_e);
  H.di = (float)exp(-(double)d->dt / (double)d->tau_i);
  H.a = (float)((double)d->dt / (double)d->tau_m);
  H.v_rest = d->v_rest;
  H.v_th = d->v_th;
  H.v_reset = d->v_reset;
  H.e_exc = d->e_exc;
  H.e_inh = d->e_inh;
  H.r = d->r;
  H.i_ext = d->i_ext;
  H.n_wg = L.n_wg;
  H.range = L.range;
  H.push = L.push;
  H.ibw = L.ibw;
  H.V = (float*)(base + L.off_V);
  H.ge = (float*)(base + L.off_ge);
  H.gi = (float*)(base + L.off_gi);
  H.ref = (int32_t*)(base + L.off_ref);
  H.rec = (uint64_t*)(base + L.off_rec);
  H.inbox = L.n_wg > 1 ? (uint64_t*)(base + L.off_inbox) : nullptr;
  H.events = (unsigned long long*)(base + L.off_events);
  H.error = (uint32_t*)(base + L.off_error);
  H.indptr = d->conn == BP_CONN_CSR ? (const int32_t*)(base + L.off_indptr) : nullptr;
  H.indices = d->conn == BP_CONN_CSR ? (const int32_t*)(base + L.off_indices) : nullptr;
  H.blkptr = L.blk ? (const int32_t*)(base + L.off_blkptr) : nullptr;
  net->dev = (NetDev*)(base + L.off_hdr);
  net->desc = *d;
  net->lay = L;
  net->step = 0;
  net->nnz = 0;
  net->magic = kNetMagic;
  auto fail = [&](bp_status code) {
    net->magic = 0;
    delete net;
    return code;
  };
  hipError_t e = hipMemcpyAsync(net->dev, &net->host, sizeof(NetDev), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(set_error(BP_EDEVICE, "header copy failed: %s", hipGetErrorString(e)));
  int64_t slots = 2 * (int64_t)L.n_wg * (L.range + 1);
  if (L.n_wg > 1 && 2 * (int64_t)L.n_wg * L.n_wg * L.ibw > slots) slots = 2 * (int64_t)L.n_wg * L.n_wg * L.ibw;
  const int64_t init_n = d->n > slots ? d->n : slots;
  net_init_k<<<(unsigned)((init_n + 255) / 256), 256, 0, st>>>(net->dev, d->v0_lo, d->v0_hi);
  if ((e = hipGetLastError()) != hipSuccess)
    return fail(set_error(BP_EDEVICE, "net_init_k launch failed: %s", hipGetErrorString(e)));
  if (d->conn == BP_CONN_CSR) {
    bp_jit_conn c{};
    c.n_pre = d->n;
    c.n_post = d->n;
    c.max_gap = d->max_gap;
    c.block = d->block;
    c.seed = d->seed;
    c.rule = d->rule;
    c.geo_inv_rate = d->geo_inv_rate;
    c.degree = d->degree;
    int32_t* indptr = (int32_t*)(base + L.off_indptr);
    int32_t* indices = (int32_t*)(base + L.off_indices);
    if ((s = bp_csr_count(&c, indptr, stream))) return fail(s);
    int32_t nnz = 0;
    if ((e = hipMemcpyAsync(&nnz, indptr + d->n, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return fail(set_error(BP_EDEVICE, "reading nnz failed: %s", hipGetErrorString(e)));
    if (nnz < 0) return fail(set_error(BP_EUNSUPPORTED, "more than 2^31-1 synapses"));
    if (nnz > L.nnz_cap)
      return fail(set_error(BP_ENOMEM, "nnz %d above the workspace bound %lld", nnz, (long long)L.nnz_cap));
    net->nnz = nnz;
    if ((s = bp_csr_fill(&c, indptr, indices, stream))) return fail(s);
    if (L.blk && (s = launch_tile_index(indptr, indices, d->n, d->block, L.nb, (int32_t*)(base + L.off_blkptr), st)))
      return fail(s);
  }
  {
    std::lock_guard<std::mutex> g(g_nets_mu);
    g_nets.insert(net);
  }
  *out = net;
  return BP_OK;
}

bp_status bp_run(bp_net net, int64_t n_steps, const float* i_ext_vec, uint8_t* raster, int32_t* counts,
                 bp_stream stream) {
  bp_status s = check_net(net);
  if (s) return s;
  BP_REQUIRE(n_steps >= 0, "negative n_steps");
  return launch_batch(&net, 1, &n_steps, &counts, &raster, &i_ext_vec, as_stream(stream));
}

bp_status bp_step(bp_net net, const float* i_ext_vec, uint8_t* spikes, bp_stream stream) {
  return bp_run(net, 1, i_ext_vec, spikes, nullptr, stream);
}

bp_status bp_run_batch(const bp_net* nets, int32_t n_nets, const int64_t* n_steps, int32_t* const* counts,
                       bp_stream stream) {
  BP_REQUIRE(n_nets >= 0, "negative n_nets");
  if (n_nets == 0) return BP_OK;
  BP_REQUIRE(nets && n_steps, "null pointer");
  return launch_batch(nets, n_nets, n_steps, counts, nullptr, nullptr, as_stream(stream));
}

bp_status bp_net_get_info(bp_net net, bp_net_info* info) {
  bp_status s = check_net(net);
  if (s) return s;
  BP_REQUIRE(info != nullptr, "null info");
  info->n = net->desc.n;
  info->n_wg = net->lay.n_wg;
  info->wg_range = net->lay.range;
  info->nnz = net->nnz;
  info->step = net->step;
  info->bytes_used = net->lay.total;
  info->events_dev = (const uint64_t*)net->host.events;
  info->error_dev = net->host.error;
  return BP_OK;
}

bp_status bp_net_events(bp_net net, uint64_t* dst, bp_stream stream) {
  bp_status s = check_net(net);
  if (s) return s;
  BP_REQUIRE(dst != nullptr, "null dst");
  net_events_k<<<1, 256, 0, as_stream(stream)>>>(net->dev, (unsigned long long*)dst);
  BP_LAUNCHED("net_events_k");
  return BP_OK;
}

size_t bp_state_bytes(bp_net net) {
  if (check_net(net)) return 0;
  const size_t n = (size_t)net->desc.n;
  return n * (4 + 4 + 4 + 4 + 1);
}

bp_status bp_get_state(bp_net net, void* dst, size_t bytes, bp_stream stream) {
  bp_status s = check_net(net);
  if (s) return s;
  BP_REQUIRE(dst != nullptr, "null dst");
  BP_REQUIRE(bytes >= bp_state_bytes(net), "state buffer too small");
  const int64_t n = net->desc.n;
  char* p = (char*)dst;
  const int par = (int)((net->step + 1) & 1);
  net_get_state_k<<<net->lay.n_wg, kNetThreads, 0, as_stream(stream)>>>(
      net->dev, par, (uint32_t)net->step, (float*)p, (float*)(p + 4 * n), (float*)(p + 8 * n), (int32_t*)(p + 12 * n), (uint8_t*)(p + 16 * n));
  BP_LAUNCHED("net_get_state_k");
  return BP_OK;
}

bp_status bp_set_state(bp_net net, const void* src, size_t bytes, int64_t step, bp_stream stream) {
  bp_status s = check_net(net);
  if (s) return s;
  BP_REQUIRE(src != nullptr, "null src");
  BP_REQUIRE(bytes >= bp_state_bytes(net), "state buffer too small");
  BP_REQUIRE(step >= 0 && step <= 0xFFFFFFFFLL, "step out of range");
  const int64_t n = net->desc.n;
  const char* p = (const char*)src;
  const int par = (int)((step + 1) & 1);
  net_set_state_k<<<net->lay.n_wg, kNetThreads, 0, as_stream(stream)>>>(
      net->dev, par, (uint32_t)step, (const float*)p, (const float*)(p + 4 * n), (const float*)(p + 8 * n),
      (const int32_t*)(p + 12 * n), (const uint8_t*)(p + 16 * n));
  BP_LAUNCHED("net_set_state_k");
  net->step = step;
  return BP_OK;
}

bp_status bp_destroy_net(bp_net net) {
  {
    std::lock_guard<std::mutex> g(g_nets_mu);
    if (net == nullptr || g_nets.erase(net) == 0)
      return set_error(BP_ESTATE, "invalid or destroyed network handle");
  }
  net->magic = 0;
  delete net;
  return BP_OK;
}

}  // extern "C"

#endif  // BP_NET_RULES_TU
