// Host-side helpers of the C ABI: thread-local error text, status macros,
// launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/bp.h"
#include "bp_device.h"

namespace bp {

bp_status set_error(bp_status s, const char* fmt, ...);

#define BP_REQUIRE(cond, ...)                                  \
  do {                                                         \
    if (!(cond)) return ::bp::set_error(BP_EINVAL, __VA_ARGS__); \
  } while (0)

#define BP_HIP(call)                                                                                    \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      return ::bp::set_error(BP_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                                 \
  } while (0)

// After a kernel launch: report launch-configuration errors.
#define BP_LAUNCHED(name)                                                                                    \
  do {                                                                                                       \
    hipError_t e_ = hipGetLastError();                                                                       \
    if (e_ != hipSuccess) return ::bp::set_error(BP_EDEVICE, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
  } while (0)

inline hipStream_t as_stream(bp_stream s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int device_cu_count();

// The device generator of a connectivity descriptor.
__host__ __device__ inline ConnGen conn_gen(const bp_jit_conn& c) {
  ConnGen g;
  g.seed = c.seed;
  g.K = (uint32_t)c.max_gap;
  g.n_post = c.n_post;
  g.B = c.block;
  g.rule = c.rule;
  g.inv_rate = c.geo_inv_rate;
  g.degree = c.degree;
  return g;
}

bp_status check_conn(const bp_jit_conn* c, bool weights);
bp_status check_rule(int32_t rule, int32_t max_gap, float inv_rate, int32_t degree, int32_t block);

// tp[j][t] = first position of sorted row j with column >= t * tile
// (tp[j][n_tiles] = end of row); tp has n_pre * (n_tiles + 1) entries.
bp_status launch_tile_index(const int32_t* indptr, const int32_t* indices, int32_t n_pre, int32_t tile,
                            int32_t n_tiles, int32_t* tp, hipStream_t st);

}  // namespace bp
