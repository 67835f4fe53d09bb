// The network kernel for nets of every connectivity rule (geometric gaps,
// exactly fixed out-degree, and the paper's uniform gaps), compiled in a
// translation unit of its own so that the uniform-gap kernel of net.hip keeps
// its own code generation.  Everything but the kernel template comes from
// net.hip.
#define BP_NET_RULES_TU
#include "net.hip"

namespace bp {

bp_status launch_net_rules(BatchArgs& args, int32_t wg, bool coop, hipStream_t st) {
  if (coop) {
    void* kargs[] = {&args};
    hipError_t e = hipLaunchCooperativeKernel((const void*)net_run_k<true>, dim3(wg), dim3(kNetThreads), kargs, 0,
                                              st);
    if (e != hipSuccess)
      return set_error(BP_EDEVICE, "cooperative launch of %d workgroups failed: %s", wg, hipGetErrorString(e));
  } else {
    net_run_k<true><<<wg, kNetThreads, 0, st>>>(args);
    BP_LAUNCHED("net_run_k");
  }
  return BP_OK;
}

}  // namespace bp
