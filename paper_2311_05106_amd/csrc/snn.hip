// Recurrent LIF network trained by backpropagation through time with a
// surrogate spike derivative (Section 5.3; Appendix I).
#include "bp_device.h"
#include "bp_host.h"

using namespace bp;

extern "C" {

size_t bp_snn_ckpt_bytes(const bp_snn* m) { return 0; }
size_t bp_snn_ws_bytes(const bp_snn* m) { return 0; }

bp_status bp_snn_forward(const bp_snn* m, void* ckpt, float* logits, float* loss, uint8_t* raster, bp_stream stream) {
  return set_error(BP_EUNSUPPORTED, "not built yet");
}

bp_status bp_snn_backward(const bp_snn* m, const void* ckpt, const float* logits, float* dW_in, float* dw_rec,
                          float* dW_out, float* db_out, void* ws, size_t ws_bytes, bp_stream stream) {
  return set_error(BP_EUNSUPPORTED, "not built yet");
}

}  // extern "C"
