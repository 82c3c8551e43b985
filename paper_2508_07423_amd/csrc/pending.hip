// Entry points whose kernels are not built yet.
#include "internal.hpp"
namespace etx {
int prefilter_attributes(size_t) { return 0; }
hipError_t launch_prefilter_infer(const RunArgs&) { return hipErrorNotSupported; }
hipError_t launch_prefilter_train(const RunArgs&, const uint8_t*, float, float, int64_t, float*) { return hipErrorNotSupported; }
hipError_t build_low_precision(etx_ctx*) { return hipErrorNotSupported; }
}  // namespace etx
extern "C" {
etx_status etx_autotune(etx_ctx*, const etx_hits*, etx_out*, void*, size_t, etx_stream, const char*) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_calibrate(etx_ctx*, const etx_hits*, etx_out*, void*, size_t, etx_stream) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_set_precision(etx_ctx*, int32_t) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_prefilter_set(etx_ctx*, const float*, int64_t) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_prefilter_get(const etx_ctx*, float*, int64_t) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_prefilter_train_step(etx_ctx*, const etx_hits*, etx_out*, const uint8_t*, float, float, int64_t, float*, void*, size_t, etx_stream) { return ETX_ERR_UNSUPPORTED; }
etx_status etx_prefilter_state(etx_ctx*, float*, int64_t, int32_t) { return ETX_ERR_UNSUPPORTED; }
}
