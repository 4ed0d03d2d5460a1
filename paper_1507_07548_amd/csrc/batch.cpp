// Batched, device-resident simulation: slots, admission, stepping, sampling.
#include <hip/hip_runtime.h>

#include "batch.h"

using namespace ms2;

extern "C" {
ms2_status ms2_batch_create(ms2_ctx*, int32_t, size_t, ms2_batch** out) {
  if (out) *out = nullptr;
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
void ms2_batch_destroy(ms2_batch*) {}
ms2_status ms2_slot_footprint(ms2_ctx*, const ms2_system*, size_t*) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
ms2_status ms2_slot_admit(ms2_batch*, const ms2_system*, int32_t*, void*) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
ms2_status ms2_slot_retire(ms2_batch*, int32_t) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
ms2_status ms2_step(ms2_batch*, int32_t, int32_t, void*) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
ms2_status ms2_sample(ms2_batch*, int32_t, ms2_samples*, void*) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
ms2_status ms2_slot_status(ms2_batch*, int32_t, int64_t*, int32_t*, void*) {
  return set_error(MS2_EINVAL, "batched path not available in this build");
}
}
