// Reduced-precision mu-mode products (FP32 and split-BF16); filled in below.
#include "common.h"

namespace adr {

hipError_t launch_mode_product_f32(const ModeArgs&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_mode_product_bf16x3(const ModeArgs&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace adr
