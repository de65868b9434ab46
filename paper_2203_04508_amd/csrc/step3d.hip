// D3Q19 fused step (placeholder until the 3-D marching kernel lands).
#include "kernels_common.h"

namespace mcb {
hipError_t step3d(mcb_ctx*, const void*, void*, bool) { return hipErrorNotSupported; }
}  // namespace mcb
