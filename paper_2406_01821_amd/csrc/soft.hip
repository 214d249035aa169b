// Soft (sigmoid-relaxed) forward and backward passes.
#include "internal.h"

namespace aerl {

size_t soft_ws_bytes(const DatasetRec &, const PopRec &, bool) { return 0; }
hipError_t launch_soft_forward(const SoftLaunch &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_soft_backward(const SoftLaunch &, hipStream_t) { return hipErrorNotSupported; }

}  // namespace aerl
