// Fused single-pass LADMM iteration (placeholder until the MFMA kernel lands).
#include "internal.h"

#include <hip/hip_runtime.h>

namespace ssmap {

bool fused_supported(int, int) { return false; }

void launch_iter_fused(int, const IterArgs &, hipStream_t) {}

}  // namespace ssmap
