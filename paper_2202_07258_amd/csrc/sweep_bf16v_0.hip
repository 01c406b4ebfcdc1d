// Instantiation unit of the column sweep: bf16 storage, 16-byte loads, variants with id % kSweepParts == 0.
#include "sweep.h"

namespace bxs {
hipError_t sweep_bf16v_0(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first)
{
    return sweep_dispatch_part<__bf16, 8, kSweepParts, 0>(c, variant, mode, items, n_items, first);
}
}  // namespace bxs
