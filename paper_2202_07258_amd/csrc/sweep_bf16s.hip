// Instantiation unit of the column sweep: bf16 storage, element loads (unaligned columns), every variant.
#include "sweep.h"

namespace bxs {
hipError_t sweep_bf16s(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first)
{
    return sweep_dispatch_part<__bf16, 1, 1, 0>(c, variant, mode, items, n_items, first);
}
}  // namespace bxs
