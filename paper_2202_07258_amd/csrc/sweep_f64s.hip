// Instantiation unit of the column sweep: double storage, element loads (unaligned columns), every variant.
#include "sweep.h"

namespace bxs {
hipError_t sweep_f64s(const LaunchCtx& c, int variant, int mode, const Item* items, int n_items, int first)
{
    return sweep_dispatch_part<double, 1, 1, 0>(c, variant, mode, items, n_items, first);
}
}  // namespace bxs
