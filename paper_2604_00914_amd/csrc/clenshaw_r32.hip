// Clenshaw-step kernels (single block, batched and grouped slices) for one element type (TrR32).
#include "clenshaw_batched.h"
#include "clenshaw_grouped.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r32, afsi::TrR32, afsi::SR32)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_r32, afsi::TrR32)
AFSI_DEFINE_GROUPED_ENTRY(clenshaw_r32, afsi::TrR32)
