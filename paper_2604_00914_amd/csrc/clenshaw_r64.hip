// Clenshaw-step kernels (single block, batched and grouped slices) for one element type (TrR64).
#include "clenshaw_batched.h"
#include "clenshaw_grouped.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r64, afsi::TrR64, afsi::SR64)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_r64, afsi::TrR64)
AFSI_DEFINE_GROUPED_ENTRY(clenshaw_r64, afsi::TrR64)
