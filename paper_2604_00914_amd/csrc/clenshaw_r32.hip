// Clenshaw-step kernels (single block and batched slices) for one element type (TrR32).
#include "clenshaw_batched.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r32, afsi::TrR32, afsi::SR32)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_r32, afsi::TrR32)
