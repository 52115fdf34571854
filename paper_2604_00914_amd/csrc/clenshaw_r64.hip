// Clenshaw-step kernels (single block and batched slices) for one element type (TrR64).
#include "clenshaw_batched.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r64, afsi::TrR64, afsi::SR64)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_r64, afsi::TrR64)
