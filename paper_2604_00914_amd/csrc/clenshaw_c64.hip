// Clenshaw-step kernels (single block and batched slices) for one element type (TrC64).
#include "clenshaw_batched.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_c64, afsi::TrC64, afsi::SC64)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_c64, afsi::TrC64)
