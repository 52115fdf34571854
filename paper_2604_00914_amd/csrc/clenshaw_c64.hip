// Clenshaw-step kernels (single block, batched and grouped slices) for one element type (TrC64).
#include "clenshaw_batched.h"
#include "clenshaw_grouped.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_c64, afsi::TrC64, afsi::SC64)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_c64, afsi::TrC64)
AFSI_DEFINE_GROUPED_ENTRY(clenshaw_c64, afsi::TrC64)
