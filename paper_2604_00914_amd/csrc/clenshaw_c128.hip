// Clenshaw-step kernels (single block, batched and grouped slices) for one element type (TrC128).
#include "clenshaw_batched.h"
#include "clenshaw_grouped.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_c128, afsi::TrC128, afsi::SC128)
AFSI_DEFINE_BATCHED_ENTRY(clenshaw_c128, afsi::TrC128)
AFSI_DEFINE_GROUPED_ENTRY(clenshaw_c128, afsi::TrC128)
