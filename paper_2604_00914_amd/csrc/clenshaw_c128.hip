// Clenshaw-step kernels instantiated for one element type (TrC128).
#include "clenshaw_dispatch.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_c128, afsi::TrC128, afsi::SC128)
