// Clenshaw-step kernels instantiated for one element type (TrR32).
#include "clenshaw_dispatch.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r32, afsi::TrR32, afsi::SR32)
