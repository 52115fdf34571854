// Clenshaw-step kernels instantiated for one element type (TrR64).
#include "clenshaw_dispatch.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_r64, afsi::TrR64, afsi::SR64)
