// Clenshaw-step kernels instantiated for one element type (TrC64).
#include "clenshaw_dispatch.h"

AFSI_DEFINE_STEP_ENTRY(clenshaw_c64, afsi::TrC64, afsi::SC64)
