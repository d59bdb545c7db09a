// Tiled matrix-core X-engine kernels of one arithmetic path (see xeng_mfma_impl.h).
#include "xeng_mfma_impl.h"

XENG_MFMA_PATH(ACC_F16, f16)
