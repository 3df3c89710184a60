// Placeholder translation unit for the BF16 matrix-core walk of correlated
// Gaussians; until it lands the engine rejects GGNS_FP32_BF16MMA runs at init.
#include "ggns_common.h"

namespace ggns {

int launch_walk_mfma(void *, const RunDev *, const Tile *, int, int, hipStream_t) {
    return GGNS_EUNSUPPORTED;
}

}  // namespace ggns
