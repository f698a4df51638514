// Instantiation unit of the Dyson kernel for band windows padded to 32.
#include "dyson_impl.h"

namespace dmft {
DMFT_DEFINE_LAUNCH(32)
}  // namespace dmft
