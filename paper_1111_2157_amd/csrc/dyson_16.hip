// Instantiation unit of the Dyson kernel for band windows padded to 16.
#include "dyson_impl.h"

namespace dmft {
DMFT_DEFINE_LAUNCH(16)
}  // namespace dmft
