// Instantiation unit of the Dyson kernel for band windows padded to 48.
#include "dyson_impl.h"

namespace dmft {
DMFT_DEFINE_LAUNCH_SLDS(48)
}  // namespace dmft
