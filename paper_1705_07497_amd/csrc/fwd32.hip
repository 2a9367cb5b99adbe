// Forward products of operators whose ray bundles are 32 rays wide.
#include "fwd_kernels.hpp"

namespace sct {
SCT_FWD_INST(32)
}  // namespace sct
