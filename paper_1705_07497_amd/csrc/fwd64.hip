// Forward products of operators whose ray bundles are 64 rays wide.
#include "fwd_kernels.hpp"

namespace sct {
SCT_FWD_INST(64)
}  // namespace sct
