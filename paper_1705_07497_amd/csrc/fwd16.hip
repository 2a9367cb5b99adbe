// Forward products of operators whose ray bundles are 16 rays wide.
#include "fwd_kernels.hpp"

namespace sct {
SCT_FWD_INST(16)
}  // namespace sct
