// Instantiations of the fused MFMA passes for one precision.
#include "bf_fused_kernel.h"

namespace bfly {
namespace fused {
BF_FUSED_DEFINE_LAUNCH(kF16)
}  // namespace fused
}  // namespace bfly
