// Solve steps for f32 storage, f32 compute.
#include "solve.hpp"

namespace rsvd {
RSVD_DEFINE_SOLVE(f32, float, float)
}  // namespace rsvd
