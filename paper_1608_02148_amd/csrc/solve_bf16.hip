// Solve steps for bf16 storage, f32 compute.
#include "solve.hpp"

namespace rsvd {
RSVD_DEFINE_SOLVE(bf16, bf16_t, float)
}  // namespace rsvd
