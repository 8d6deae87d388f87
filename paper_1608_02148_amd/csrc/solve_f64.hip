// Solve steps for f64 storage, f64 compute.
#include "solve.hpp"

namespace rsvd {
RSVD_DEFINE_SOLVE(f64, double, double)
}  // namespace rsvd
