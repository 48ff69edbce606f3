// fp64 instantiations of the fused RK4 step (tile table in kern_fused_f32.hip).
#include "kern_fused.hpp"

namespace lll {

hipError_t fused_f64_rk4(LLL_FUSED_ARGS) { return fused_f64<0>(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st); }

}  // namespace lll
