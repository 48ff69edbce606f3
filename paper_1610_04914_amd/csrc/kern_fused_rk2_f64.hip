// fp64 instantiations of the fused RK2-midpoint steps: two steps per
// launch (scheme 1) and a single step (scheme 2).
#include "kern_fused.hpp"

namespace lll {

hipError_t fused_f64_rk2(int scheme, LLL_FUSED_ARGS) {
    if (scheme == 1)
        return fused_f64<1>(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st);
    if (scheme == 2)
        return fused_f64<2>(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st);
    return hipErrorInvalidValue;
}

}  // namespace lll
