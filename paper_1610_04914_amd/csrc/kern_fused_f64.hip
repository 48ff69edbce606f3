// fp64 instantiations of the fused RK4 step (tile table in kern_fused_f32.hip).
#include "kern_fused.hpp"

namespace lll {

hipError_t fused_f64_stages(int precession, int anis, int variant, int bz, const RepDev* reps,
                            const int4* tiles, int ntiles, State in, State out, const State* y,
                            hipStream_t st) {
#define LLL_ST_PASS precession, anis, reps, tiles, ntiles, in, out, y, bz, st
    switch (variant) {
        case 1: return launch_stages_v<double, 32, 8, 640>(LLL_ST_PASS);
        case 2: return launch_stages_v<double, 16, 16, 576>(LLL_ST_PASS);
        case 3: return launch_stages_v<double, 16, 16, 256>(LLL_ST_PASS);
        case 4: return launch_stages_v<double, 32, 8, 256>(LLL_ST_PASS);
        case 5: return launch_stages_v<double, 16, 8, 384>(LLL_ST_PASS);
        case 6: return launch_stages_v<double, 16, 16, 512>(LLL_ST_PASS);
        case 7: return launch_stages_v<double, 32, 8, 512>(LLL_ST_PASS);
        default: return hipErrorInvalidValue;
    }
#undef LLL_ST_PASS
}

hipError_t fused_f64_rk4(LLL_FUSED_ARGS) { return fused_f64<0>(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st); }

}  // namespace lll
