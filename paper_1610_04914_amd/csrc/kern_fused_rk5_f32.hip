// fp32 instantiations of the fused Butcher RK5 step.  Variant v has the tile
// shape of RK4 variant v; the thread counts are those of each launch.
#include "kern_fused_rk5.hpp"

namespace lll {

hipError_t fused_f32_rk5(int precession, int anis, int variant, int bz, const RepDev* reps,
                         const int4* tiles, int ntiles, State in, State out, const State* k,
                         int kick, uint64_t kp, double so, unsigned long long* kd, hipStream_t st) {
#define LLL_RK5_PASS precession, anis, reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st
    switch (variant) {
        case 1: return launch_rk5_p<float, 32, 16, 960, 768>(LLL_RK5_PASS);
        case 2: return launch_rk5_p<float, 32, 16, 512, 512>(LLL_RK5_PASS);
        case 3: return launch_rk5_p<float, 16, 16, 576, 448>(LLL_RK5_PASS);
        case 4: return launch_rk5_p<float, 32, 8, 640, 448>(LLL_RK5_PASS);
        case 5: return launch_rk5_p<float, 64, 8, 512, 512>(LLL_RK5_PASS);
        case 6: return launch_rk5_p<float, 32, 16, 1024, 768>(LLL_RK5_PASS);
        default: return hipErrorInvalidValue;
    }
#undef LLL_RK5_PASS
}

}  // namespace lll
