// fp64 instantiations of the fused Butcher RK5 step (tile shapes of the fp64
// RK4 variants) and the precision dispatch.
#include "kern_fused_rk5.hpp"

namespace lll {

hipError_t fused_f32_rk5(int precession, int anis, int variant, int bz, const RepDev* reps,
                         const int4* tiles, int ntiles, State in, State out, const State* k,
                         int kick, uint64_t kp, double so, unsigned long long* kd, hipStream_t st);

static hipError_t fused_f64_rk5(int precession, int anis, int variant, int bz, const RepDev* reps,
                                const int4* tiles, int ntiles, State in, State out, const State* k,
                                int kick, uint64_t kp, double so, unsigned long long* kd,
                                hipStream_t st) {
#define LLL_RK5_PASS precession, anis, reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st
    switch (variant) {
        case 1: return launch_rk5_p<double, 32, 8, 640, 448>(LLL_RK5_PASS);
        case 2: return launch_rk5_p<double, 16, 16, 576, 448>(LLL_RK5_PASS);
        case 3: return launch_rk5_p<double, 16, 16, 256, 256>(LLL_RK5_PASS);
        case 4: return launch_rk5_p<double, 32, 8, 256, 256>(LLL_RK5_PASS);
        case 5: return launch_rk5_p<double, 16, 8, 384, 256>(LLL_RK5_PASS);
        case 6: return launch_rk5_p<double, 16, 16, 512, 448>(LLL_RK5_PASS);
        case 7: return launch_rk5_p<double, 32, 8, 512, 448>(LLL_RK5_PASS);
        default: return hipErrorInvalidValue;
    }
#undef LLL_RK5_PASS
}

hipError_t launch_step_rk5_fused(int prec, int precession, int anis, int variant, int bz,
                                 const RepDev* reps, const int4* tiles, int ntiles, State in,
                                 State out, const State* k, int kick, uint64_t kp, double so,
                                 unsigned long long* kd, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return prec == 0 ? fused_f64_rk5(precession, anis, variant, bz, reps, tiles, ntiles, in, out, k,
                                     kick, kp, so, kd, st)
                     : fused_f32_rk5(precession, anis, variant, bz, reps, tiles, ntiles, in, out, k,
                                     kick, kp, so, kd, st);
}

}  // namespace lll
