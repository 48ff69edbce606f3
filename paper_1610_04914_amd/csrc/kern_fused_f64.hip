// fp64 instantiations of the fused RK4 step (tile table in kern_fused_f32.hip).
#include "kern_fused.hpp"

namespace lll {

hipError_t launch_step_fused_f64(int precession, int anis, int variant, int bz, const RepDev* reps,
                                 const int4* tiles, int ntiles, State in, State out, int kick,
                                 uint64_t k, double so, double* kd, const LaunchEvents* ev,
                                 hipStream_t st) {
    switch (variant) {
        case 1: return launch_p<double, 32, 8, 640>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case 2: return launch_p<double, 16, 16, 576>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case 3: return launch_p<double, 16, 16, 256>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case 4: return launch_p<double, 32, 8, 256>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case 5: return launch_p<double, 16, 8, 384>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lll
