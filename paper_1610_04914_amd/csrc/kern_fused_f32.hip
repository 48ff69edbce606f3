// fp32 instantiations of the fused RK4 step and the tile-shape table.
#include "kern_fused.hpp"

namespace lll {

struct VariantDesc {
    int bx, by, nt;
};
// Output tile (bx, by) and threads per workgroup.  LDS bytes =
// 6 * sizeof(T) * (R0 + R1 + R2 + R3) with Rs = (bx + 2(4-s)) (by + 2(4-s)).
static const VariantDesc kVar32[] = {{32, 16, 512}, {32, 16, 256}, {16, 16, 256}, {32, 8, 256},
                                     {64, 8, 512}};
static const VariantDesc kVar64[] = {{16, 16, 256}, {32, 8, 256}, {16, 8, 128}, {24, 16, 384}};

static int lds_bytes(int bx, int by, int es) {
    const int r = (bx + 8) * (by + 8) + (bx + 6) * (by + 6) + (bx + 4) * (by + 4) + (bx + 2) * (by + 2);
    return 6 * es * r;
}

int fused_variant_count(int prec) {
    return prec == 0 ? (int)(sizeof(kVar64) / sizeof(kVar64[0]))
                     : (int)(sizeof(kVar32) / sizeof(kVar32[0]));
}

bool fused_variant_info(int prec, int variant, FusedInfo* out) {
    if (variant < 1 || variant > fused_variant_count(prec)) return false;
    const VariantDesc& d = prec == 0 ? kVar64[variant - 1] : kVar32[variant - 1];
    out->bx = d.bx;
    out->by = d.by;
    out->threads = d.nt;
    out->lds_bytes = lds_bytes(d.bx, d.by, prec == 0 ? 8 : 4);
    return true;
}

hipError_t launch_step_fused_f64(int precession, int anis, int variant, int bz, const RepDev* reps,
                                 const int4* tiles, int ntiles, State in, State out, int kick,
                                 uint64_t k, double so, unsigned long long* kd, hipStream_t st);

hipError_t launch_step_fused(int prec, int precession, int anis, int variant, int bz,
                             const RepDev* reps, const int4* tiles, int ntiles, State in,
                             State out, int kick, uint64_t k, double so,
                             unsigned long long* kd, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (prec == 0)
        return launch_step_fused_f64(precession, anis, variant, bz, reps, tiles, ntiles, in, out,
                                     kick, k, so, kd, st);
    switch (variant) {
        case 1: return launch_p<float, 32, 16, 512>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, st);
        case 2: return launch_p<float, 32, 16, 256>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, st);
        case 3: return launch_p<float, 16, 16, 256>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, st);
        case 4: return launch_p<float, 32, 8, 256>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, st);
        case 5: return launch_p<float, 64, 8, 512>(precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lll
