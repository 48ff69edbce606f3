// fp32 instantiations of the fused RK4 step and the tile-shape table.
#include "kern_fused.hpp"

namespace lll {

struct VariantDesc {
    int bx, by, nt;
};
// Output tile (bx, by) and threads per workgroup.  LDS bytes = 6 * sizeof(T) *
// sum over s = 0..3 of ((bx + 2(4-s)) | 1) (by + 2(4-s)) (double-buffered x, y,
// z planes of the four stage inputs, rows padded to an odd pitch).
static const VariantDesc kVar32[] = {{32, 16, 960}, {32, 16, 512}, {16, 16, 576}, {32, 8, 640},
                                     {64, 8, 512}, {32, 16, 1024}};
static const VariantDesc kVar64[] = {{32, 8, 640}, {16, 16, 576}, {16, 16, 256}, {32, 8, 256},
                                     {16, 8, 384}, {16, 16, 512}, {32, 8, 512}};

static int lds_bytes(int bx, int by, int es) {
    int r = 0;
    for (int s = 0; s < 4; ++s) r += ((bx + 2 * (4 - s)) | 1) * (by + 2 * (4 - s));
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

hipError_t fused_f32_rk4(LLL_FUSED_ARGS) { return fused_f32<0>(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st); }

hipError_t fused_f64_stages(int precession, int anis, int variant, int bz, const RepDev* reps,
                            const int4* tiles, int ntiles, State in, State out, const State* y,
                            hipStream_t st);

static hipError_t fused_f32_stages(int precession, int anis, int variant, int bz, const RepDev* reps,
                                   const int4* tiles, int ntiles, State in, State out,
                                   const State* y, hipStream_t st) {
#define LLL_ST_PASS precession, anis, reps, tiles, ntiles, in, out, y, bz, st
    switch (variant) {
        case 1: return launch_stages_v<float, 32, 16, 960>(LLL_ST_PASS);
        case 2: return launch_stages_v<float, 32, 16, 512>(LLL_ST_PASS);
        case 3: return launch_stages_v<float, 16, 16, 576>(LLL_ST_PASS);
        case 4: return launch_stages_v<float, 32, 8, 640>(LLL_ST_PASS);
        case 5: return launch_stages_v<float, 64, 8, 512>(LLL_ST_PASS);
        case 6: return launch_stages_v<float, 32, 16, 1024>(LLL_ST_PASS);
        default: return hipErrorInvalidValue;
    }
#undef LLL_ST_PASS
}

hipError_t launch_step_fused_stages(int prec, int precession, int anis, int variant, int bz,
                                    const RepDev* reps, const int4* tiles, int ntiles, State in,
                                    State out, const State* y, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return prec == 0 ? fused_f64_stages(precession, anis, variant, bz, reps, tiles, ntiles, in, out, y, st)
                     : fused_f32_stages(precession, anis, variant, bz, reps, tiles, ntiles, in, out, y, st);
}

hipError_t launch_step_fused(int prec, int precession, int anis, int variant, int bz, int scheme,
                             const RepDev* reps, const int4* tiles, int ntiles, State in,
                             State out, int kick, uint64_t k, double so,
                             unsigned long long* kd, const LaunchEvents* ev, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (scheme == 0)
        return prec == 0 ? fused_f64_rk4(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st)
                         : fused_f32_rk4(precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st);
    return prec == 0 ? fused_f64_rk2(scheme, precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st)
                     : fused_f32_rk2(scheme, precession, anis, variant, bz, reps, tiles, ntiles, in, out, kick, k, so, kd, ev, st);
}

}  // namespace lll
