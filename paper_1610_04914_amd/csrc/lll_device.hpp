// Device-side building blocks of the pulse-noise path: the counter-based
// generator, Box-Muller normals, the kick (Eqs. (5)-(6) + renormalisation) and
// the per-site right-hand side of the noise-free Landau-Lifshitz equation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lll_internal.hpp"

namespace lll {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // three-input XORs as one gfx950 bitop3 (truth table 0x96); in the first
        // round the words other than c0 are wave-uniform in every caller, so n0
        // is left to the scalar unit there
        const uint32_t n0 = r == 0 ? hi1 ^ c1 ^ k0 : __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 philox_site(uint64_t seed, uint32_t i, uint32_t k, uint32_t r,
                                             uint32_t tag) {
    return philox4x32_10(i, k, r, tag, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
}

// Three unit normals by Box-Muller from one Philox block, u = (w + 1/2) 2^-32:
// G = (r0 cos 2pi u1, r0 sin 2pi u1, r1 cos 2pi u3), r = sqrt(-2 ln u).
template <typename T>
__device__ __forceinline__ void gauss3(uint4 w, T G[3]);

template <>
__device__ __forceinline__ void gauss3<double>(uint4 w, double G[3]) {
    const double s = 2.3283064365386963e-10;  // 2^-32
    const double u0 = ((double)w.x + 0.5) * s;
    const double u2 = ((double)w.z + 0.5) * s;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    // sin/cos(2 pi u) = sinpi/cospi(2u); 2u = (w + 1/2) 2^-31 exactly
    const double a1 = ((double)w.y + 0.5) * 4.656612873077393e-10;
    const double a3 = ((double)w.w + 0.5) * 4.656612873077393e-10;
    double sn, cs;
    sincospi(a1, &sn, &cs);
    G[0] = r0 * cs;
    G[1] = r0 * sn;
    G[2] = r1 * cospi(a3);
}

// -ln u in fp32 with full relative accuracy over all of (0,1) from one
// hardware log2 (about 1 ulp on gfx950).  u < 1/2: -ln u = -log2(u) ln 2.
// u >= 1/2: -ln u = -log1p(-v) with v = 1 - u formed exactly from the
// complemented word, evaluated by Kahan's identity
// log1p(x) = ln(1 + x) x / ((1 + x) - 1) (D. Goldberg, "What every computer
// scientist should know about floating-point arithmetic", 1991), y = 1 - v.
__device__ __forceinline__ float neglog_u01(uint32_t w) {
    const bool lo = w < 0x80000000u;
    const float v = ((float)(lo ? w : ~w) + 0.5f) * 2.3283064365386963e-10f;  // u, or 1 - u
    const float y = lo ? v : 1.0f - v;
    const float L = __builtin_amdgcn_logf(y) * 0.6931471805599453f;            // ln y
    const float hi = (y == 1.0f) ? v : L * v * __builtin_amdgcn_rcpf(y - 1.0f);
    return lo ? -L : hi;
}

template <>
__device__ __forceinline__ void gauss3<float>(uint4 w, float G[3]) {
    const float r0 = __builtin_amdgcn_sqrtf(2.0f * neglog_u01(w.x));
    const float r1 = __builtin_amdgcn_sqrtf(2.0f * neglog_u01(w.z));
    // hardware sin/cos take the angle in revolutions: sin(2 pi u)
    const float u1 = ((float)w.y + 0.5f) * 2.3283064365386963e-10f;
    const float u3 = ((float)w.w + 0.5f) * 2.3283064365386963e-10f;
    G[0] = r0 * __builtin_amdgcn_cosf(u1);
    G[1] = r0 * __builtin_amdgcn_sinf(u1);
    G[2] = r1 * __builtin_amdgcn_cosf(u3);
}

// |phi|, 1/|phi| and sin/cos |phi| of the rotation angle.
template <typename T>
__device__ __forceinline__ void angle_of(T ph2, T& inv, T& sn, T& cs);

template <>
__device__ __forceinline__ void angle_of<double>(double ph2, double& inv, double& sn, double& cs) {
    const double ph = sqrt(ph2);
    inv = 1.0 / ph;
    sincospi(ph * 0.3183098861837907, &sn, &cs);  // sin/cos(pi * ph/pi)
}

template <>
__device__ __forceinline__ void angle_of<float>(float ph2, float& inv, float& sn, float& cs) {
    const float ph = __builtin_amdgcn_sqrtf(ph2);
    inv = __builtin_amdgcn_rcpf(ph);
    const float rev = __builtin_amdgcn_fractf(ph * 0.15915494309189535f);  // ph / 2pi, in [0,1)
    sn = __builtin_amdgcn_sinf(rev);
    cs = __builtin_amdgcn_cosf(rev);
}

// Renormalisation s = s'/|s'| after a kick; returns | |s'| - 1 | in fp64.
// fp64 state: the norm and the quotient in fp64.  fp32 state: |s'|^2 of the
// fp32 components is formed in fp64 (each square exact, so the deviation
// |s'|^2 - 1 keeps its relative accuracy however small it is); 1/|s'| is the
// hardware's fp32 reciprocal square root refined by one Newton step in fp64
// (the estimate alone is about 1 ulp off and leans low: spins rescaled with
// it kept |s| about 4e-8 below 1 on average, which lowered |E| by about two
// parts in 1e7), and each component is rounded to fp32 once, from fp64, so
// that |s| - 1 averages zero; | |s'| - 1 | = | |s'|^2 - 1 | / (|s'| + 1)
// with the well-conditioned denominator.
template <typename T>
__device__ __forceinline__ double renorm(T ox, T oy, T oz, T& sx, T& sy, T& sz);

template <>
__device__ __forceinline__ double renorm<double>(double ox, double oy, double oz, double& sx,
                                                 double& sy, double& sz) {
    const double nrm = sqrt(ox * ox + oy * oy + oz * oz);
    const double inv = 1.0 / nrm;
    sx = ox * inv;
    sy = oy * inv;
    sz = oz * inv;
    return fabs(nrm - 1.0);
}

template <>
__device__ __forceinline__ double renorm<float>(float ox, float oy, float oz, float& sx, float& sy,
                                                float& sz) {
    const double dx = (double)ox, dy = (double)oy, dz = (double)oz;
    const double n2 = dx * dx + dy * dy + dz * dz;
    const double r0 = (double)__builtin_amdgcn_rsqf((float)n2);
    const double inv = r0 * (1.5 - 0.5 * n2 * (r0 * r0));
    sx = (float)(dx * inv);
    sy = (float)(dy * inv);
    sz = (float)(dz * inv);
    const float den = (float)(n2 * inv) + 1.0f;
    return fabs(n2 - 1.0) * (double)__builtin_amdgcn_rcpf(den);
}

// Kick of one spin: rotation by phi = sigma G about n = phi/|phi| (Eq. (6)),
// identity when phi = 0, then renormalisation (renorm above).
// Returns | |s'| - 1 | (fp64).  Multiply-adds contract only within one
// expression (the library's build setting), so the kick gives identical bits
// wherever it is inlined (separate kernel or epilogue).
template <typename T>
__device__ __forceinline__ double kick_spin(T& sx, T& sy, T& sz, uint4 w, T sigma) {
    T G[3];
    gauss3<T>(w, G);
    const T px = sigma * G[0], py = sigma * G[1], pz = sigma * G[2];
    const T ph2 = px * px + py * py + pz * pz;
    T ox = sx, oy = sy, oz = sz;
    if (ph2 > T(0)) {
        T inv, sn, cs;
        angle_of<T>(ph2, inv, sn, cs);
        const T nx = px * inv, ny = py * inv, nz = pz * inv;
        const T cx = ny * sz - nz * sy;  // n x s
        const T cy = nz * sx - nx * sz;
        const T cz = nx * sy - ny * sx;
        const T sdn = sx * nx + sy * ny + sz * nz;
        const T omc = T(1) - cs;
        ox = sx * cs + cx * sn + nx * sdn * omc;
        oy = sy * cs + cy * sn + ny * sdn * omc;
        oz = sz * cs + cz * sn + nz * sdn * omc;
    }
    return renorm<T>(ox, oy, oz, sx, sy, sz);
}

// Folds m >= 0 (or NaN) into a running-maximum slot holding double bit
// patterns.  The slot only grows, so a plain read that already shows a value
// >= m, however stale, makes the atomic unnecessary: after the first kick of
// a run almost every workgroup skips it, and workgroups that finish together
// do not queue on the slot's cache line.
__device__ __forceinline__ void fold_max_slot(unsigned long long* slot, double m) {
    const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
    if (*(volatile const unsigned long long*)slot < mb) atomicMax(slot, mb);
}

// Load at a wave-uniform base plus a 32-bit per-lane byte offset.  The base
// (pinned to scalar registers) and the offset are hidden from the optimiser,
// which would otherwise fold them into a 64-bit per-lane address.
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t byte_off) {
    asm volatile("" : "+s"(base), "+v"(byte_off));
    const __attribute__((address_space(1))) char* g = (const __attribute__((address_space(1))) char*)base;
    return *(const __attribute__((address_space(1))) T*)(g + byte_off);
}


// Coordinates of site i of an Lx x Ly x Lz lattice.  Sites number fewer than
// 2^31, so two 32-bit unsigned divisions suffice (a 64-bit division is a long
// software sequence on the GPU).
__device__ __forceinline__ void site_xyz(int64_t i, int Lx, int Ly, int& x, int& y, int& z) {
    const uint32_t u = (uint32_t)i, lx = (uint32_t)Lx, ly = (uint32_t)Ly;
    const uint32_t q = u / lx;
    const uint32_t zz = q / ly;
    x = (int)(u - q * lx);
    y = (int)(q - zz * ly);
    z = (int)zz;
}

// Stage coefficients of one replica in the working precision.
template <typename T>
struct Coef {
    T cJ, cH0, cH1, cH2, cD, e0, e1, e2, lam;
};

template <typename T>
__device__ __forceinline__ Coef<T> load_coef(const RepDev& R) {
    Coef<T> c;
    c.cJ = (T)R.cJ;
    c.cH0 = (T)R.cH[0];
    c.cH1 = (T)R.cH[1];
    c.cH2 = (T)R.cH[2];
    c.cD = (T)R.cD;
    c.e0 = (T)R.e[0];
    c.e1 = (T)R.e[1];
    c.e2 = (T)R.e[2];
    c.lam = (T)R.lam;
    return c;
}

// k = dt f(s) for one site given the sum of its neighbours' spins (n).
// PREC: k = s x (h~ - lam (s x h~)), h~ = dt h; slow: k = s x (s x h~) with
// h~ = -lambda dt h (the factors are folded into the coefficients).
template <typename T, bool PREC, int ANIS>
__device__ __forceinline__ void stage_k(T sx, T sy, T sz, T nx, T ny, T nz, const Coef<T>& C,
                                        T Di, T ex, T ey, T ez, T& kx, T& ky, T& kz) {
    T hx = C.cJ * nx + C.cH0;
    T hy = C.cJ * ny + C.cH1;
    T hz = C.cJ * nz + C.cH2;
    if constexpr (ANIS == ANIS_Z) {
        hz = C.cD * sz + hz;
    } else if constexpr (ANIS == ANIS_AXIS) {
        const T c = C.cD * (sx * C.e0 + sy * C.e1 + sz * C.e2);
        hx = c * C.e0 + hx;
        hy = c * C.e1 + hy;
        hz = c * C.e2 + hz;
    } else if constexpr (ANIS == ANIS_SITE) {
        const T c = C.cD * Di * (sx * ex + sy * ey + sz * ez);
        hx = c * ex + hx;
        hy = c * ey + hy;
        hz = c * ez + hz;
    }
    const T px = sy * hz - sz * hy;
    const T py = sz * hx - sx * hz;
    const T pz = sx * hy - sy * hx;
    T gx, gy, gz;
    if constexpr (PREC) {
        gx = hx - C.lam * px;
        gy = hy - C.lam * py;
        gz = hz - C.lam * pz;
    } else {
        gx = px;
        gy = py;
        gz = pz;
    }
    kx = sy * gz - sz * gy;
    ky = sz * gx - sx * gz;
    kz = sx * gy - sy * gx;
}

__device__ __forceinline__ int wrap_coord(int v, int L) {
    v %= L;
    return v < 0 ? v + L : v;
}

}  // namespace lll
