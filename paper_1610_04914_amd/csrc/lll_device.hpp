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
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
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

// Three unit normals by Box-Muller from one Philox block, u = (w + 1/2) 2^-32.
template <typename T>
__device__ __forceinline__ void gauss3(uint4 w, T G[3]);

template <>
__device__ __forceinline__ void gauss3<double>(uint4 w, double G[3]) {
    const double s = 2.3283064365386963e-10;  // 2^-32
    const double two_pi = 6.283185307179586;
    const double u0 = ((double)w.x + 0.5) * s;
    const double u1 = ((double)w.y + 0.5) * s;
    const double u2 = ((double)w.z + 0.5) * s;
    const double u3 = ((double)w.w + 0.5) * s;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double sn, cs;
    sincos(two_pi * u1, &sn, &cs);
    G[0] = r0 * cs;
    G[1] = r0 * sn;
    G[2] = r1 * cos(two_pi * u3);
}

// -ln(u) in fp32 with full relative accuracy at both ends of (0,1): for
// u >= 1/2 it is -log1p(-(1-u)) with 1-u = (~w + 1/2) 2^-32 formed exactly
// from the complemented word.
__device__ __forceinline__ float neglog_u01(uint32_t w) {
    if (w < 0x80000000u) return -logf(((float)w + 0.5f) * 2.3283064365386963e-10f);
    const uint32_t c = ~w;
    return -log1pf(-(((float)c + 0.5f) * 2.3283064365386963e-10f));
}

template <>
__device__ __forceinline__ void gauss3<float>(uint4 w, float G[3]) {
    const float r0 = sqrtf(2.0f * neglog_u01(w.x));
    const float r1 = sqrtf(2.0f * neglog_u01(w.z));
    // 2 u = (w + 1/2) 2^-31; sin/cos(pi * 2u) = sin/cos(2 pi u)
    const float a1 = ((float)w.y + 0.5f) * 4.656612873077393e-10f;
    const float a3 = ((float)w.w + 0.5f) * 4.656612873077393e-10f;
    float sn, cs;
    sincospif(a1, &sn, &cs);
    G[0] = r0 * cs;
    G[1] = r0 * sn;
    G[2] = r1 * cospif(a3);
}

template <typename T>
__device__ __forceinline__ T dsqrt(T v);
template <>
__device__ __forceinline__ double dsqrt<double>(double v) { return sqrt(v); }
template <>
__device__ __forceinline__ float dsqrt<float>(float v) { return sqrtf(v); }

template <typename T>
__device__ __forceinline__ void dsincos(T a, T* s, T* c);
template <>
__device__ __forceinline__ void dsincos<double>(double a, double* s, double* c) { sincos(a, s, c); }
template <>
__device__ __forceinline__ void dsincos<float>(float a, float* s, float* c) { sincosf(a, s, c); }

// Kick of one spin: rotation by phi = sigma G about n = phi/|phi| (Eq. (6)),
// identity when phi = 0, then renormalisation with the norm taken in fp64.
// Returns | |s'| - 1 | (fp64).  Contraction is fixed here so that the kick
// gives identical bits wherever it is inlined (separate kernel or epilogue).
template <typename T>
__device__ __forceinline__ double kick_spin(T& sx, T& sy, T& sz, uint4 w, T sigma) {
#pragma clang fp contract(off)
    T G[3];
    gauss3<T>(w, G);
    const T px = sigma * G[0], py = sigma * G[1], pz = sigma * G[2];
    const T ph2 = px * px + py * py + pz * pz;
    T ox = sx, oy = sy, oz = sz;
    if (ph2 > T(0)) {
        const T ph = dsqrt<T>(ph2);
        const T nx = px / ph, ny = py / ph, nz = pz / ph;
        T sn, cs;
        dsincos<T>(ph, &sn, &cs);
        const T cx = ny * sz - nz * sy;  // n x s
        const T cy = nz * sx - nx * sz;
        const T cz = nx * sy - ny * sx;
        const T sdn = sx * nx + sy * ny + sz * nz;
        const T omc = T(1) - cs;
        ox = sx * cs + cx * sn + nx * sdn * omc;
        oy = sy * cs + cy * sn + ny * sdn * omc;
        oz = sz * cs + cz * sn + nz * sdn * omc;
    }
    const double dx = (double)ox, dy = (double)oy, dz = (double)oz;
    const double nrm = sqrt(dx * dx + dy * dy + dz * dz);
    sx = (T)(dx / nrm);
    sy = (T)(dy / nrm);
    sz = (T)(dz / nrm);
    return fabs(nrm - 1.0);
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
