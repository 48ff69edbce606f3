// Fused Butcher RK5 step (Appendix, six stages) in two launches.  The first
// is rk4_fused_kernel with SCHEME 3: stages 1-4 on the four-deep cone of the
// RK4 kernel, writing Y5, the partial Q6 = x + a50 k1 + ... + a53 k4 and the
// partial result R = x + b0 k1 + b2 k3 + b3 k4.  The second, below, does
// stages 5 and 6 on a two-deep cone: Y6 = Q6 + a54 k5, x' = R + b4 k5 + b5 k6,
// with the pulse-noise kick (Eqs. (5)-(6)) as an optional epilogue.  The step
// thus reads the state once and moves Y5, Q6 and R through memory once (each
// written by the first launch and read by the second), instead of the six
// launches and stage increments of the per-stage path.
#pragma once

#include "kern_fused.hpp"

namespace lll {

// Ring order of a tile grown by two sites: core BX x BY, then ring 1, ring 2
// (each stage region is a prefix of the point list).
template <int BX, int BY>
__host__ __device__ inline void ring_decode2(int idx, int& lx, int& ly) {
    if (idx < BX * BY) {
        lx = idx % BX;
        ly = idx / BX;
        return;
    }
    int j = idx - BX * BY;
    int L = 1;
    const int c1 = (BX + 2) * (BY + 2) - BX * BY;
    if (j >= c1) {
        j -= c1;
        L = 2;
    }
    const int w = BX + 2 * L, h = BY + 2 * L;
    if (j < w) {
        lx = -L + j;
        ly = -L;
    } else if (j < 2 * w) {
        lx = -L + (j - w);
        ly = BY + L - 1;
    } else {
        const int jj = j - 2 * w;
        if (jj < h - 2) {
            lx = -L;
            ly = -L + 1 + jj;
        } else {
            lx = BX + L - 1;
            ly = -L + 1 + (jj - (h - 2));
        }
    }
}

// Stages 5 and 6 of Butcher's RK5.  Each workgroup owns the output tile
// BX x BY x bz and marches along z: while plane P of Y5 (with Q6 and R) is
// loaded, stage 5 works on plane P-1 over the tile grown by one site and
// stage 6 writes plane P-2 of the tile.  Y5 and Y6 of the current plane are
// shared through LDS (double-buffered by plane parity); a point's values on
// the planes below and above stay in registers of its thread.
template <typename T, int BX, int BY, int NT, bool PREC, int ANIS, bool KICK>
__global__ void __launch_bounds__(NT)
    rk5_tail_kernel(const RepDev* __restrict__ reps, const int4* __restrict__ tiles, State y5,
                    State q6, State rr, State out, int bz_arg, uint64_t kpulse,
                    double sigma_override, unsigned long long* kickdev) {
    constexpr int R0 = (BX + 4) * (BY + 4);
    constexpr int R1 = (BX + 2) * (BY + 2);
    constexpr int R2 = BX * BY;
    constexpr int NI = (R0 + NT - 1) / NT;
    constexpr int V0 = (BX + 4) | 1, V1 = (BX + 2) | 1;
    using BT = Rk5B<T>;

    __shared__ T sB5[2][3][V0 * (BY + 4)];
    __shared__ T sB6[2][3][V1 * (BY + 2)];

    const int tid = threadIdx.x;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    const int4 tl = tiles[blockIdx.x];
    const RepDev& R = reps[tl.x];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const bool pbc = R.bc == 0;
    int bzr = bz_arg > 0 ? bz_arg : 16;
    if (bzr > Lz) bzr = Lz;
    const int x0 = tl.y * BX, y0 = tl.z * BY, z0 = tl.w * bzr;
    const int zend = min(z0 + bzr, Lz);
    // planes z0-2 .. zend+1 are loaded; padded to a multiple of four
    const int niter = (zend - z0) + 4;
    const int niter4 = (niter + 3) & ~3;
    const int64_t plane = (int64_t)Lx * Ly;
    const int64_t N = plane * Lz;
    const T* __restrict__ iy5x = static_cast<const T*>(y5.x) + R.off;
    const T* __restrict__ iy5y = static_cast<const T*>(y5.y) + R.off;
    const T* __restrict__ iy5z = static_cast<const T*>(y5.z) + R.off;
    const T* __restrict__ iq6x = static_cast<const T*>(q6.x) + R.off;
    const T* __restrict__ iq6y = static_cast<const T*>(q6.y) + R.off;
    const T* __restrict__ iq6z = static_cast<const T*>(q6.z) + R.off;
    const T* __restrict__ irx = static_cast<const T*>(rr.x) + R.off;
    const T* __restrict__ iry = static_cast<const T*>(rr.y) + R.off;
    const T* __restrict__ irz = static_cast<const T*>(rr.z) + R.off;
    T* __restrict__ ox = static_cast<T*>(out.x) + R.off;
    T* __restrict__ oy = static_cast<T*>(out.y) + R.off;
    T* __restrict__ oz = static_cast<T*>(out.z) + R.off;
    const Coef<T> C = load_coef<T>(R);
    const T* Dsite = static_cast<const T*>(R.D_site);
    const T* esite = static_cast<const T*>(R.e_site);

    int pidx[NI], pfirst[NI], o5[NI], o6[NI], r5[NI], r6[NI], col[NI];
    bool colok[NI], outok[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int idx = j * NT + tid;
        pidx[j] = idx;
        pfirst[j] = j * NT + wbase;
        int lx = 0, ly = 0;
        if (idx < R0) ring_decode2<BX, BY>(idx, lx, ly);
        o5[j] = (ly + 2) * V0 + (lx + 2);
        o6[j] = (ly + 1) * V1 + (lx + 1);
        r5[j] = idx < R1 ? o5[j] : V0 + 1;
        r6[j] = idx < R2 ? o6[j] : V1 + 1;
        int gx = x0 + lx, gy = y0 + ly;
        bool ok = idx < R0;
        if (pbc) {
            gx = wrap_coord(gx, Lx);
            gy = wrap_coord(gy, Ly);
        } else {
            ok = ok && gx >= 0 && gx < Lx && gy >= 0 && gy < Ly;
        }
        colok[j] = ok;
        col[j] = ok ? gx + Lx * gy : 0;
        outok[j] = idx < R2 && (x0 + lx) < Lx && (y0 + ly) < Ly;
    }

    // Register FIFOs by plane mod 4: Y5, Y6, Q6 (as loaded), R (loaded, then
    // + b4 k5 after stage 5); next plane's loads in the N arrays.
    T Y5F[NI][4][3], Y6F[NI][4][3], QF[NI][4][3], RF[NI][4][3];
    T Y5N[NI][3], QN[NI][3], RN[NI][3];
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) Y5F[j][s][c] = Y6F[j][s][c] = QF[j][s][c] = RF[j][s][c] = T(0);

    auto load_plane = [&](int P) {
        bool zok = true;
        int gz = P;
        if (pbc)
            gz = wrap_coord(P, Lz);
        else
            zok = P >= 0 && P < Lz;
#pragma unroll
        for (int j = 0; j < NI; ++j) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Y5N[j][c] = QN[j][c] = RN[j][c] = T(0);
            if (zok && colok[j]) {  // the only indices formed are of sites of the lattice
                const int64_t g = (int64_t)col[j] + plane * gz;
                Y5N[j][0] = iy5x[g];
                Y5N[j][1] = iy5y[g];
                Y5N[j][2] = iy5z[g];
                if (pidx[j] < R1) {  // Q6 is read where stage 5 runs
                    QN[j][0] = iq6x[g];
                    QN[j][1] = iq6y[g];
                    QN[j][2] = iq6z[g];
                }
                if (pidx[j] < R2) {  // R where stage 6 runs
                    RN[j][0] = irx[g];
                    RN[j][1] = iry[g];
                    RN[j][2] = irz[g];
                }
            }
        }
    };

    auto site_aniso = [&](int j, int q, T& Di, T& ex, T& ey, T& ez) {
        Di = T(0);
        ex = ey = ez = T(0);
        if constexpr (ANIS == ANIS_SITE) {
            int gz = q;
            bool zok = true;
            if (pbc)
                gz = wrap_coord(q, Lz);
            else
                zok = q >= 0 && q < Lz;
            if (zok && colok[j]) {
                const int64_t g = (int64_t)col[j] + plane * gz;
                Di = Dsite[g];
                ex = esite[g];
                ey = esite[N + g];
                ez = esite[2 * N + g];
            }
        }
    };

    double kmax = 0.0;
    T sg = T(0);
    uint32_t kp = 0;
    if constexpr (KICK) {
        sg = (T)(sigma_override >= 0.0 ? sigma_override : R.sigma);
        kp = (uint32_t)(kpulse + R.kbase);
    }

#define LLL_T_WAVE_IN(j, Rs) (((j) + 1) * NT <= (Rs) || pfirst[j] < (Rs))
#define LLL_T_LANE_IN(j, Rs) (((j) + 1) * NT <= (Rs) || pidx[j] < (Rs))

    // F = 0: iterations 0-3, stage 5 from iteration 2 on, no stage 6 yet
    // (its input planes exist from iteration 4); F = 1: steady state.
    auto plane_block = [&](const int t0, auto Fc) {
        constexpr int F = decltype(Fc)::value;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u;
            const int P = z0 - 2 + t;
            const int u1 = (u + 3) & 3, u2 = (u + 2) & 3, u3 = (u + 1) & 3;  // planes P-1, P-2, P-3
#pragma unroll
            for (int j = 0; j < NI; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Y5F[j][u][c] = Y5N[j][c];
                    QF[j][u][c] = QN[j][c];
                    RF[j][u][c] = RN[j][c];
                }
            {
                const int sl = t & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j)
                    if (LLL_T_LANE_IN(j, R0)) {
                        sB5[sl][0][o5[j]] = Y5F[j][u][0];
                        sB5[sl][1][o5[j]] = Y5F[j][u][1];
                        sB5[sl][2][o5[j]] = Y5F[j][u][2];
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
            load_plane(P + 1);
            // ---- stage 5 on plane P-1 (tile grown by one): Y6 = Q6 + a54 k5, R += b4 k5
            if (F == 1 || u >= 2) {
                const int sl = (t - 1) & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R1) continue;
                    if (LLL_T_WAVE_IN(j, R1)) {
                        T Di, ex, ey, ez, kx, ky, kz;
                        site_aniso(j, P - 1, Di, ex, ey, ez);
                        stage_at<T, PREC, ANIS, V0>(sB5[sl][0], sB5[sl][1], sB5[sl][2], r5[j],
                                                    Y5F[j][u1], Y5F[j][u2], Y5F[j][u], C, Di, ex, ey,
                                                    ez, kx, ky, kz);
                        const T kk[3] = {kx, ky, kz};
#pragma unroll
                        for (int c = 0; c < 3; ++c) Y6F[j][u1][c] = kk[c] * BT::a54 + QF[j][u1][c];
                        if (pfirst[j] < R2) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) RF[j][u1][c] = kk[c] * BT::b4 + RF[j][u1][c];
                        }
                        if (LLL_T_LANE_IN(j, R1)) {
                            sB6[sl][0][o6[j]] = Y6F[j][u1][0];
                            sB6[sl][1][o6[j]] = Y6F[j][u1][1];
                            sB6[sl][2][o6[j]] = Y6F[j][u1][2];
                        }
                    }
                }
            }
            // ---- stage 6 on plane P-2 (tile): x' = R + b5 k6, optional kick, store
            if (F == 1) {
                const int sl = (t - 2) & 1;
                const int gz = P - 2;
                const bool zst = gz >= z0 && gz < zend;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R2) continue;
                    if (LLL_T_WAVE_IN(j, R2)) {
                        T Di, ex, ey, ez, kx, ky, kz;
                        site_aniso(j, gz, Di, ex, ey, ez);
                        stage_at<T, PREC, ANIS, V1>(sB6[sl][0], sB6[sl][1], sB6[sl][2], r6[j],
                                                    Y6F[j][u2], Y6F[j][u3], Y6F[j][u1], C, Di, ex, ey,
                                                    ez, kx, ky, kz);
                        T rx = kx * BT::b5 + RF[j][u2][0];
                        T ry = ky * BT::b5 + RF[j][u2][1];
                        T rz = kz * BT::b5 + RF[j][u2][2];
                        if (zst && outok[j]) {
                            const int64_t g = (int64_t)col[j] + plane * gz;
                            if constexpr (KICK) {
                                const uint4 w = philox_site(R.seed, (uint32_t)g, kp, R.rid, 0u);
                                const double d = kick_spin<T>(rx, ry, rz, w, sg);
                                kmax = (d > kmax || d != d) ? d : kmax;
                            }
                            ox[g] = rx;
                            oy[g] = ry;
                            oz[g] = rz;
                        }
                    }
                }
            }
            __syncthreads();
        }
    };

    load_plane(z0 - 2);
    plane_block(0, std::integral_constant<int, 0>{});
    for (int t0 = 4; t0 < niter4; t0 += 4) plane_block(t0, std::integral_constant<int, 1>{});
#undef LLL_T_WAVE_IN
#undef LLL_T_LANE_IN
    if constexpr (KICK) {
        // tile maximum of the kick deviation, folded as in the RK4 kernel
        static_assert(NT >= 64 && NT <= 1024 && NT % 64 == 0, "threads per block");
        double v = kmax;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double c = __shfl_xor(v, o, 64);
            v = (c > v || c != c) ? c : v;
        }
        __shared__ double wred[NT / 64];
        if ((tid & 63) == 0) wred[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double m = wred[0];
#pragma unroll
            for (int w = 1; w < NT / 64; ++w) {
                const double c = wred[w];
                m = (c > m || c != c) ? c : m;
            }
            fold_max_slot(kickdev + (int64_t)tl.x * kKickSlots + (blockIdx.x & (kKickSlots - 1)), m);
        }
    }
}

// One fused RK5 step: the first launch (stages 1-4) from in into the three
// scratch states k[0] (Y5), k[1] (Q6), k[2] (R); the second (stages 5-6, kick
// when kick != 0) from them into out.
template <typename T, int BX, int BY, int NTA, int NTB, bool PREC, int ANIS>
inline hipError_t launch_rk5_v(const RepDev* reps, const int4* tiles, int ntiles, State in,
                               State out, const State* k, int bz, int kick, uint64_t kp, double so,
                               unsigned long long* kd, hipStream_t st) {
    hipLaunchKernelGGL((rk4_fused_kernel<T, BX, BY, NTA, PREC, ANIS, false, 3>), dim3(ntiles),
                       dim3(NTA), 0, st, reps, tiles, in, k[0], bz, kp, so, kd, k[1], k[2],
                       State{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (kick)
        hipLaunchKernelGGL((rk5_tail_kernel<T, BX, BY, NTB, PREC, ANIS, true>), dim3(ntiles),
                           dim3(NTB), 0, st, reps, tiles, k[0], k[1], k[2], out, bz, kp, so, kd);
    else
        hipLaunchKernelGGL((rk5_tail_kernel<T, BX, BY, NTB, PREC, ANIS, false>), dim3(ntiles),
                           dim3(NTB), 0, st, reps, tiles, k[0], k[1], k[2], out, bz, kp, so, kd);
    return hipGetLastError();
}

template <typename T, int BX, int BY, int NTA, int NTB>
inline hipError_t launch_rk5_p(int precession, int anis, const RepDev* reps, const int4* tiles,
                               int ntiles, State in, State out, const State* k, int bz, int kick,
                               uint64_t kp, double so, unsigned long long* kd, hipStream_t st) {
#define LLL_RK5_ANIS(PR)                                                                              \
    switch (anis) {                                                                                   \
        case ANIS_NONE: return launch_rk5_v<T, BX, BY, NTA, NTB, PR, ANIS_NONE>(reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st); \
        case ANIS_Z: return launch_rk5_v<T, BX, BY, NTA, NTB, PR, ANIS_Z>(reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st);       \
        case ANIS_AXIS: return launch_rk5_v<T, BX, BY, NTA, NTB, PR, ANIS_AXIS>(reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st); \
        case ANIS_SITE: return launch_rk5_v<T, BX, BY, NTA, NTB, PR, ANIS_SITE>(reps, tiles, ntiles, in, out, k, bz, kick, kp, so, kd, st); \
        default: return hipErrorInvalidValue;                                                         \
    }
    if (precession) {
        LLL_RK5_ANIS(true)
    }
    LLL_RK5_ANIS(false)
#undef LLL_RK5_ANIS
}

}  // namespace lll
