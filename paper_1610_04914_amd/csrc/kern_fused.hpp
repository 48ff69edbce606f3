// Fused classical RK4 step: one launch advances every replica of the batch
// by one step, reading the state once and writing it once.
//
// Each workgroup owns an output tile BX x BY x bz and marches along z.  The
// four stages are pipelined one plane apart: while plane P is loaded,
// stage 1 works on plane P-1, stage 2 on P-2, stage 3 on P-3 and stage 4
// writes plane P-4.  Stage s of RK4 needs its input one lattice step further
// out than stage s+1, so stage s is evaluated on the tile grown by 4-s sites
// in x and y (the "cone"); stage inputs of the current plane are shared
// through LDS, while the values of a point on the planes below/above stay in
// registers of the thread that owns the point in every stage.  Points are
// handed to threads in ring order (core first, then rings 1..4), so each
// stage's region is a prefix of the point list and idle lanes are confined to
// one partial wave per stage.  With the kick flag, the pulse-noise kick of
// Eqs. (5)-(6) is applied to the output before it is stored.
#pragma once
#include <hip/hip_ext.h>

#include <type_traits>

#include "lll_device.hpp"

namespace lll {

template <int BX, int BY>
__host__ __device__ inline void ring_decode(int idx, int& lx, int& ly) {
    if (idx < BX * BY) {
        lx = idx % BX;
        ly = idx / BX;
        return;
    }
    int base = BX * BY;
    int L = 1;
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
        const int cnt = (BX + 2 * q) * (BY + 2 * q) - (BX + 2 * q - 2) * (BY + 2 * q - 2);
        if (L == q && idx >= base + cnt) {
            base += cnt;
            L = q + 1;
        }
    }
    const int j = idx - base;
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

// Assignment of ring chunks to waves.  Workgroup waves are dealt to the four
// SIMDs round-robin; the core waves evaluate all four stages, while a ring
// chunk (64 consecutive ring points) evaluates between zero and three.  When
// one point per thread covers the whole load region, the ring chunks are
// handed to waves greedily (costliest chunk to the least loaded SIMD) so the
// SIMDs carry equal work.
template <int BX, int BY, int NT>
struct WavePlan {
    static constexpr int R4 = BX * BY;
    static constexpr int R3 = (BX + 2) * (BY + 2);
    static constexpr int R2 = (BX + 4) * (BY + 4);
    static constexpr int R1 = (BX + 6) * (BY + 6);
    static constexpr int R0 = (BX + 8) * (BY + 8);
    static constexpr int NW = NT / 64;
    static constexpr int NC = R4 / 64;
    static constexpr bool ON = (R4 % 64 == 0) && (NT >= R0) && (NW > NC);
    int chunk[16];
    static constexpr int cost(int c) {
        const int first = R4 + 64 * c;
        return (first < R1 ? 1 : 0) + (first < R2 ? 1 : 0) + (first < R3 ? 1 : 0);
    }
    constexpr WavePlan() : chunk{} {
        if (!ON) return;
        int load[4] = {0, 0, 0, 0};
        for (int w = 0; w < NC; ++w) load[w % 4] += 4;
        const int nring = NW - NC;
        bool used[16] = {};
        bool taken[16] = {};
        for (int pass = 0; pass < nring; ++pass) {
            int bc = -1, bcost = -1;
            for (int c = 0; c < nring; ++c)
                if (!used[c] && cost(c) > bcost) {
                    bcost = cost(c);
                    bc = c;
                }
            int bk = -1, bload = 1 << 30;
            for (int k = 0; k < nring; ++k)
                if (!taken[k] && load[(NC + k) % 4] < bload) {
                    bload = load[(NC + k) % 4];
                    bk = k;
                }
            used[bc] = true;
            taken[bk] = true;
            chunk[bk] = bc;
            load[(NC + bk) % 4] += bcost;
        }
    }
};

// k of one stage at a point whose own values on the planes below/at/above
// are zm, c, zp, with the four in-plane neighbours read from the LDS plane
// (L0, L1, L2) of frame width W at offset o.
template <typename T, bool PREC, int ANIS, int W>
__device__ __forceinline__ void stage_at(const T* L0, const T* L1, const T* L2, int o, const T* c,
                                         const T* zm, const T* zp, const Coef<T>& C, T Di, T ex,
                                         T ey, T ez, T& kx, T& ky, T& kz) {
    const T nx = (L0[o - 1] + L0[o + 1]) + (L0[o - W] + L0[o + W]) + (zm[0] + zp[0]);
    const T ny = (L1[o - 1] + L1[o + 1]) + (L1[o - W] + L1[o + W]) + (zm[1] + zp[1]);
    const T nz = (L2[o - 1] + L2[o + 1]) + (L2[o - W] + L2[o + W]) + (zm[2] + zp[2]);
    stage_k<T, PREC, ANIS>(c[0], c[1], c[2], nx, ny, nz, C, Di, ex, ey, ez, kx, ky, kz);
}

// Coefficients of Butcher's six-stage fifth-order method (Appendix): stage
// inputs Y_{i+1} = x + sum_j a_ij k_j, result x' = x + sum_i b_i k_i.
template <typename T>
struct Rk5B {
    static constexpr T a10 = T(1) / T(4), a20 = T(1) / T(8), a21 = T(1) / T(8);
    static constexpr T a31 = T(-1) / T(2), a32 = T(1);
    static constexpr T a40 = T(3) / T(16), a43 = T(9) / T(16);
    static constexpr T a50 = T(-3) / T(7), a51 = T(2) / T(7), a52 = T(12) / T(7),
                       a53 = T(-12) / T(7), a54 = T(8) / T(7);
    static constexpr T b0 = T(7) / T(90), b2 = T(32) / T(90), b3 = T(12) / T(90),
                       b4 = T(32) / T(90), b5 = T(7) / T(90);
};

// SCHEME 0: one classical RK4 step.  SCHEME 1: two RK2-midpoint steps, whose
// four stage evaluations have the same dependency depth (y2 = x + k1/2,
// x1 = x + k2, y4 = x1 + k3/2, x2 = x1 + k4).  SCHEME 2: one RK2-midpoint step
// (stages 1 and 2 only; x1 is the output).  SCHEME 3: the first four stages
// of Butcher's RK5 (the second launch, rk5_tail_kernel, does stages 5 and 6):
// Y2 = x + a10 k1, Y3 = P3 + a21 k2 with P3 = x + a20 k1, Y4 = P4 + a32 k3
// with P4 = x + a31 k2; per point the partial sums P5 = x + a40 k1,
// Q6 = x + a50 k1 + a51 k2 + a52 k3 (+ a53 k4) and R = x + b0 k1 + b2 k3
// (+ b3 k4) ride along, and the last stage writes Y5 = P5 + a43 k4 to out,
// Q6 to out2 and R to out3 (b1 = 0).  SCHEME 4: one classical RK4 step, as
// SCHEME 0 and with the same bits, that also writes its stage inputs y2, y3
// and y4 of the output tile to out2, out3 and out4 (the discrete adjoint's
// recompute of a checkpoint block needs them).
template <typename T, int BX, int BY, int NT, bool PREC, int ANIS, bool KICK, int SCHEME>
__global__ void __launch_bounds__(NT)
    rk4_fused_kernel(const RepDev* __restrict__ reps, const int4* __restrict__ tiles, State in,
                     State out, int bz_arg, uint64_t kpulse, double sigma_override,
                     unsigned long long* kickdev, State out2, State out3, State out4) {
    constexpr bool RK4S = SCHEME == 0 || SCHEME == 4;  // classical RK4 arithmetic
    // Region Rs = the tile grown by 4-s sites in x and y (R0: loaded points).
    constexpr int R0 = (BX + 8) * (BY + 8);
    constexpr int R1 = (BX + 6) * (BY + 6);
    constexpr int R2 = (BX + 4) * (BY + 4);
    constexpr int R3 = (BX + 2) * (BY + 2);
    constexpr int R4 = BX * BY;
    constexpr int NI = (R0 + NT - 1) / NT;
    // LDS row pitches: the frame widths rounded up to odd, so that points of
    // a ring column (one row apart) fall in distinct LDS banks.
    constexpr int W0 = (BX + 8) | 1, W1 = (BX + 6) | 1, W2 = (BX + 4) | 1, W3 = (BX + 2) | 1;

    // Stage-input planes, double-buffered by plane parity: A1 = x on the
    // load region, A2 = y2 on R1, A3 = y3 on R2, A4 = y4 on R3.
    __shared__ T sA1[2][3][W0 * (BY + 8)];
    __shared__ T sA2[2][3][W1 * (BY + 6)];
    __shared__ T sA3[2][3][W2 * (BY + 4)];
    __shared__ T sA4[2][3][W3 * (BY + 2)];

    const int tid = threadIdx.x;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // first thread of this wave
    const int4 tl = tiles[blockIdx.x];
    const RepDev& R = reps[tl.x];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const bool pbc = R.bc == 0;
    int bzr = bz_arg > 0 ? bz_arg : 16;
    if (bzr > Lz) bzr = Lz;
    const int x0 = tl.y * BX, y0 = tl.z * BY, z0 = tl.w * bzr;
    const int zend = min(z0 + bzr, Lz);
    // Planes z0-4 .. zend+3 are loaded; the trip count is padded to a multiple
    // of four (the padding computes planes whose results are never stored).
    const int niter = (zend - z0) + 8;
    const int niter4 = (niter + 3) & ~3;
    const int64_t plane = (int64_t)Lx * Ly;
    const int64_t N = plane * Lz;
    const T* __restrict__ ix = static_cast<const T*>(in.x) + R.off;
    const T* __restrict__ iy = static_cast<const T*>(in.y) + R.off;
    const T* __restrict__ iz = static_cast<const T*>(in.z) + R.off;
    T* __restrict__ ox = static_cast<T*>(out.x) + R.off;
    T* __restrict__ oy = static_cast<T*>(out.y) + R.off;
    T* __restrict__ oz = static_cast<T*>(out.z) + R.off;
    const Coef<T> C = load_coef<T>(R);
    const T* Dsite = static_cast<const T*>(R.D_site);
    const T* esite = static_cast<const T*>(R.e_site);

    // Per point: LDS offsets of its own value in frames A1..A4 (written by the
    // stage that produces it), read offsets (its own offset inside the stage's
    // region, else a harmless interior point), global column, flags.
    // pidx: point index of this thread's item j; pfirst: lowest point index of
    // the wave's item j (wave-uniform).
    using Plan = WavePlan<BX, BY, NT>;
    constexpr Plan plan{};
    int pidx[NI], pfirst[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        pidx[j] = j * NT + tid;
        pfirst[j] = j * NT + wbase;
    }
    if constexpr (Plan::ON) {
        const int wave = wbase >> 6;
        if (wave >= Plan::NC) {
            // select by compile-time index: a run-time index into the plan
            // would place the whole table in per-lane private memory
            int ch = 0;
#pragma unroll
            for (int q = 0; q < Plan::NW - Plan::NC; ++q)
                if (wave - Plan::NC == q) ch = plan.chunk[q];
            pfirst[0] = R4 + 64 * ch;
            pidx[0] = pfirst[0] + (tid & 63);
        }
    }
    int o1[NI], o2[NI], o3[NI], o4[NI];
    int r1[NI], r2[NI], r3[NI], r4[NI];
    int col[NI];
    bool colok[NI], outok[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int idx = pidx[j];
        int lx = 0, ly = 0;
        if (idx < R0) ring_decode<BX, BY>(idx, lx, ly);
        o1[j] = (ly + 4) * W0 + (lx + 4);
        o2[j] = (ly + 3) * W1 + (lx + 3);
        o3[j] = (ly + 2) * W2 + (lx + 2);
        o4[j] = (ly + 1) * W3 + (lx + 1);
        r1[j] = idx < R1 ? o1[j] : W0 + 1;
        r2[j] = idx < R2 ? o2[j] : W1 + 1;
        r3[j] = idx < R3 ? o3[j] : W2 + 1;
        r4[j] = idx < R4 ? o4[j] : W3 + 1;
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
        outok[j] = idx < R4 && (x0 + lx) < Lx && (y0 + ly) < Ly;
    }

    // Register FIFOs indexed by plane mod 4: x, stage inputs y2..y4, RK4 accumulator.
    T X[NI][4][3], Y2[NI][4][3], Y3[NI][4][3], Y4[NI][4][3], A[NI][4][3], XN[NI][3];
    // SCHEME 3: the partial sums (P3, P4 by plane parity; P5, Q6, R by plane mod 4)
    constexpr int N5 = SCHEME == 3 ? NI : 1;
    T P3[N5][2][3], P4[N5][2][3], P5[N5][4][3], Q6[N5][4][3], RR[N5][4][3];
    using BT = Rk5B<T>;
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) X[j][s][c] = Y2[j][s][c] = Y3[j][s][c] = Y4[j][s][c] = A[j][s][c] = T(0);

    auto load_plane = [&](int P) {
        bool zok = true;
        int gz = P;
        if (pbc)
            gz = wrap_coord(P, Lz);
        else
            zok = P >= 0 && P < Lz;
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            if (zok && colok[j]) {
                const int64_t g = (int64_t)col[j] + plane * gz;
                XN[j][0] = ix[g];
                XN[j][1] = iy[g];
                XN[j][2] = iz[g];
            } else {
                XN[j][0] = T(0);
                XN[j][1] = T(0);
                XN[j][2] = T(0);
            }
        }
    };

    // per-site anisotropy of point j on plane q (zero outside the lattice)
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

    // SCHEME 4: a stage input of output-tile point j on plane q, stored when the
    // plane belongs to this tile's z-chunk
    auto store_core = [&](int j, int q, const State& dst, const T* v) {
        if (j * NT < R4 && pidx[j] < R4 && outok[j] && q >= z0 && q < zend) {
            const int64_t g = R.off + (int64_t)col[j] + plane * q;
            static_cast<T*>(dst.x)[g] = v[0];
            static_cast<T*>(dst.y)[g] = v[1];
            static_cast<T*>(dst.z)[g] = v[2];
        }
    };

    const T c6 = T(1) / T(6), c3 = T(1) / T(3), c2 = T(0.5);
    double kmax = 0.0;
    T sg = T(0);
    uint32_t kp = 0;  // Philox counter word 1 of this launch's kick
    if constexpr (KICK) {
        sg = (T)(sigma_override >= 0.0 ? sigma_override : R.sigma);
        kp = (uint32_t)(kpulse + R.kbase);
    }

    // Item j's points cover stage region Rs entirely (compile time), or this
    // wave holds at least one of its points (wave-uniform).
#define LLL_ITEM_WAVE_IN(j, Rs) (((j) + 1) * NT <= (Rs) || pfirst[j] < (Rs))
#define LLL_ITEM_LANE_IN(j, Rs) (((j) + 1) * NT <= (Rs) || pidx[j] < (Rs))

    // Four planes per block (FIFO slots are then compile-time).  F = 0, 1:
    // iterations 0-3 and 4-7, where stage s runs only from iteration 2s on (its
    // input planes exist from then; earlier results would never be used);
    // F = 2: the steady state, all four stages every iteration.
    auto plane_block = [&](const int t0, auto Fc) {
        constexpr int F = decltype(Fc)::value;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u;
            const int P = z0 - 4 + t;
            const int u1 = (u + 3) & 3, u2 = (u + 2) & 3, u3 = (u + 1) & 3;  // planes P-1, P-2, P-3
            // ---- commit x(P) (loaded one plane ago) to registers and LDS, then
            // issue the loads of x(P+1); the scheduling barrier keeps the new
            // loads behind the LDS stores, so the stores wait only for the
            // previous plane's loads and the new ones stay in flight.
#pragma unroll
            for (int j = 0; j < NI; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) X[j][u][c] = XN[j][c];
            {
                const int sl = t & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (LLL_ITEM_LANE_IN(j, R0)) {
                        sA1[sl][0][o1[j]] = X[j][u][0];
                        sA1[sl][1][o1[j]] = X[j][u][1];
                        sA1[sl][2][o1[j]] = X[j][u][2];
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            load_plane(P + 1);
            // ---- stage 1 on plane P-1 (region R1); k1, y2 = x + k1/2, acc = x + k1/6
            if (F == 2 || 4 * F + u >= 2 * 1) {
                const int sl = (t - 1) & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R1) continue;
                    if (LLL_ITEM_WAVE_IN(j, R1)) {
                        T Di, ex, ey, ez, kx, ky, kz;
                        site_aniso(j, P - 1, Di, ex, ey, ez);
                        stage_at<T, PREC, ANIS, W0>(sA1[sl][0], sA1[sl][1], sA1[sl][2], r1[j], X[j][u1],
                                                    X[j][u2], X[j][u], C, Di, ex, ey, ez, kx, ky, kz);
                        if constexpr (SCHEME == 3) {
                            const T kk[3] = {kx, ky, kz};
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                Y2[j][u1][c] = kk[c] * BT::a10 + X[j][u1][c];
                                P3[j][u1 & 1][c] = kk[c] * BT::a20 + X[j][u1][c];
                            }
                            if (pfirst[j] < R4) {  // the partial sums serve the core only
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    P5[j][u1][c] = kk[c] * BT::a40 + X[j][u1][c];
                                    Q6[j][u1][c] = kk[c] * BT::a50 + X[j][u1][c];
                                    RR[j][u1][c] = kk[c] * BT::b0 + X[j][u1][c];
                                }
                            }
                        } else {
                            Y2[j][u1][0] = kx * c2 + X[j][u1][0];
                            Y2[j][u1][1] = ky * c2 + X[j][u1][1];
                            Y2[j][u1][2] = kz * c2 + X[j][u1][2];
                        }
                        if (RK4S && j * NT < R4) {
                            A[j][u1][0] = kx * c6 + X[j][u1][0];
                            A[j][u1][1] = ky * c6 + X[j][u1][1];
                            A[j][u1][2] = kz * c6 + X[j][u1][2];
                        }
                        if (LLL_ITEM_LANE_IN(j, R1)) {
                            sA2[sl][0][o2[j]] = Y2[j][u1][0];
                            sA2[sl][1][o2[j]] = Y2[j][u1][1];
                            sA2[sl][2][o2[j]] = Y2[j][u1][2];
                        }
                        if constexpr (SCHEME == 4) store_core(j, P - 1, out2, Y2[j][u1]);
                    }
                }
            }
            // ---- stage 2 on plane P-2 (region R2); y3 = x + k2/2, acc += k2/3
            if (F == 2 || 4 * F + u >= 2 * 2) {
                const int sl = (t - 2) & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R2) continue;
                    if (LLL_ITEM_WAVE_IN(j, R2)) {
                        T Di, ex, ey, ez, kx, ky, kz;
                        site_aniso(j, P - 2, Di, ex, ey, ez);
                        stage_at<T, PREC, ANIS, W1>(sA2[sl][0], sA2[sl][1], sA2[sl][2], r2[j], Y2[j][u2],
                                                    Y2[j][u3], Y2[j][u1], C, Di, ex, ey, ez, kx, ky, kz);
                        if constexpr (RK4S) {
                            Y3[j][u2][0] = kx * c2 + X[j][u2][0];
                            Y3[j][u2][1] = ky * c2 + X[j][u2][1];
                            Y3[j][u2][2] = kz * c2 + X[j][u2][2];
                            if (j * NT < R4) {
                                A[j][u2][0] = kx * c3 + A[j][u2][0];
                                A[j][u2][1] = ky * c3 + A[j][u2][1];
                                A[j][u2][2] = kz * c3 + A[j][u2][2];
                            }
                        } else if constexpr (SCHEME == 3) {
                            const T kk[3] = {kx, ky, kz};
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                Y3[j][u2][c] = kk[c] * BT::a21 + P3[j][u2 & 1][c];
                                P4[j][u2 & 1][c] = kk[c] * BT::a31 + X[j][u2][c];
                            }
                            if (pfirst[j] < R4) {
#pragma unroll
                                for (int c = 0; c < 3; ++c) Q6[j][u2][c] = kk[c] * BT::a51 + Q6[j][u2][c];
                            }
                        } else {  // x1 = x + k2
                            Y3[j][u2][0] = kx + X[j][u2][0];
                            Y3[j][u2][1] = ky + X[j][u2][1];
                            Y3[j][u2][2] = kz + X[j][u2][2];
                        }
                        if (SCHEME != 2 && LLL_ITEM_LANE_IN(j, R2)) {
                            sA3[sl][0][o3[j]] = Y3[j][u2][0];
                            sA3[sl][1][o3[j]] = Y3[j][u2][1];
                            sA3[sl][2][o3[j]] = Y3[j][u2][2];
                        }
                        if constexpr (SCHEME == 4) store_core(j, P - 2, out3, Y3[j][u2]);
                    }
                }
            }
            // ---- stage 3 on plane P-3 (region R3); y4 = x + k3, acc += k3/3
            if (SCHEME != 2 && (F == 2 || 4 * F + u >= 2 * 3)) {
                const int sl = (t - 3) & 1;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R3) continue;
                    if (LLL_ITEM_WAVE_IN(j, R3)) {
                        T Di, ex, ey, ez, kx, ky, kz;
                        site_aniso(j, P - 3, Di, ex, ey, ez);
                        stage_at<T, PREC, ANIS, W2>(sA3[sl][0], sA3[sl][1], sA3[sl][2], r3[j], Y3[j][u3],
                                                    Y3[j][u], Y3[j][u2], C, Di, ex, ey, ez, kx, ky, kz);
                        if constexpr (RK4S) {
                            Y4[j][u3][0] = kx + X[j][u3][0];
                            Y4[j][u3][1] = ky + X[j][u3][1];
                            Y4[j][u3][2] = kz + X[j][u3][2];
                            if (j * NT < R4) {
                                A[j][u3][0] = kx * c3 + A[j][u3][0];
                                A[j][u3][1] = ky * c3 + A[j][u3][1];
                                A[j][u3][2] = kz * c3 + A[j][u3][2];
                            }
                        } else if constexpr (SCHEME == 3) {  // a32 = 1
                            const T kk[3] = {kx, ky, kz};
#pragma unroll
                            for (int c = 0; c < 3; ++c) Y4[j][u3][c] = kk[c] + P4[j][u3 & 1][c];
                            if (pfirst[j] < R4) {
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    Q6[j][u3][c] = kk[c] * BT::a52 + Q6[j][u3][c];
                                    RR[j][u3][c] = kk[c] * BT::b2 + RR[j][u3][c];
                                }
                            }
                        } else {  // y4 = x1 + k3/2
                            Y4[j][u3][0] = kx * c2 + Y3[j][u3][0];
                            Y4[j][u3][1] = ky * c2 + Y3[j][u3][1];
                            Y4[j][u3][2] = kz * c2 + Y3[j][u3][2];
                        }
                        if (LLL_ITEM_LANE_IN(j, R3)) {
                            sA4[sl][0][o4[j]] = Y4[j][u3][0];
                            sA4[sl][1][o4[j]] = Y4[j][u3][1];
                            sA4[sl][2][o4[j]] = Y4[j][u3][2];
                        }
                        if constexpr (SCHEME == 4) store_core(j, P - 3, out4, Y4[j][u3]);
                    }
                }
            }
            // ---- stage 4 on plane P-4 (core): x' = acc + k4/6, optional kick, store
            if (F == 2 || 4 * F + u >= 2 * 4) {
                const int sl = (t - 4) & 1;
                const int gz = P - 4;
                const bool zst = gz >= z0 && gz < zend;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if (j * NT >= R4) continue;
                    if (LLL_ITEM_WAVE_IN(j, R4)) {
                        T rx, ry, rz;
                        if constexpr (SCHEME == 2) {  // output x1
                            rx = Y3[j][u][0];
                            ry = Y3[j][u][1];
                            rz = Y3[j][u][2];
                        } else {
                            T Di, ex, ey, ez, kx, ky, kz;
                            site_aniso(j, gz, Di, ex, ey, ez);
                            stage_at<T, PREC, ANIS, W3>(sA4[sl][0], sA4[sl][1], sA4[sl][2], r4[j],
                                                        Y4[j][u], Y4[j][u1], Y4[j][u3], C, Di, ex,
                                                        ey, ez, kx, ky, kz);
                            if constexpr (RK4S) {
                                rx = kx * c6 + A[j][u][0];
                                ry = ky * c6 + A[j][u][1];
                                rz = kz * c6 + A[j][u][2];
                            } else if constexpr (SCHEME == 3) {  // Y5; Q6 and R finished
                                rx = kx * BT::a43 + P5[j][u][0];
                                ry = ky * BT::a43 + P5[j][u][1];
                                rz = kz * BT::a43 + P5[j][u][2];
                                Q6[j][u][0] = kx * BT::a53 + Q6[j][u][0];
                                Q6[j][u][1] = ky * BT::a53 + Q6[j][u][1];
                                Q6[j][u][2] = kz * BT::a53 + Q6[j][u][2];
                                RR[j][u][0] = kx * BT::b3 + RR[j][u][0];
                                RR[j][u][1] = ky * BT::b3 + RR[j][u][1];
                                RR[j][u][2] = kz * BT::b3 + RR[j][u][2];
                            } else {  // x2 = x1 + k4
                                rx = kx + Y3[j][u][0];
                                ry = ky + Y3[j][u][1];
                                rz = kz + Y3[j][u][2];
                            }
                        }
                        if (zst && outok[j]) {
                            const int64_t g = (int64_t)col[j] + plane * gz;
                            if constexpr (KICK) {
                                const uint4 w =
                                    philox_site(R.seed, (uint32_t)g, kp, R.rid, 0u);
                                const double d = kick_spin<T>(rx, ry, rz, w, sg);
                                kmax = (d > kmax || d != d) ? d : kmax;
                            }
                            ox[g] = rx;
                            oy[g] = ry;
                            oz[g] = rz;
                            if constexpr (SCHEME == 3) {
                                static_cast<T*>(out2.x)[R.off + g] = Q6[j][u][0];
                                static_cast<T*>(out2.y)[R.off + g] = Q6[j][u][1];
                                static_cast<T*>(out2.z)[R.off + g] = Q6[j][u][2];
                                static_cast<T*>(out3.x)[R.off + g] = RR[j][u][0];
                                static_cast<T*>(out3.y)[R.off + g] = RR[j][u][1];
                                static_cast<T*>(out3.z)[R.off + g] = RR[j][u][2];
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    };

    load_plane(z0 - 4);
    plane_block(0, std::integral_constant<int, 0>{});
    plane_block(4, std::integral_constant<int, 1>{});
    for (int t0 = 8; t0 < niter4; t0 += 4) plane_block(t0, std::integral_constant<int, 2>{});
#undef LLL_ITEM_WAVE_IN
#undef LLL_ITEM_LANE_IN
    if constexpr (KICK) {
        // Tile maximum of the renormalisation deviation (a NaN compares above
        // all): butterfly over each wave, thread 0 over the wave maxima, then one
        // integer atomic max per tile into one of the replica's running-maximum
        // slots (spread by workgroup, so that the tiles finishing together do
        // not queue on one address).  The deviation is >= 0 (or NaN), and such
        // doubles order as their bit patterns do, NaN above +inf.
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

template <typename T, int BX, int BY, int NT, bool PREC, int ANIS, int SCHEME>
inline hipError_t launch_v(const RepDev* reps, const int4* tiles, int ntiles, State in, State out,
                           int bz, int kick, uint64_t k, double so, unsigned long long* kd,
                           const LaunchEvents* ev, hipStream_t st) {
    const State none{};
    if (kick)
        hipLaunchKernelGGL((rk4_fused_kernel<T, BX, BY, NT, PREC, ANIS, true, SCHEME>), dim3(ntiles),
                           dim3(NT), 0, st, reps, tiles, in, out, bz, k, so, kd, none, none, none);
    else if (ev)  // start/stop events taken from the dispatch itself
        hipExtLaunchKernelGGL((rk4_fused_kernel<T, BX, BY, NT, PREC, ANIS, false, SCHEME>),
                              dim3(ntiles), dim3(NT), 0, st, ev->start, ev->stop, 0, reps, tiles, in,
                              out, bz, k, so, kd, none, none, none);
    else
        hipLaunchKernelGGL((rk4_fused_kernel<T, BX, BY, NT, PREC, ANIS, false, SCHEME>), dim3(ntiles),
                           dim3(NT), 0, st, reps, tiles, in, out, bz, k, so, kd, none, none, none);
    return hipGetLastError();
}

template <typename T, int BX, int BY, int NT, bool PREC, int SCHEME>
inline hipError_t launch_a(int anis, const RepDev* reps, const int4* tiles, int ntiles, State in,
                           State out, int bz, int kick, uint64_t k, double so,
                           unsigned long long* kd, const LaunchEvents* ev, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: return launch_v<T, BX, BY, NT, PREC, ANIS_NONE, SCHEME>(reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case ANIS_Z: return launch_v<T, BX, BY, NT, PREC, ANIS_Z, SCHEME>(reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case ANIS_AXIS: return launch_v<T, BX, BY, NT, PREC, ANIS_AXIS, SCHEME>(reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        case ANIS_SITE: return launch_v<T, BX, BY, NT, PREC, ANIS_SITE, SCHEME>(reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int BX, int BY, int NT, int SCHEME>
inline hipError_t launch_p(int precession, int anis, const RepDev* reps, const int4* tiles,
                           int ntiles, State in, State out, int bz, int kick, uint64_t k,
                           double so, unsigned long long* kd, const LaunchEvents* ev, hipStream_t st) {
    if (precession)
        return launch_a<T, BX, BY, NT, true, SCHEME>(anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
    return launch_a<T, BX, BY, NT, false, SCHEME>(anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st);
}

// One RK4 step (SCHEME 4) from in to out that also writes the stage inputs
// y2, y3, y4 (no kick).
template <typename T, int BX, int BY, int NT>
inline hipError_t launch_stages_v(int precession, int anis, const RepDev* reps, const int4* tiles,
                                  int ntiles, State in, State out, const State* y, int bz,
                                  hipStream_t st) {
#define LLL_ST_LAUNCH(PR, AN)                                                                          \
    hipLaunchKernelGGL((rk4_fused_kernel<T, BX, BY, NT, PR, AN, false, 4>), dim3(ntiles), dim3(NT), 0, \
                       st, reps, tiles, in, out, bz, (uint64_t)0, -1.0, (unsigned long long*)nullptr,  \
                       y[0], y[1], y[2]);                                                              \
    break;
#define LLL_ST_ANIS(PR)                                             \
    switch (anis) {                                                 \
        case ANIS_NONE: LLL_ST_LAUNCH(PR, ANIS_NONE)                \
        case ANIS_Z: LLL_ST_LAUNCH(PR, ANIS_Z)                      \
        case ANIS_AXIS: LLL_ST_LAUNCH(PR, ANIS_AXIS)                \
        case ANIS_SITE: LLL_ST_LAUNCH(PR, ANIS_SITE)                \
        default: return hipErrorInvalidValue;                       \
    }
    if (precession) {
        LLL_ST_ANIS(true)
    } else {
        LLL_ST_ANIS(false)
    }
#undef LLL_ST_ANIS
#undef LLL_ST_LAUNCH
    return hipGetLastError();
}

// Tile variants (bx, by, threads) by precision, for one scheme.  The same
// lists give the variant table (kern_fused_f32.hip).
#define LLL_FUSED_ARGS                                                                    \
    int precession, int anis, int variant, int bz, const RepDev *reps, const int4 *tiles, \
        int ntiles, State in, State out, int kick, uint64_t k, double so, unsigned long long *kd,     \
        const LaunchEvents *ev, hipStream_t st
#define LLL_FUSED_PASS precession, anis, reps, tiles, ntiles, in, out, bz, kick, k, so, kd, ev, st

template <int SCHEME>
inline hipError_t fused_f32(LLL_FUSED_ARGS) {
    switch (variant) {
        case 1: return launch_p<float, 32, 16, 960, SCHEME>(LLL_FUSED_PASS);
        case 2: return launch_p<float, 32, 16, 512, SCHEME>(LLL_FUSED_PASS);
        case 3: return launch_p<float, 16, 16, 576, SCHEME>(LLL_FUSED_PASS);
        case 4: return launch_p<float, 32, 8, 640, SCHEME>(LLL_FUSED_PASS);
        case 5: return launch_p<float, 64, 8, 512, SCHEME>(LLL_FUSED_PASS);
        case 6: return launch_p<float, 32, 16, 1024, SCHEME>(LLL_FUSED_PASS);
        default: return hipErrorInvalidValue;
    }
}

template <int SCHEME>
inline hipError_t fused_f64(LLL_FUSED_ARGS) {
    switch (variant) {
        case 1: return launch_p<double, 32, 8, 640, SCHEME>(LLL_FUSED_PASS);
        case 2: return launch_p<double, 16, 16, 576, SCHEME>(LLL_FUSED_PASS);
        case 3: return launch_p<double, 16, 16, 256, SCHEME>(LLL_FUSED_PASS);
        case 4: return launch_p<double, 32, 8, 256, SCHEME>(LLL_FUSED_PASS);
        case 5: return launch_p<double, 16, 8, 384, SCHEME>(LLL_FUSED_PASS);
        case 6: return launch_p<double, 16, 16, 512, SCHEME>(LLL_FUSED_PASS);
        case 7: return launch_p<double, 32, 8, 512, SCHEME>(LLL_FUSED_PASS);
        default: return hipErrorInvalidValue;
    }
}

// One function per translation unit (schemes are split across them).
hipError_t fused_f32_rk4(LLL_FUSED_ARGS);
hipError_t fused_f64_rk4(LLL_FUSED_ARGS);
hipError_t fused_f32_rk2(int scheme, LLL_FUSED_ARGS);
hipError_t fused_f64_rk2(int scheme, LLL_FUSED_ARGS);

}  // namespace lll
