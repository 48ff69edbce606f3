// Per-site kernels of the pulse-noise path: random words, initial states,
// the pulse-noise kick, fp64 observables, and the unfused RK4 step (one
// launch per Runge-Kutta stage, used for small lattices and as a tuning
// candidate).
#include "lll_device.hpp"
#include "lll_site.hpp"

namespace lll {

constexpr int kSiteBlock = 256;
constexpr int kObsBlock = 256;

// ------------------------------------------------------------------ words --
__global__ void __launch_bounds__(256) philox_words_kernel(uint64_t seed, uint32_t i0, int64_t n,
                                                           uint32_t c1, uint32_t c2, uint32_t c3,
                                                           uint32_t* out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint4 w = philox_site(seed, i0 + (uint32_t)j, c1, c2, c3);
    out[4 * j + 0] = w.x;
    out[4 * j + 1] = w.y;
    out[4 * j + 2] = w.z;
    out[4 * j + 3] = w.w;
}

hipError_t launch_philox_words(uint64_t seed, uint32_t i0, int64_t n, uint32_t c1, uint32_t c2,
                               uint32_t c3, uint32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)nb), dim3(256), 0, st, seed, i0, n, c1,
                       c2, c3, out);
    return hipGetLastError();
}

// Site owned by this thread in a per-site launch: block b belongs to replica
// blk_rep[b]; returns false past the replica's last site.
struct SiteCtx {
    int r;
    int64_t i;   // site within the replica
    int64_t gi;  // site in the packed arrays
};

__device__ __forceinline__ bool site_of_thread(const RepDev* reps, const int32_t* blk_rep,
                                               SiteCtx& c) {
    const int b = blockIdx.x;
    c.r = blk_rep[b];
    const RepDev& R = reps[c.r];
    const int64_t N = (int64_t)R.Lx * R.Ly * R.Lz;
    c.i = (int64_t)(b - R.sb0) * kSiteBlock + threadIdx.x;
    c.gi = R.off + c.i;
    return c.i < N;
}

// ------------------------------------------------------------------ init ---
// Random sphere: Philox (i, 0, r, tag 1), z = 2 u0 - 1, azimuth 2 pi u1.
template <typename T>
__global__ void __launch_bounds__(kSiteBlock)
    init_kernel(const RepDev* reps, const int32_t* blk_rep, State s, double dx, double dy,
                double dz) {
    SiteCtx c;
    if (!site_of_thread(reps, blk_rep, c)) return;
    const RepDev& R = reps[c.r];
    double x, y, z;
    if (R.init == 0) {
        const uint4 w = philox_site(R.seed, (uint32_t)c.i, 0u, R.rid, 1u);
        const double sc = 2.3283064365386963e-10;
        z = 2.0 * (((double)w.x + 0.5) * sc) - 1.0;
        const double ph = 6.283185307179586 * (((double)w.y + 0.5) * sc);
        const double rho = sqrt(1.0 - __dmul_rn(z, z));  // z*z rounded, as in the definition
        double sn, cs;
        sincos(ph, &sn, &cs);
        x = rho * cs;
        y = rho * sn;
    } else {
        x = dx;
        y = dy;
        z = dz;
    }
    static_cast<T*>(s.x)[c.gi] = (T)x;
    static_cast<T*>(s.y)[c.gi] = (T)y;
    static_cast<T*>(s.z)[c.gi] = (T)z;
}

hipError_t launch_init(int prec, const RepDev* reps, const int32_t* blk_rep, int nblk, State s,
                       int mode, double dx, double dy, double dz, hipStream_t st) {
    (void)mode;
    if (nblk <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(init_kernel<double>, dim3(nblk), dim3(kSiteBlock), 0, st, reps, blk_rep,
                           s, dx, dy, dz);
    else
        hipLaunchKernelGGL(init_kernel<float>, dim3(nblk), dim3(kSiteBlock), 0, st, reps, blk_rep,
                           s, dx, dy, dz);
    return hipGetLastError();
}

// ------------------------------------------------------------------ kick ---
// NaN-propagating max / min (a NaN operand wins).
__device__ __forceinline__ double nan_max(double a, double c) { return (c > a || c != c) ? c : a; }
__device__ __forceinline__ double nan_min(double a, double c) { return (c < a || c != c) ? c : a; }

// Maximum over a block of 256 threads (a NaN compares above all): butterfly
// over each wave, then the four wave results; valid in every thread.
__device__ __forceinline__ double block_max256(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
    __shared__ double wred[4];
    if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = v;
    __syncthreads();
    return nan_max(nan_max(wred[0], wred[1]), nan_max(wred[2], wred[3]));
}

template <typename T>
__global__ void __launch_bounds__(kSiteBlock)
    kick_kernel(const RepDev* reps, const int32_t* blk_rep, State s, uint64_t k,
                double sigma_override, unsigned long long* kickdev) {
    SiteCtx c;
    const bool live = site_of_thread(reps, blk_rep, c);
    double dev = 0.0;
    if (live) {
        const RepDev& R = reps[c.r];
        const double sg = sigma_override >= 0.0 ? sigma_override : R.sigma;
        const uint4 w = philox_site(R.seed, (uint32_t)c.i, (uint32_t)(k + R.kbase), R.rid, 0u);
        T* px = static_cast<T*>(s.x);
        T* py = static_cast<T*>(s.y);
        T* pz = static_cast<T*>(s.z);
        T x = px[c.gi], y = py[c.gi], z = pz[c.gi];
        dev = kick_spin<T>(x, y, z, w, (T)sg);
        px[c.gi] = x;
        py[c.gi] = y;
        pz[c.gi] = z;
    }
    // block maximum of the deviation, then one integer atomic max into one of
    // the replica's running-maximum slots (spread by block index)
    static_assert(kSiteBlock == 256, "block_max256 assumes 256 threads");
    const double m = block_max256(dev);
    if (threadIdx.x == 0)
        fold_max_slot(kickdev + (int64_t)blk_rep[blockIdx.x] * kKickSlots +
                          (blockIdx.x & (kKickSlots - 1)),
                      m);
}

__global__ void set_pulse_base_kernel(RepDev* reps, int nrep, uint64_t base) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrep) reps[r].kbase = base;
}

hipError_t launch_set_pulse_base(RepDev* reps, int nrep, uint64_t base, hipStream_t st) {
    if (nrep <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_pulse_base_kernel, dim3((nrep + 63) / 64), dim3(64), 0, st, reps, nrep,
                       base);
    return hipGetLastError();
}

hipError_t launch_kick(int prec, const RepDev* reps, const int32_t* blk_rep, int nblk, State s,
                       uint64_t k, double sigma_override, unsigned long long* kickdev,
                       hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(kick_kernel<double>, dim3(nblk), dim3(kSiteBlock), 0, st, reps, blk_rep,
                           s, k, sigma_override, kickdev);
    else
        hipLaunchKernelGGL(kick_kernel<float>, dim3(nblk), dim3(kSiteBlock), 0, st, reps, blk_rep,
                           s, k, sigma_override, kickdev);
    return hipGetLastError();
}

// ----------------------------------------------------------- observables ---
// Pass 1: per-block fp64 partial sums {sum_bonds s_i.s_j, sum H.s,
// sum D (s.e)^2, sum s (3), max | |s| - 1 |} in a fixed order; pass 2 sums
// the partials of every replica in block order.  No floating-point atomics:
// results are bit-identical from run to run.  (A single pass that lets the
// last block finish would need a device-scope release per block, which
// writes back the L2 of its XCD each time and costs far more than a launch.)
// Each site owns its bonds to its +x, +y and +z neighbours, so every bond is
// counted once: E = -J sum over bonds, the convention under which the
// simple-cubic T_c / J = 1.44 quoted in Sec. IV holds.

// The 8 reduced quantities: sums 0..5, max (6) and min (7) of |s|^2.  The
// norm deviation max_i | |s_i| - 1 | follows from the extremes alone (sqrt and
// the subtraction are monotone on each side of 1), so no per-site square root.
__device__ __forceinline__ double red8(int j, double a, double c) {
    return j < 6 ? a + c : (j == 6 ? nan_max(a, c) : nan_min(a, c));
}

// Butterfly over the 64 lanes of a wavefront (fixed pairing, so the result
// does not depend on timing); every lane ends with the wave's result.
__device__ __forceinline__ void wave_reduce8(double q[8]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = red8(j, q[j], __shfl_xor(q[j], o, 64));
    }
}

// Reduction of the 8 quantities over a block of NT threads into out[0..7]
// (written by threads 0..7).
template <int NT>
__device__ __forceinline__ void block_reduce8(double q[8], double* out) {
    constexpr int NW = NT / 64;
    __shared__ double red[NW][8];
    wave_reduce8(q);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int j = 0; j < 8; ++j) red[w][j] = q[j];
    __syncthreads();
    if (threadIdx.x < 8) {
        const int j = threadIdx.x;
        double a = red[0][j];
        for (int v = 1; v < NW; ++v) a = red8(j, a, red[v][j]);
        out[j] = a;
    }
}

// Planes per observables work item.  A work item is a run of kObsBlock
// consecutive (x, y) columns over kObsZ consecutive z-planes; each thread
// marches up its column, so the +z neighbour of a plane is the next plane's
// own spin, already in registers, and only the +x and +y neighbours (same
// and adjacent rows, cache hits) are loaded besides it.
constexpr int kObsZ = 8;

__host__ __device__ inline int64_t obs_items(int Lx, int Ly, int Lz) {
    const int64_t Lxy = (int64_t)Lx * Ly;
    return ((Lxy + kObsBlock - 1) / kObsBlock) * ((Lz + kObsZ - 1) / kObsZ);
}

int64_t obs_item_count(int Lx, int Ly, int Lz) { return obs_items(Lx, Ly, Lz); }

// Per-thread quantities of the observables pass: q[0] sum of s_i.s_j over the
// bonds, q[1] unused (0), q[2] the anisotropy sum before its constant D
// (sum (s.e)^2; per-site D included for site-dependent axes), q[3..5] sum s,
// q[6] / q[7] max / min of |s|^2 ignoring NaN (a NaN is kept in a flag).  The
// Zeeman sum H.(sum s) and the factor D are applied once per replica.
template <typename T, int ANIS>
__device__ __forceinline__ void obs_site(const RepDev& R, double sx, double sy, double sz, double bx,
                                         double by, double bz, const T* Ds, const T* es, int64_t N,
                                         int64_t g, double q[8], bool& nan) {
    q[0] += sx * bx + sy * by + sz * bz;
    if constexpr (ANIS == ANIS_Z) {
        q[2] += sz * sz;
    } else if constexpr (ANIS == ANIS_AXIS) {
        const double se = sx * R.e[0] + sy * R.e[1] + sz * R.e[2];
        q[2] += se * se;
    } else if constexpr (ANIS == ANIS_SITE) {
        const double se = sx * (double)es[g] + sy * (double)es[N + g] + sz * (double)es[2 * N + g];
        q[2] += (double)Ds[g] * se * se;
    }
    q[3] += sx;
    q[4] += sy;
    q[5] += sz;
    const double n2 = sx * sx + sy * sy + sz * sz;
    q[6] = __builtin_fmax(q[6], n2);
    q[7] = __builtin_fmin(q[7], n2);
    nan |= n2 != n2;
}

template <typename T, int ANIS>
__global__ void __launch_bounds__(kObsBlock)
    obs_partial_kernel(const RepDev* reps, const int32_t* oblk_rep, State s, double* partials) {
    const int b = blockIdx.x;
    const RepDev& R = reps[oblk_rep[b]];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const int64_t Lxy = (int64_t)Lx * Ly;
    const int64_t N = Lxy * Lz;
    const bool pbc = R.bc == 0;
    const T* __restrict__ px = static_cast<const T*>(s.x) + R.off;
    const T* __restrict__ py = static_cast<const T*>(s.y) + R.off;
    const T* __restrict__ pz = static_cast<const T*>(s.z) + R.off;
    const T* Ds = static_cast<const T*>(R.D_site);
    const T* es = static_cast<const T*>(R.e_site);
    // plane-relative byte offsets fit 32 bits: loads take a uniform plane
    // base plus a 32-bit lane offset (no 64-bit address arithmetic per load)
    const bool off32 = Lxy * (int64_t)sizeof(T) <= (int64_t)0x7fffffff;
    // items are numbered slab-major; block h takes a contiguous range of
    // them.  Workgroups are dealt out to the eight XCDs round-robin, so when
    // the replica's blocks start on an XCD boundary the hardware index is
    // permuted to give each XCD a contiguous range of slabs: the +y rows of
    // a column run and the +z plane of a slab then sit in the same L2.
    const int64_t ncb = (Lxy + kObsBlock - 1) / kObsBlock;
    const int64_t nitems = obs_items(Lx, Ly, Lz);
    const int nob = R.nob;
    int h = b - R.ob0;
    if ((nob & 7) == 0 && (R.ob0 & 7) == 0) h = (h & 7) * (nob >> 3) + (h >> 3);
    const int64_t per = (nitems + nob - 1) / nob;
    const int64_t it0 = (int64_t)h * per;
    const int64_t it1 = it0 + per < nitems ? it0 + per : nitems;
    double q[8] = {0, 0, 0, 0, 0, 0, 0, __builtin_huge_val()};
    bool nan = false;
    for (int64_t it = it0; it < it1; ++it) {
        const int slab = (int)(it / ncb);
        const int64_t cb = it - (int64_t)slab * ncb;
        const int z0 = slab * kObsZ;
        // every load of the item is issued before any arithmetic
        T v[kObsZ + 1][3], a[kObsZ][3], bq[kObsZ][3];
        if (pbc && off32 && z0 + kObsZ <= Lz && (cb + 1) * kObsBlock <= Lxy) {
            // whole item inside the lattice, every bond present (uniform
            // branch); column indices and byte offsets in 32 bits
            const uint32_t c = (uint32_t)cb * kObsBlock + threadIdx.x;
            const uint32_t y = c / (uint32_t)Lx, x = c - y * (uint32_t)Lx;
            const uint32_t cx = x + 1 < (uint32_t)Lx ? c + 1 : c + 1 - (uint32_t)Lx;
            const uint32_t cy = y + 1 < (uint32_t)Ly ? c + (uint32_t)Lx : c + (uint32_t)Lx - (uint32_t)Lxy;
            const uint32_t o0 = c * (uint32_t)sizeof(T);
            const uint32_t o1 = cx * (uint32_t)sizeof(T);
            const uint32_t o2 = cy * (uint32_t)sizeof(T);
#pragma unroll
            for (int j = 0; j <= kObsZ; ++j) {
                const int64_t po = (int64_t)(z0 + j < Lz ? z0 + j : 0) * Lxy;
                v[j][0] = ld_off(px + po, o0);
                v[j][1] = ld_off(py + po, o0);
                v[j][2] = ld_off(pz + po, o0);
            }
#pragma unroll
            for (int j = 0; j < kObsZ; ++j) {
                const int64_t po = (int64_t)(z0 + j) * Lxy;
                a[j][0] = ld_off(px + po, o1);
                a[j][1] = ld_off(py + po, o1);
                a[j][2] = ld_off(pz + po, o1);
                bq[j][0] = ld_off(px + po, o2);
                bq[j][1] = ld_off(py + po, o2);
                bq[j][2] = ld_off(pz + po, o2);
            }
#pragma unroll
            for (int j = 0; j < kObsZ; ++j) {
                double bn[3];
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    bn[m] = (double)a[j][m] + (double)bq[j][m] + (double)v[j + 1][m];
                obs_site<T, ANIS>(R, (double)v[j][0], (double)v[j][1], (double)v[j][2], bn[0], bn[1],
                                  bn[2], Ds, es, N, (int64_t)(z0 + j) * Lxy + c, q, nan);
            }
        } else {
            // general item: planes past Lz (last slab) address plane 0, lanes
            // past the last column address column 0; both count nothing
            const int64_t c = cb * kObsBlock + threadIdx.x;
            const bool okc = c < Lxy;
            const int64_t cc = okc ? c : 0;
            const int y = (int)((uint32_t)cc / (uint32_t)Lx), x = (int)(cc - (int64_t)y * Lx);
            // +x and +y offsets (wrapped at the far face; a missing
            // free-boundary bond still reads a valid site and is dropped)
            const int64_t ox = x + 1 < Lx ? 1 : 1 - Lx;
            const int64_t oy = y + 1 < Ly ? (int64_t)Lx : (int64_t)Lx - Lxy;
            const bool hx = pbc || x + 1 < Lx, hy = pbc || y + 1 < Ly;
            int64_t gp[kObsZ + 1];
            gp[0] = (int64_t)z0 * Lxy + cc;
#pragma unroll
            for (int j = 0; j < kObsZ; ++j) gp[j + 1] = z0 + j + 1 < Lz ? gp[j] + Lxy : cc;
#pragma unroll
            for (int j = 0; j <= kObsZ; ++j) {
                v[j][0] = px[gp[j]];
                v[j][1] = py[gp[j]];
                v[j][2] = pz[gp[j]];
            }
#pragma unroll
            for (int j = 0; j < kObsZ; ++j) {
                a[j][0] = px[gp[j] + ox];
                a[j][1] = py[gp[j] + ox];
                a[j][2] = pz[gp[j] + ox];
                bq[j][0] = px[gp[j] + oy];
                bq[j][1] = py[gp[j] + oy];
                bq[j][2] = pz[gp[j] + oy];
            }
#pragma unroll
            for (int j = 0; j < kObsZ; ++j) {
                const int z = z0 + j;
                if (!(okc && z < Lz)) continue;
                const bool hz = pbc || z + 1 < Lz;
                double bn[3];
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    bn[m] = (hx ? (double)a[j][m] : 0.0) + (hy ? (double)bq[j][m] : 0.0) +
                            (hz ? (double)v[j + 1][m] : 0.0);
                obs_site<T, ANIS>(R, (double)v[j][0], (double)v[j][1], (double)v[j][2], bn[0], bn[1],
                                  bn[2], Ds, es, N, gp[j], q, nan);
            }
        }
    }
    if (nan) q[6] = q[7] = __builtin_nan("");
    block_reduce8<kObsBlock>(q, partials + (int64_t)b * 8);
}

constexpr int kObsFinal = 256;

// Running sums of one measurement o[8] (result layout) added to a[8]: count,
// E, E^2, |m|, m^2, m.  One definition for every caller, so the sums do not
// depend on which launch adds them.
__device__ __forceinline__ void accum_add(double a[8], const double o[8]) {
    const double Et = o[0], mx = o[4], my = o[5], mz = o[6];
    const double m2 = mx * mx + my * my + mz * mz;
    a[0] = a[0] + 1.0;
    a[1] = a[1] + Et;
    a[2] = a[2] + Et * Et;
    a[3] = a[3] + sqrt(m2);
    a[4] = a[4] + m2;
    a[5] = a[5] + mx;
    a[6] = a[6] + my;
    a[7] = a[7] + mz;
}

// One block: sums the partials of replica R (global blocks ob0 .. ob0+nob-1 of
// `partials`) in block order into o[8].  accum (optional): the replica's
// running sums, updated.
__device__ __forceinline__ void obs_final_block(const RepDev& R, int anis, const double* partials,
                                                double* o, double* accum) {
    // the running sums are fetched first: their address needs nothing else
    double a_old[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (accum && threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 8; ++j) a_old[j] = accum[j];
    // at most kFinalU partials per thread and pass, loaded together
    constexpr int kFinalU = 8;
    double q[8] = {0, 0, 0, 0, 0, 0, 0, __builtin_huge_val()};
    const int pend = R.ob0 + R.nob;
    for (int b0 = R.ob0; b0 < pend; b0 += kFinalU * kObsFinal) {
        double v[kFinalU][8];
#pragma unroll
        for (int u = 0; u < kFinalU; ++u) {
            const int bb = b0 + u * kObsFinal + (int)threadIdx.x;
            const double* p = partials + (int64_t)(bb < pend ? bb : R.ob0) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[u][j] = p[j];
        }
#pragma unroll
        for (int u = 0; u < kFinalU; ++u)
            if (b0 + u * kObsFinal + (int)threadIdx.x < pend)
#pragma unroll
                for (int j = 0; j < 8; ++j) q[j] = red8(j, q[j], v[u][j]);
    }
    __shared__ double tot[8];
    block_reduce8<kObsFinal>(q, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double N = (double)R.Lx * R.Ly * R.Lz;
        double r8[8];
        r8[1] = -R.J * tot[0];
        r8[2] = -(R.H[0] * tot[3] + R.H[1] * tot[4] + R.H[2] * tot[5]);
        r8[3] = -(anis == ANIS_Z || anis == ANIS_AXIS ? R.D * tot[2] : tot[2]);
        r8[0] = r8[1] + r8[2] + r8[3];
        r8[4] = tot[3] / N;
        r8[5] = tot[4] / N;
        r8[6] = tot[5] / N;
        r8[7] = nan_max(sqrt(tot[6]) - 1.0, 1.0 - sqrt(tot[7]));
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = r8[j];
        if (accum) {
            accum_add(a_old, r8);
#pragma unroll
            for (int j = 0; j < 8; ++j) accum[j] = a_old[j];
        }
    }
}

// Block r: observables of replica r into result[r] (and its running sums when
// accumulate).
__global__ void __launch_bounds__(kObsFinal)
    obs_final_kernel(const RepDev* reps, int anis, const double* partials, double* result,
                     double* accum, int accumulate) {
    const int r = blockIdx.x;
    obs_final_block(reps[r], anis, partials, result + (int64_t)r * 8,
                    accumulate ? accum + (int64_t)r * 8 : nullptr);
}

// Block (r, j): observables of replica r in staged measurement j, whose
// partials start at stage + j * nobblk * 8, into out + j * ostride + r * 8.
__global__ void __launch_bounds__(kObsFinal)
    obs_final_staged_kernel(const RepDev* reps, int anis, const double* stage, int nobblk,
                            double* out, int64_t ostride) {
    const int r = blockIdx.x, j = blockIdx.y;
    obs_final_block(reps[r], anis, stage + (int64_t)j * nobblk * 8,
                    out + (int64_t)j * ostride + (int64_t)r * 8, nullptr);
}

// Thread r: the n staged measurements of replica r added to its running sums
// in measurement order; the last one is also copied to result[r].
__global__ void __launch_bounds__(64)
    accum_staged_kernel(int nrep, const double* out, int64_t ostride, int n, double* accum,
                        double* result) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = accum[(int64_t)r * 8 + j];
#pragma unroll 4
    for (int m = 0; m < n; ++m) {
        double o[8];
        const double* src = out + (int64_t)m * ostride + (int64_t)r * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = src[j];
        accum_add(a, o);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) accum[(int64_t)r * 8 + j] = a[j];
    const double* last = out + (int64_t)(n - 1) * ostride + (int64_t)r * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) result[(int64_t)r * 8 + j] = last[j];
}

template <typename T>
static void launch_obs_t(int anis, const RepDev* reps, const int32_t* oblk_rep, int nobblk, State s,
                         double* partials, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE:
            hipLaunchKernelGGL((obs_partial_kernel<T, ANIS_NONE>), dim3(nobblk), dim3(kObsBlock), 0,
                               st, reps, oblk_rep, s, partials);
            break;
        case ANIS_Z:
            hipLaunchKernelGGL((obs_partial_kernel<T, ANIS_Z>), dim3(nobblk), dim3(kObsBlock), 0, st,
                               reps, oblk_rep, s, partials);
            break;
        case ANIS_AXIS:
            hipLaunchKernelGGL((obs_partial_kernel<T, ANIS_AXIS>), dim3(nobblk), dim3(kObsBlock), 0,
                               st, reps, oblk_rep, s, partials);
            break;
        default:
            hipLaunchKernelGGL((obs_partial_kernel<T, ANIS_SITE>), dim3(nobblk), dim3(kObsBlock), 0,
                               st, reps, oblk_rep, s, partials);
            break;
    }
}

hipError_t launch_obs(int prec, int anis, const RepDev* reps, const int32_t* oblk_rep,
                      int nobblk, int nrep, State s, double* partials, double* result,
                      double* accum, int accumulate, hipStream_t st) {
    if (nobblk <= 0 || nrep <= 0) return hipSuccess;
    if (prec == 0)
        launch_obs_t<double>(anis, reps, oblk_rep, nobblk, s, partials, st);
    else
        launch_obs_t<float>(anis, reps, oblk_rep, nobblk, s, partials, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obs_final_kernel, dim3(nrep), dim3(kObsFinal), 0, st, reps, anis, partials,
                       result, accum, accumulate);
    return hipGetLastError();
}

hipError_t launch_obs_partials(int prec, int anis, const RepDev* reps, const int32_t* oblk_rep,
                               int nobblk, State s, double* partials, hipStream_t st) {
    if (nobblk <= 0) return hipSuccess;
    if (prec == 0)
        launch_obs_t<double>(anis, reps, oblk_rep, nobblk, s, partials, st);
    else
        launch_obs_t<float>(anis, reps, oblk_rep, nobblk, s, partials, st);
    return hipGetLastError();
}

hipError_t launch_obs_staged(int anis, const RepDev* reps, int nrep, int nobblk, int n,
                             const double* stage, double* out, int64_t ostride, double* accum,
                             double* result, hipStream_t st) {
    if (n <= 0 || nrep <= 0 || nobblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(obs_final_staged_kernel, dim3(nrep, n), dim3(kObsFinal), 0, st, reps, anis,
                       stage, nobblk, out, ostride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(accum_staged_kernel, dim3((nrep + 63) / 64), dim3(64), 0, st, nrep, out,
                       ostride, n, accum, result);
    return hipGetLastError();
}

// -------------------------------------------------------- unfused RK4 step --
// Stage s reads its input y_s (neighbourhood), the step's start state x and
// the accumulator; stage 1: acc = x + k/6, y2 = x + k/2; stage 2: acc += k/3,
// y3 = x + k/2; stage 3: acc += k/3, y4 = x + k; stage 4: x' = acc + k/6
// (written over x, which stage 4 does not read).
// k = dt f(y) at the site of c: the six-neighbour sum of y (missing neighbours
// of free boundaries contribute nothing), then Eq. (1).
template <typename T, bool PREC, int ANIS>
__device__ __forceinline__ void site_k(const RepDev& R, const SiteCtx& c, const State& yin, T& kx,
                                       T& ky, T& kz) {
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const int64_t N = (int64_t)Lx * Ly * Lz;
    int x, y, z;
    site_xyz(c.i, Lx, Ly, x, y, z);
    const T* yx = static_cast<const T*>(yin.x);
    const T* yy = static_cast<const T*>(yin.y);
    const T* yz = static_cast<const T*>(yin.z);
    int64_t d[6];
    bool has[6];
    nbr_offsets(R, x, y, z, d, has);
    T vx[6], vy[6], vz[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        vx[k] = yx[c.gi + d[k]];
        vy[k] = yy[c.gi + d[k]];
        vz[k] = yz[c.gi + d[k]];
    }
    // adding zero for a missing neighbour leaves the sum's bits unchanged
    T nx = 0, ny = 0, nz = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        nx += has[k] ? vx[k] : T(0);
        ny += has[k] ? vy[k] : T(0);
        nz += has[k] ? vz[k] : T(0);
    }
    const T sx = yx[c.gi], sy = yy[c.gi], sz = yz[c.gi];
    const Coef<T> C = load_coef<T>(R);
    T Di = 0, ex = 0, ey = 0, ez = 0;
    if constexpr (ANIS == ANIS_SITE) {
        Di = static_cast<const T*>(R.D_site)[c.i];
        const T* es = static_cast<const T*>(R.e_site);
        ex = es[c.i];
        ey = es[N + c.i];
        ez = es[2 * N + c.i];
    }
    stage_k<T, PREC, ANIS>(sx, sy, sz, nx, ny, nz, C, Di, ex, ey, ez, kx, ky, kz);
}

template <typename T, bool PREC, int ANIS>
__global__ void __launch_bounds__(kSiteBlock)
    stage_kernel(const RepDev* reps, const int32_t* blk_rep, State yin, State xs, State acc,
                 State out, int stage) {
    SiteCtx c;
    if (!site_of_thread(reps, blk_rep, c)) return;
    T kx, ky, kz;
    site_k<T, PREC, ANIS>(reps[c.r], c, yin, kx, ky, kz);
    T* ax = static_cast<T*>(acc.x);
    T* ay = static_cast<T*>(acc.y);
    T* az = static_cast<T*>(acc.z);
    T* ox = static_cast<T*>(out.x);
    T* oy = static_cast<T*>(out.y);
    T* oz = static_cast<T*>(out.z);
    const T* xx = static_cast<const T*>(xs.x);
    const T* xy = static_cast<const T*>(xs.y);
    const T* xz = static_cast<const T*>(xs.z);
    const T c6 = T(1) / T(6), c3 = T(1) / T(3), c2 = T(0.5);
    const int64_t g = c.gi;
    if (stage == 1) {
        const T x0 = xx[g], x1 = xy[g], x2 = xz[g];
        ax[g] = kx * c6 + x0;
        ay[g] = ky * c6 + x1;
        az[g] = kz * c6 + x2;
        ox[g] = kx * c2 + x0;
        oy[g] = ky * c2 + x1;
        oz[g] = kz * c2 + x2;
    } else if (stage == 2 || stage == 3) {
        ax[g] = kx * c3 + ax[g];
        ay[g] = ky * c3 + ay[g];
        az[g] = kz * c3 + az[g];
        const T w = stage == 2 ? c2 : T(1);
        ox[g] = kx * w + xx[g];
        oy[g] = ky * w + xy[g];
        oz[g] = kz * w + xz[g];
    } else {
        ox[g] = kx * c6 + ax[g];
        oy[g] = ky * c6 + ay[g];
        oz[g] = kz * c6 + az[g];
    }
}

template <typename T, bool PREC, int ANIS>
static hipError_t step_unfused_t(const RepDev* reps, const int32_t* blk_rep, int nblk, State s,
                                 State yA, State yB, State acc, hipStream_t st) {
    const State ins[4] = {s, yA, yB, yA};
    const State outs[4] = {yA, yB, yA, s};
    for (int q = 0; q < 4; ++q) {
        hipLaunchKernelGGL((stage_kernel<T, PREC, ANIS>), dim3(nblk), dim3(kSiteBlock), 0, st, reps,
                           blk_rep, ins[q], s, acc, outs[q], q + 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool PREC>
static hipError_t step_unfused_p(int anis, const RepDev* reps, const int32_t* blk_rep, int nblk,
                                 State s, State yA, State yB, State acc, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: return step_unfused_t<T, PREC, ANIS_NONE>(reps, blk_rep, nblk, s, yA, yB, acc, st);
        case ANIS_Z: return step_unfused_t<T, PREC, ANIS_Z>(reps, blk_rep, nblk, s, yA, yB, acc, st);
        case ANIS_AXIS: return step_unfused_t<T, PREC, ANIS_AXIS>(reps, blk_rep, nblk, s, yA, yB, acc, st);
        default: return step_unfused_t<T, PREC, ANIS_SITE>(reps, blk_rep, nblk, s, yA, yB, acc, st);
    }
}

hipError_t launch_step_unfused(int prec, int precession, int anis, const RepDev* reps,
                               const int32_t* blk_rep, int nblk, State s, State yA, State yB,
                               State acc, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    if (prec == 0)
        return precession ? step_unfused_p<double, true>(anis, reps, blk_rep, nblk, s, yA, yB, acc, st)
                          : step_unfused_p<double, false>(anis, reps, blk_rep, nblk, s, yA, yB, acc, st);
    return precession ? step_unfused_p<float, true>(anis, reps, blk_rep, nblk, s, yA, yB, acc, st)
                      : step_unfused_p<float, false>(anis, reps, blk_rep, nblk, s, yA, yB, acc, st);
}

// RK4 step that keeps its stage inputs: y2, y3, y4 and the result xnext are
// separate buffers (the adjoint stores them); acc is scratch.
template <typename T, bool PREC, int ANIS>
static hipError_t stages_t(const RepDev* reps, const int32_t* blk_rep, int nblk, State x, State y2,
                           State y3, State y4, State acc, State xnext, hipStream_t st) {
    const State ins[4] = {x, y2, y3, y4};
    const State outs[4] = {y2, y3, y4, xnext};
    for (int q = 0; q < 4; ++q) {
        hipLaunchKernelGGL((stage_kernel<T, PREC, ANIS>), dim3(nblk), dim3(kSiteBlock), 0, st, reps,
                           blk_rep, ins[q], x, acc, outs[q], q + 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool PREC>
static hipError_t stages_p(int anis, const RepDev* reps, const int32_t* blk, int nblk, State x,
                           State y2, State y3, State y4, State acc, State xn, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: return stages_t<T, PREC, ANIS_NONE>(reps, blk, nblk, x, y2, y3, y4, acc, xn, st);
        case ANIS_Z: return stages_t<T, PREC, ANIS_Z>(reps, blk, nblk, x, y2, y3, y4, acc, xn, st);
        case ANIS_AXIS: return stages_t<T, PREC, ANIS_AXIS>(reps, blk, nblk, x, y2, y3, y4, acc, xn, st);
        default: return stages_t<T, PREC, ANIS_SITE>(reps, blk, nblk, x, y2, y3, y4, acc, xn, st);
    }
}

hipError_t launch_rk4_stages(int prec, int precession, int anis, const RepDev* reps,
                             const int32_t* blk_rep, int nblk, State x, State y2, State y3,
                             State y4, State acc, State xnext, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    if (prec == 0)
        return precession ? stages_p<double, true>(anis, reps, blk_rep, nblk, x, y2, y3, y4, acc, xnext, st)
                          : stages_p<double, false>(anis, reps, blk_rep, nblk, x, y2, y3, y4, acc, xnext, st);
    return precession ? stages_p<float, true>(anis, reps, blk_rep, nblk, x, y2, y3, y4, acc, xnext, st)
                      : stages_p<float, false>(anis, reps, blk_rep, nblk, x, y2, y3, y4, acc, xnext, st);
}

// ---------------------------------------------------- explicit RK tableau --
// One stage j of an explicit Runge-Kutta step given by its tableau: k_j =
// dt f(y_j) from the neighbourhood of yin = y_j; then either the next stage's
// input y_{j+1} = x + sum_{l<=j} a[j+1][l] k_l (k_j kept in K[j]) or, for the
// last stage, x' = x + sum_l b[l] k_l written over x (which no thread reads
// as a neighbour in that stage).
template <typename T, bool PREC, int ANIS>
__global__ void __launch_bounds__(kSiteBlock)
    tableau_stage_kernel(const RepDev* reps, const int32_t* blk_rep, State yin, State xs, KSet ks,
                         Tableau tb, int j, State out) {
    SiteCtx c;
    if (!site_of_thread(reps, blk_rep, c)) return;
    T kx, ky, kz;
    site_k<T, PREC, ANIS>(reps[c.r], c, yin, kx, ky, kz);
    const int64_t g = c.gi;
    const bool last = j == tb.stages - 1;
    const double* w = last ? tb.b : tb.a[j + 1];
    T* px = static_cast<T*>(xs.x);
    T* py = static_cast<T*>(xs.y);
    T* pz = static_cast<T*>(xs.z);
    T ox = px[g], oy = py[g], oz = pz[g];
    for (int l = 0; l < j; ++l) {
        if (w[l] == 0.0) continue;
        const T wl = (T)w[l];
        ox += wl * static_cast<const T*>(ks.K[l].x)[g];
        oy += wl * static_cast<const T*>(ks.K[l].y)[g];
        oz += wl * static_cast<const T*>(ks.K[l].z)[g];
    }
    const T wj = (T)w[j];
    ox += wj * kx;
    oy += wj * ky;
    oz += wj * kz;
    if (last) {
        px[g] = ox;
        py[g] = oy;
        pz[g] = oz;
        return;
    }
    static_cast<T*>(ks.K[j].x)[g] = kx;
    static_cast<T*>(ks.K[j].y)[g] = ky;
    static_cast<T*>(ks.K[j].z)[g] = kz;
    static_cast<T*>(out.x)[g] = ox;
    static_cast<T*>(out.y)[g] = oy;
    static_cast<T*>(out.z)[g] = oz;
}

template <typename T, bool PREC, int ANIS>
static hipError_t tableau_t(const RepDev* reps, const int32_t* blk_rep, int nblk, const Tableau& tb,
                            State s, State yA, State yB, const KSet& ks, hipStream_t st) {
    State yin = s;
    for (int j = 0; j < tb.stages; ++j) {
        const State out = (j % 2 == 0) ? yA : yB;
        hipLaunchKernelGGL((tableau_stage_kernel<T, PREC, ANIS>), dim3(nblk), dim3(kSiteBlock), 0, st,
                           reps, blk_rep, yin, s, ks, tb, j, out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        yin = out;
    }
    return hipSuccess;
}

template <typename T, bool PREC>
static hipError_t tableau_p(int anis, const RepDev* reps, const int32_t* blk_rep, int nblk,
                            const Tableau& tb, State s, State yA, State yB, const KSet& ks,
                            hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: return tableau_t<T, PREC, ANIS_NONE>(reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
        case ANIS_Z: return tableau_t<T, PREC, ANIS_Z>(reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
        case ANIS_AXIS: return tableau_t<T, PREC, ANIS_AXIS>(reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
        default: return tableau_t<T, PREC, ANIS_SITE>(reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
    }
}

hipError_t launch_step_tableau(int prec, int precession, int anis, const RepDev* reps,
                               const int32_t* blk_rep, int nblk, const Tableau& tb, State s,
                               State yA, State yB, const KSet& ks, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    if (tb.stages < 1 || tb.stages > 6) return hipErrorInvalidValue;
    if (prec == 0)
        return precession ? tableau_p<double, true>(anis, reps, blk_rep, nblk, tb, s, yA, yB, ks, st)
                          : tableau_p<double, false>(anis, reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
    return precession ? tableau_p<float, true>(anis, reps, blk_rep, nblk, tb, s, yA, yB, ks, st)
                      : tableau_p<float, false>(anis, reps, blk_rep, nblk, tb, s, yA, yB, ks, st);
}

// ------------------------------------------------------------------ copy ---
template <typename T>
__global__ void __launch_bounds__(256) copy_kernel(State dst, State src, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    static_cast<T*>(dst.x)[i] = static_cast<const T*>(src.x)[i];
    static_cast<T*>(dst.y)[i] = static_cast<const T*>(src.y)[i];
    static_cast<T*>(dst.z)[i] = static_cast<const T*>(src.z)[i];
}

hipError_t launch_copy(int prec, State dst, State src, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    if (prec == 0)
        hipLaunchKernelGGL(copy_kernel<double>, dim3((unsigned)nb), dim3(256), 0, st, dst, src, n);
    else
        hipLaunchKernelGGL(copy_kernel<float>, dim3((unsigned)nb), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

}  // namespace lll
