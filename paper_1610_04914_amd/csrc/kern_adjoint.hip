// Kernels of the discrete adjoint (reverse mode) of the RK4 + kick schedule.
//
// For f(s) = s x h - lam s x (s x h) (the slow equation drops s x h) and a
// cotangent u of f at a site:
//   q   = (df/dh)^T u         = u x s - lam [ s (s.u) - u (s.s) ]
//   loc = (df/ds)^T u (h fixed) = h x u - lam [ u (s.h) + h (s.u) - 2 s (h.u) ]
// and, because h_i = J sum_nn s_j + H + 2 D_i (s_i.e_i) e_i couples sites
// through a symmetric stencil, the cotangent of the stage input is
//   ybar_i = loc_i + J sum_nn q_j + 2 D_i e_i (e_i.q_i).
// Pass A computes q and loc (one stencil on y for h), pass B ybar (one stencil
// on q) and folds it into the RK4 cotangents.  Parameter cotangents are
//   Hbar += sum q, Jbar += sum q . sum_nn y, Dbar_i += 2 (y.e_i)(q.e_i),
// reduced per block into fp64 partials and summed in a fixed order (no
// floating-point atomics).
#include "lll_device.hpp"
#include "lll_site.hpp"

namespace lll {


struct SiteA {
    int r;
    int64_t i, gi;
    int x, y, z;
};

// The adjoint runs on one lattice, whose descriptor comes by value as a
// kernel argument: no dependent loads of a block table and a replica record
// before the first data load.
__device__ __forceinline__ bool adj_site(const RepDev& R, SiteA& c) {
    const int b = blockIdx.x;
    c.r = 0;
    const int64_t N = (int64_t)R.Lx * R.Ly * R.Lz;
    c.i = (int64_t)(b - R.sb0) * kAdjBlock + threadIdx.x;
    c.gi = R.off + c.i;
    if (c.i >= N) return false;
    site_xyz(c.i, R.Lx, R.Ly, c.x, c.y, c.z);
    return true;
}

// Sum over the (up to six) neighbours of site c of the field a, in the order
// -x, +x, -y, +y, -z, +z.  Branch-free: a missing neighbour (free boundary)
// reads the site itself and adds 0.0 instead, which leaves the sum's bits as
// they are; all eighteen loads are independent, so they are in flight
// together rather than each waiting for the one before.
template <typename T>
__device__ __forceinline__ void nbr_sum(const RepDev& R, const SiteA& c, const T* ax, const T* ay,
                                        const T* az, double& sx, double& sy, double& sz) {
    int64_t d[6];
    bool has[6];
    nbr_offsets(R, c.x, c.y, c.z, d, has);
    double vx[6], vy[6], vz[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t j = c.gi + d[k];
        vx[k] = (double)ax[j];
        vy[k] = (double)ay[j];
        vz[k] = (double)az[j];
    }
    sx = sy = sz = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        sx += has[k] ? vx[k] : 0.0;
        sy += has[k] ? vy[k] : 0.0;
        sz += has[k] ? vz[k] : 0.0;
    }
}

template <typename T, int ANIS>
__device__ __forceinline__ void aniso_of(const RepDev& R, int64_t i, double& D, double& e0,
                                         double& e1, double& e2) {
    if constexpr (ANIS == ANIS_SITE) {
        const int64_t N = (int64_t)R.Lx * R.Ly * R.Lz;
        const T* Ds = static_cast<const T*>(R.D_site);
        const T* es = static_cast<const T*>(R.e_site);
        D = (double)Ds[i];
        e0 = (double)es[i];
        e1 = (double)es[N + i];
        e2 = (double)es[2 * N + i];
    } else if constexpr (ANIS == ANIS_NONE) {
        D = 0.0;
        e0 = R.e[0];
        e1 = R.e[1];
        e2 = R.e[2];
    } else {
        D = R.D;
        e0 = R.e[0];
        e1 = R.e[1];
        e2 = R.e[2];
    }
}

// Block sum of five fp64 partials added to part[blockIdx.x][0..4] (each block
// owns its row, so the running sums are deterministic; they are reduced once,
// in block order, at the end of the backward pass).  A butterfly within each
// wave, then the wave sums in wave order: a fixed order with one barrier.
__device__ __forceinline__ void block_sum5(double v[5], double* part) {
    constexpr int kWaves = kAdjBlock / 64;
    __shared__ double red[5][kWaves];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < 5; ++q) v[q] += __shfl_xor(v[q], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 5; ++q) red[q][w] = v[q];
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = red[threadIdx.x][0];
        for (int k = 1; k < kWaves; ++k) t += red[threadIdx.x][k];
        part[(int64_t)blockIdx.x * 5 + threadIdx.x] += t;
    }
}

// Cotangent of the loss L = <c, s> + wE E(s) + wm . m(s) at the final state:
// sbar_i = c_i - wE h_i + wm / N (c = 0 when cot.x is null), with the direct
// parameter terms dE/dH = -sum s_i, dE/dJ = -sum_bonds s_i.s_j,
// dE/dD_i = -(s_i.e_i)^2.
template <typename T, int ANIS>
__global__ void __launch_bounds__(kAdjBlock)
    adj_loss_kernel(const RepDev R, State s, State cot, State sbar, double wE, double wm0,
                    double wm1, double wm2, double* gD, double* part) {
    SiteA c;
    double v[5] = {0, 0, 0, 0, 0};
    if (adj_site(R, c)) {
        const T* sx = static_cast<const T*>(s.x);
        const T* sy = static_cast<const T*>(s.y);
        const T* sz = static_cast<const T*>(s.z);
        const double x0 = sx[c.gi], x1 = sy[c.gi], x2 = sz[c.gi];
        double n0, n1, n2;
        nbr_sum<T>(R, c, sx, sy, sz, n0, n1, n2);
        double D, e0, e1, e2;
        aniso_of<T, ANIS>(R, c.i, D, e0, e1, e2);
        const double se = x0 * e0 + x1 * e1 + x2 * e2;
        const double h0 = R.J * n0 + R.H[0] + 2.0 * D * se * e0;
        const double h1 = R.J * n1 + R.H[1] + 2.0 * D * se * e1;
        const double h2 = R.J * n2 + R.H[2] + 2.0 * D * se * e2;
        const double N = (double)R.Lx * R.Ly * R.Lz;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        if (cot.x) {
            c0 = (double)static_cast<const T*>(cot.x)[c.gi];
            c1 = (double)static_cast<const T*>(cot.y)[c.gi];
            c2 = (double)static_cast<const T*>(cot.z)[c.gi];
        }
        static_cast<T*>(sbar.x)[c.gi] = (T)(c0 + (-wE * h0 + wm0 / N));
        static_cast<T*>(sbar.y)[c.gi] = (T)(c1 + (-wE * h1 + wm1 / N));
        static_cast<T*>(sbar.z)[c.gi] = (T)(c2 + (-wE * h2 + wm2 / N));
        // bonds along +x, +y, +z of this site
        const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
        const bool pbc = R.bc == 0;
        double bonds = 0.0;
        auto bond = [&](int xx, int yy, int zz) {
            const int64_t j = R.off + xx + (int64_t)Lx * (yy + (int64_t)Ly * zz);
            bonds += x0 * (double)sx[j] + x1 * (double)sy[j] + x2 * (double)sz[j];
        };
        if (pbc || c.x + 1 < Lx) bond(c.x + 1 < Lx ? c.x + 1 : 0, c.y, c.z);
        if (pbc || c.y + 1 < Ly) bond(c.x, c.y + 1 < Ly ? c.y + 1 : 0, c.z);
        if (pbc || c.z + 1 < Lz) bond(c.x, c.y, c.z + 1 < Lz ? c.z + 1 : 0);
        v[0] = -wE * x0;
        v[1] = -wE * x1;
        v[2] = -wE * x2;
        v[3] = -wE * bonds;
        if constexpr (ANIS == ANIS_SITE)
            gD[c.i] += -wE * se * se;
        else
            v[4] = -wE * se * se;
    }
    block_sum5(v, part);
}

// What the reverse of f at a site reads: the stage input there, the sum of
// its neighbours, the site's anisotropy and (per-site anisotropy) its running
// dL/dD_i.  Loaded ahead of any store of the same launch, so that these loads
// are not held behind the stores (the compiler cannot move a load across a
// store it might alias).
struct AIn {
    double s0, s1, s2, n0, n1, n2, D, e0, e1, e2, gd;
};

template <typename T, int ANIS>
__device__ __forceinline__ AIn load_a_in(const RepDev& R, const SiteA& c, const State& y,
                                         const double* gD) {
    AIn a;
    a.gd = ANIS == ANIS_SITE ? gD[c.i] : 0.0;
    const T* yx = static_cast<const T*>(y.x);
    const T* yy = static_cast<const T*>(y.y);
    const T* yz = static_cast<const T*>(y.z);
    a.s0 = yx[c.gi];
    a.s1 = yy[c.gi];
    a.s2 = yz[c.gi];
    nbr_sum<T>(R, c, yx, yy, yz, a.n0, a.n1, a.n2);
    aniso_of<T, ANIS>(R, c.i, a.D, a.e0, a.e1, a.e2);
    return a;
}

// Reverse of f at one site: u is the cotangent of f(y) there; writes q and
// loc and adds the site's parameter terms to v (Hbar 0..2, Jbar 3, Dbar 4;
// per-site Dbar goes to gD).
template <typename T, bool PREC, int ANIS>
__device__ __forceinline__ void adj_a_site(const RepDev& R, const SiteA& c, const AIn& a,
                                           double u0, double u1, double u2, const State& q,
                                           const State& loc, double* gD, double v[5]) {
    const double s0 = a.s0, s1 = a.s1, s2 = a.s2;
    const double n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const double D = a.D, e0 = a.e0, e1 = a.e1, e2 = a.e2;
    const double se = s0 * e0 + s1 * e1 + s2 * e2;
    const double h0 = R.J * n0 + R.H[0] + 2.0 * D * se * e0;
    const double h1 = R.J * n1 + R.H[1] + 2.0 * D * se * e1;
    const double h2 = R.J * n2 + R.H[2] + 2.0 * D * se * e2;
    const double lam = R.lambda;
    const double su = s0 * u0 + s1 * u1 + s2 * u2;
    const double ss = s0 * s0 + s1 * s1 + s2 * s2;
    const double sh = s0 * h0 + s1 * h1 + s2 * h2;
    const double hu = h0 * u0 + h1 * u1 + h2 * u2;
    double q0 = -lam * (s0 * su - u0 * ss);
    double q1 = -lam * (s1 * su - u1 * ss);
    double q2 = -lam * (s2 * su - u2 * ss);
    double l0 = -lam * (u0 * sh + h0 * su - 2.0 * s0 * hu);
    double l1 = -lam * (u1 * sh + h1 * su - 2.0 * s1 * hu);
    double l2 = -lam * (u2 * sh + h2 * su - 2.0 * s2 * hu);
    if constexpr (PREC) {
        q0 += u1 * s2 - u2 * s1;  // u x s
        q1 += u2 * s0 - u0 * s2;
        q2 += u0 * s1 - u1 * s0;
        l0 += h1 * u2 - h2 * u1;  // h x u
        l1 += h2 * u0 - h0 * u2;
        l2 += h0 * u1 - h1 * u0;
    }
    static_cast<T*>(q.x)[c.gi] = (T)q0;
    static_cast<T*>(q.y)[c.gi] = (T)q1;
    static_cast<T*>(q.z)[c.gi] = (T)q2;
    static_cast<T*>(loc.x)[c.gi] = (T)l0;
    static_cast<T*>(loc.y)[c.gi] = (T)l1;
    static_cast<T*>(loc.z)[c.gi] = (T)l2;
    v[0] += q0;
    v[1] += q1;
    v[2] += q2;
    v[3] += q0 * n0 + q1 * n1 + q2 * n2;
    const double dD = 2.0 * se * (q0 * e0 + q1 * e1 + q2 * e2);
    if constexpr (ANIS == ANIS_SITE)
        gD[c.i] = a.gd + dD;
    else
        v[4] += dD;
}

// Pass A: u = scale * kb is the cotangent of f(y); writes q and loc and the
// parameter partials.
template <typename T, bool PREC, int ANIS>
__global__ void __launch_bounds__(kAdjBlock)
    adj_pass_a(const RepDev R, State y, State kb, double scale, State q, State loc, double* gD,
               double* part) {
    SiteA c;
    double v[5] = {0, 0, 0, 0, 0};
    if (adj_site(R, c)) {
        const double u0 = scale * (double)static_cast<const T*>(kb.x)[c.gi];
        const double u1 = scale * (double)static_cast<const T*>(kb.y)[c.gi];
        const double u2 = scale * (double)static_cast<const T*>(kb.z)[c.gi];
        adj_a_site<T, PREC, ANIS>(R, c, load_a_in<T, ANIS>(R, c, y, gD), u0, u1, u2, q, loc, gD,
                                  v);
    }
    block_sum5(v, part);
}

// Pass B at one site: ybar = loc + J sum_nn q + 2 D e (e.q), folded into the
// RK4 cotangents (stage 4: xbar = sbar + ybar, kb = sbar/3 + ybar; stage 3:
// xbar += ybar, kb = sbar/3 + ybar/2; stage 2: xbar += ybar,
// kb = sbar/6 + ybar/2; stage 1: xbar += ybar).  Returns the new kb at the
// site as stored (stages 4..2), or at stage 1 the finished xbar as stored:
// the cotangent of the step's input, which is the output of the step before.
template <typename T, int ANIS>
__device__ __forceinline__ void adj_b_site(const RepDev& R, const SiteA& c, const State& q,
                                           const State& loc, const State& sbar, const State& xbar,
                                           const State& kb, int stage, double D, double e0,
                                           double e1, double e2, T& kb0, T& kb1, T& kb2) {
    const T* qx = static_cast<const T*>(q.x);
    const T* qy = static_cast<const T*>(q.y);
    const T* qz = static_cast<const T*>(q.z);
    double n0, n1, n2;
    nbr_sum<T>(R, c, qx, qy, qz, n0, n1, n2);
    const double q0 = qx[c.gi], q1 = qy[c.gi], q2 = qz[c.gi];
    const double eq = e0 * q0 + e1 * q1 + e2 * q2;
    const int64_t g = c.gi;
    const double y0 = (double)static_cast<const T*>(loc.x)[g] + R.J * n0 + 2.0 * D * e0 * eq;
    const double y1 = (double)static_cast<const T*>(loc.y)[g] + R.J * n1 + 2.0 * D * e1 * eq;
    const double y2 = (double)static_cast<const T*>(loc.z)[g] + R.J * n2 + 2.0 * D * e2 * eq;
    const double b0 = static_cast<const T*>(sbar.x)[g];
    const double b1 = static_cast<const T*>(sbar.y)[g];
    const double b2 = static_cast<const T*>(sbar.z)[g];
    T* xb0 = static_cast<T*>(xbar.x);
    T* xb1 = static_cast<T*>(xbar.y);
    T* xb2 = static_cast<T*>(xbar.z);
    if (stage == 4) {
        xb0[g] = (T)(b0 + y0);
        xb1[g] = (T)(b1 + y1);
        xb2[g] = (T)(b2 + y2);
    } else {
        const T x0 = (T)((double)xb0[g] + y0);
        const T x1 = (T)((double)xb1[g] + y1);
        const T x2 = (T)((double)xb2[g] + y2);
        xb0[g] = x0;
        xb1[g] = x1;
        xb2[g] = x2;
        kb0 = x0;
        kb1 = x1;
        kb2 = x2;
    }
    if (stage == 4) {
        kb0 = (T)(b0 / 3.0 + y0);
        kb1 = (T)(b1 / 3.0 + y1);
        kb2 = (T)(b2 / 3.0 + y2);
    } else if (stage == 3) {
        kb0 = (T)(b0 / 3.0 + 0.5 * y0);
        kb1 = (T)(b1 / 3.0 + 0.5 * y1);
        kb2 = (T)(b2 / 3.0 + 0.5 * y2);
    } else if (stage == 2) {
        kb0 = (T)(b0 / 6.0 + 0.5 * y0);
        kb1 = (T)(b1 / 6.0 + 0.5 * y1);
        kb2 = (T)(b2 / 6.0 + 0.5 * y2);
    }
    if (stage >= 2) {
        static_cast<T*>(kb.x)[g] = kb0;
        static_cast<T*>(kb.y)[g] = kb1;
        static_cast<T*>(kb.z)[g] = kb2;
    }
}

// Pass B of one stage alone (the last stage of a step's reverse).
template <typename T, int ANIS>
__global__ void __launch_bounds__(kAdjBlock)
    adj_pass_b(const RepDev R, State q, State loc, State sbar, State xbar, State kb, int stage) {
    SiteA c;
    if (!adj_site(R, c)) return;
    T k0, k1, k2;
    double D, e0, e1, e2;
    aniso_of<T, ANIS>(R, c.i, D, e0, e1, e2);
    adj_b_site<T, ANIS>(R, c, q, loc, sbar, xbar, kb, stage, D, e0, e1, e2, k0, k1, k2);
}

// Pass B of stage s followed by pass A of stage s - 1 at the same site: the
// cotangent of k_{s-1} is pointwise in B's result, so one launch does both
// (q, loc of stage s are read; qn, locn of stage s - 1 are written).  With
// stage = 1 the pass A is stage 4 of the step before (y its stage-4 input,
// scale dt/6), whose k4 cotangent is the finished xbar / 6.
template <typename T, bool PREC, int ANIS>
__global__ void __launch_bounds__(kAdjBlock)
    adj_pass_ba(const RepDev R, State q, State loc, State sbar, State xbar, State kb, int stage,
                State y, double scale, State qn, State locn, double* gD, double* part) {
    SiteA c;
    double v[5] = {0, 0, 0, 0, 0};
    if (adj_site(R, c)) {
        T k0, k1, k2;
        const AIn a = load_a_in<T, ANIS>(R, c, y, gD);
        adj_b_site<T, ANIS>(R, c, q, loc, sbar, xbar, kb, stage, a.D, a.e0, a.e1, a.e2, k0, k1,
                            k2);
        adj_a_site<T, PREC, ANIS>(R, c, a, scale * (double)k0, scale * (double)k1,
                                  scale * (double)k2, qn, locn, gD, v);
    }
    block_sum5(v, part);
}

// acc[0..4] += sum over blocks of part[b][0..4], in block order.
__global__ void __launch_bounds__(256) adj_reduce5(const double* part, int nblk, double* acc) {
    __shared__ double red[5][256];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int q = 0; q < 5; ++q) v[q] += part[(int64_t)b * 5 + q];
    for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 5) acc[threadIdx.x] += red[threadIdx.x][0];
}

// Kick reverse: s'' = s'/|s'|, s' = R s  =>  sbar = R^T (I - s'' s''^T) sbar'' / |s'|,
// R^T being the rotation by -phi about the same axis.
template <typename T>
__global__ void __launch_bounds__(kAdjBlock)
    adj_kick_kernel(const RepDev R, State spre, State sbar, uint64_t k, double sigma_override) {
    SiteA c;
    if (!adj_site(R, c)) return;
    const T sg = (T)(sigma_override >= 0.0 ? sigma_override : R.sigma);
    const uint4 w = philox_site(R.seed, (uint32_t)c.i, (uint32_t)(k + R.kbase), R.rid, 0u);
    T G[3];
    gauss3<T>(w, G);  // the same normals as the forward kick of this precision
    const double p0 = (double)(T)(sg * G[0]), p1 = (double)(T)(sg * G[1]), p2 = (double)(T)(sg * G[2]);
    const double ph = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
    const int64_t g = c.gi;
    const double s0 = static_cast<const T*>(spre.x)[g];
    const double s1 = static_cast<const T*>(spre.y)[g];
    const double s2 = static_cast<const T*>(spre.z)[g];
    double n0 = 0, n1 = 0, n2 = 1, cs = 1, sn = 0;
    if (ph > 0) {
        n0 = p0 / ph;
        n1 = p1 / ph;
        n2 = p2 / ph;
        sincos(ph, &sn, &cs);
    }
    auto rot = [&](double a0, double a1, double a2, double sgn, double& o0, double& o1, double& o2) {
        const double sns = sgn * sn;
        const double c0 = n1 * a2 - n2 * a1, c1 = n2 * a0 - n0 * a2, c2 = n0 * a1 - n1 * a0;
        const double an = a0 * n0 + a1 * n1 + a2 * n2;
        o0 = a0 * cs + c0 * sns + n0 * an * (1.0 - cs);
        o1 = a1 * cs + c1 * sns + n1 * an * (1.0 - cs);
        o2 = a2 * cs + c2 * sns + n2 * an * (1.0 - cs);
    };
    double r0, r1, r2;
    rot(s0, s1, s2, 1.0, r0, r1, r2);
    const double nrm = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    const double h0 = r0 / nrm, h1 = r1 / nrm, h2 = r2 / nrm;
    T* bx = static_cast<T*>(sbar.x);
    T* by = static_cast<T*>(sbar.y);
    T* bz = static_cast<T*>(sbar.z);
    const double b0 = bx[g], b1 = by[g], b2 = bz[g];
    const double hb = h0 * b0 + h1 * b1 + h2 * b2;
    const double q0 = (b0 - h0 * hb) / nrm, q1 = (b1 - h1 * hb) / nrm, q2 = (b2 - h2 * hb) / nrm;
    double o0, o1, o2;
    rot(q0, q1, q2, -1.0, o0, o1, o2);
    bx[g] = (T)o0;
    by[g] = (T)o1;
    bz[g] = (T)o2;
}

// ------------------------------------------------------------ launchers ----
template <typename T>
static hipError_t loss_t(int anis, const RepDev& R, int nblk, State s,
                         State cot, State sbar, double wE, const double wm[3], double* gD,
                         double* part, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: hipLaunchKernelGGL((adj_loss_kernel<T, ANIS_NONE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, s, cot, sbar, wE, wm[0], wm[1], wm[2], gD, part); break;
        case ANIS_SITE: hipLaunchKernelGGL((adj_loss_kernel<T, ANIS_SITE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, s, cot, sbar, wE, wm[0], wm[1], wm[2], gD, part); break;
        default: hipLaunchKernelGGL((adj_loss_kernel<T, ANIS_AXIS>), dim3(nblk), dim3(kAdjBlock), 0, st, R, s, cot, sbar, wE, wm[0], wm[1], wm[2], gD, part); break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_loss(int prec, int anis, const RepDev& R, int nblk,
                           State s, State cot, State sbar, double wE, const double wm[3],
                           double* gD, double* part, hipStream_t st) {
    return prec == 0 ? loss_t<double>(anis, R, nblk, s, cot, sbar, wE, wm, gD, part, st)
                     : loss_t<float>(anis, R, nblk, s, cot, sbar, wE, wm, gD, part, st);
}

hipError_t launch_adj_finish(const double* part, int nblk, double* acc, hipStream_t st) {
    hipLaunchKernelGGL(adj_reduce5, dim3(1), dim3(256), 0, st, part, nblk, acc);
    return hipGetLastError();
}

template <typename T, bool PREC>
static void pass_a_t(int anis, const RepDev& R, int nblk, State y, State kb,
                     double scale, State q, State loc, double* gD, double* part, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: hipLaunchKernelGGL((adj_pass_a<T, PREC, ANIS_NONE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, y, kb, scale, q, loc, gD, part); break;
        case ANIS_SITE: hipLaunchKernelGGL((adj_pass_a<T, PREC, ANIS_SITE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, y, kb, scale, q, loc, gD, part); break;
        default: hipLaunchKernelGGL((adj_pass_a<T, PREC, ANIS_AXIS>), dim3(nblk), dim3(kAdjBlock), 0, st, R, y, kb, scale, q, loc, gD, part); break;
    }
}

template <typename T>
static void pass_b_t(int anis, const RepDev& R, int nblk, State q, State loc,
                     State sbar, State xbar, State kb, int stage, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: hipLaunchKernelGGL((adj_pass_b<T, ANIS_NONE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage); break;
        case ANIS_SITE: hipLaunchKernelGGL((adj_pass_b<T, ANIS_SITE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage); break;
        default: hipLaunchKernelGGL((adj_pass_b<T, ANIS_AXIS>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage); break;
    }
}

template <typename T, bool PREC>
static void pass_ba_t(int anis, const RepDev& R, int nblk, State q, State loc,
                      State sbar, State xbar, State kb, int stage, State y, double scale, State qn,
                      State locn, double* gD, double* part, hipStream_t st) {
    switch (anis) {
        case ANIS_NONE: hipLaunchKernelGGL((adj_pass_ba<T, PREC, ANIS_NONE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage, y, scale, qn, locn, gD, part); break;
        case ANIS_SITE: hipLaunchKernelGGL((adj_pass_ba<T, PREC, ANIS_SITE>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage, y, scale, qn, locn, gD, part); break;
        default: hipLaunchKernelGGL((adj_pass_ba<T, PREC, ANIS_AXIS>), dim3(nblk), dim3(kAdjBlock), 0, st, R, q, loc, sbar, xbar, kb, stage, y, scale, qn, locn, gD, part); break;
    }
}

// Reverse of one RK4 step given its stage inputs y[0..3] and the cotangent
// sbar of its output; on return xbar holds the cotangent of its input.
// Launches: A of stage 4, then B of stage s fused with A of stage s - 1 for
// s = 4, 3, 2, then B of stage 1; q/loc alternate between two buffers.
// Parameter partials accumulate in part (reduced by launch_adj_finish).
hipError_t launch_adj_step(int prec, int precession, int anis, const RepDev& R, int nblk, const State y[4], double dt, State sbar,
                           State xbar, State kb, const State q[2], const State loc[2], double* gD,
                           double* part, bool a4, hipStream_t st) {
    hipError_t e;
    if (a4) {
        if (prec == 0) {
            if (precession) pass_a_t<double, true>(anis, R, nblk, y[3], sbar, dt / 6.0, q[0], loc[0], gD, part, st);
            else pass_a_t<double, false>(anis, R, nblk, y[3], sbar, dt / 6.0, q[0], loc[0], gD, part, st);
        } else {
            if (precession) pass_a_t<float, true>(anis, R, nblk, y[3], sbar, dt / 6.0, q[0], loc[0], gD, part, st);
            else pass_a_t<float, false>(anis, R, nblk, y[3], sbar, dt / 6.0, q[0], loc[0], gD, part, st);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int cur = 0;
    for (int s = 4; s >= 2; --s) {
        const State& qi = q[cur];
        const State& li = loc[cur];
        const State& qo = q[cur ^ 1];
        const State& lo = loc[cur ^ 1];
        if (prec == 0) {
            if (precession) pass_ba_t<double, true>(anis, R, nblk, qi, li, sbar, xbar, kb, s, y[s - 2], dt, qo, lo, gD, part, st);
            else pass_ba_t<double, false>(anis, R, nblk, qi, li, sbar, xbar, kb, s, y[s - 2], dt, qo, lo, gD, part, st);
        } else {
            if (precession) pass_ba_t<float, true>(anis, R, nblk, qi, li, sbar, xbar, kb, s, y[s - 2], dt, qo, lo, gD, part, st);
            else pass_ba_t<float, false>(anis, R, nblk, qi, li, sbar, xbar, kb, s, y[s - 2], dt, qo, lo, gD, part, st);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    return hipSuccess;
}

hipError_t launch_adj_b1(int prec, int precession, int anis, const RepDev& R, int nblk,
                         const State* y4prev, double dt, State sbar, State xbar, State kb,
                         const State q[2], const State loc[2], double* gD, double* part,
                         hipStream_t st) {
    if (!y4prev) {
        if (prec == 0) pass_b_t<double>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, st);
        else pass_b_t<float>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, st);
        return hipGetLastError();
    }
    const double sc = dt / 6.0;
    if (prec == 0) {
        if (precession) pass_ba_t<double, true>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, *y4prev, sc, q[0], loc[0], gD, part, st);
        else pass_ba_t<double, false>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, *y4prev, sc, q[0], loc[0], gD, part, st);
    } else {
        if (precession) pass_ba_t<float, true>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, *y4prev, sc, q[0], loc[0], gD, part, st);
        else pass_ba_t<float, false>(anis, R, nblk, q[1], loc[1], sbar, xbar, kb, 1, *y4prev, sc, q[0], loc[0], gD, part, st);
    }
    return hipGetLastError();
}

hipError_t launch_adj_kick(int prec, const RepDev& R, int nblk, State spre,
                           State sbar, uint64_t k, double sigma_override, hipStream_t st) {
    if (prec == 0)
        hipLaunchKernelGGL(adj_kick_kernel<double>, dim3(nblk), dim3(kAdjBlock), 0, st, R, spre, sbar, k, sigma_override);
    else
        hipLaunchKernelGGL(adj_kick_kernel<float>, dim3(nblk), dim3(kAdjBlock), 0, st, R, spre, sbar, k, sigma_override);
    return hipGetLastError();
}

}  // namespace lll
