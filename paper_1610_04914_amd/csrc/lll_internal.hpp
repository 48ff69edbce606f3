// Internal definitions shared by the host runtime and the kernel translation
// units of liblll (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lll {

enum AnisMode : int32_t { ANIS_NONE = 0, ANIS_Z = 1, ANIS_AXIS = 2, ANIS_SITE = 3 };

// Running maximum of the kick deviation | |s'| - 1 | of each replica: kKickSlots
// unsigned 64-bit slots holding bit patterns of non-negative doubles (which
// order as their bits, NaN above +inf); the maximum is the largest slot.
// Every kick launch folds its block or tile maxima into the slots with integer
// atomic max, spread by workgroup index so that workgroups finishing together
// do not queue on one address.
constexpr int kKickSlots = 64;

// One replica (a single lattice is a batch of one).  Lives in device memory;
// every kernel reads the descriptor of the replica it works on.
struct RepDev {
    int32_t Lx, Ly, Lz, bc;       // shape, boundary (0 periodic, 1 free)
    int64_t off;                  // first site of this replica in the packed SoA arrays
    int32_t tx, ty, tz, tile0;    // fused-kernel tiles per axis and first tile id
    int32_t ob0, nob;             // observables: first partial block and block count
    int32_t sb0, nsb;             // per-site kernels: first 256-site block and block count
    // Stage coefficients.  Precessional case: k = s x (h~ - lam (s x h~)),
    // h~ = dt h.  Slow equation: k = s x (s x h~), h~ = -lambda dt h.
    // h~ = cJ * sum_nn s + cH + cD * (s.e) e   (ANIS_SITE: cD * D_i (s.e_i) e_i).
    double cJ, cH[3], cD, e[3], lam;
    // Physics for the observables (e normalised).
    double J, H[3], D, pad2;
    double sigma;                 // default kick scale sqrt(2 lambda T Dt)
    double lambda, Dt;            // to rescale sigma for a per-pulse temperature
    uint64_t seed;
    // Added to the pulse index of every kick.  0 for a lattice; a batch sets
    // it before each replay of its captured schedule, whose kicks carry the
    // pulse index relative to the run's first pulse.
    uint64_t kbase;
    uint32_t rid;                 // Philox counter word 2
    int32_t init;                 // initial state: 0 random sphere, 1 along the init direction
    const void* D_site;           // ANIS_SITE: [N] of the state precision
    const void* e_site;           // ANIS_SITE: [3N] of the state precision
};

struct State {
    void* x;
    void* y;
    void* z;
};

// Kernel launchers (defined in the .hip translation units).  prec: 0 fp64, 1 fp32.
hipError_t launch_philox_words(uint64_t seed, uint32_t i0, int64_t n, uint32_t c1, uint32_t c2,
                               uint32_t c3, uint32_t* out, hipStream_t st);
hipError_t launch_init(int prec, const RepDev* reps, const int32_t* blk_rep, int nblk, State s,
                       int mode, double dx, double dy, double dz, hipStream_t st);
// sigma_override >= 0 replaces every replica's kick scale (per-pulse temperature).
// Each block folds its maximum of | |s'| - 1 | into the running-maximum slots
// of its replica in kickdev ([nrep][kKickSlots]).
// Sets kbase of every replica's device descriptor to base.
hipError_t launch_set_pulse_base(RepDev* reps, int nrep, uint64_t base, hipStream_t st);
hipError_t launch_kick(int prec, const RepDev* reps, const int32_t* blk_rep, int nblk, State s,
                       uint64_t k, double sigma_override, unsigned long long* kickdev,
                       hipStream_t st);
// Work items of the observables pass for an Lx x Ly x Lz lattice (runs of
// columns over z-slabs); a replica needs at most this many blocks.
int64_t obs_item_count(int Lx, int Ly, int Lz);
// Observables of every replica into result[r][8] (and accum when accumulate);
// partials: [nobblk][8] scratch.
hipError_t launch_obs(int prec, int anis, const RepDev* reps, const int32_t* oblk_rep,
                      int nobblk, int nrep, State s, double* partials, double* result,
                      double* accum, int accumulate, hipStream_t st);
// Staged observables: launch_obs_partials writes the per-block partials of one
// measurement ([nobblk][8], the first pass of launch_obs); launch_obs_staged
// then reduces n staged measurements at once (measurement j's partials at
// stage + j * nobblk * 8) into out + j * ostride + r * 8, adds them to the
// running sums accum[r] in measurement order and copies the last one to
// result[r].  The values and sums equal those of n launch_obs calls with
// accumulate.
hipError_t launch_obs_partials(int prec, int anis, const RepDev* reps, const int32_t* oblk_rep,
                               int nobblk, State s, double* partials, hipStream_t st);
hipError_t launch_obs_staged(int anis, const RepDev* reps, int nrep, int nobblk, int n,
                             const double* stage, double* out, int64_t ostride, double* accum,
                             double* result, hipStream_t st);
// Unfused RK4 step: four stage launches; scratch yA, yB, acc of the same shape.
hipError_t launch_step_unfused(int prec, int precession, int anis, const RepDev* reps,
                               const int32_t* blk_rep, int nblk, State s, State yA, State yB,
                               State acc, hipStream_t st);
hipError_t launch_copy(int prec, State dst, State src, int64_t n, hipStream_t st);

// Explicit Runge-Kutta tableau of up to six stages: stage j's input is
// x + sum_{l<j} a[j][l] k_l, the step is x + sum_l b[l] k_l (k_l = dt f).
struct Tableau {
    int stages;
    double a[6][6];
    double b[6];
};
// Scratch arrays of the stage increments k_0 .. k_{stages-2}.
struct KSet {
    State K[6];
};
// One step of the tableau with one launch per stage (yA, yB: stage-input scratch).
hipError_t launch_step_tableau(int prec, int precession, int anis, const RepDev* reps,
                               const int32_t* blk_rep, int nblk, const Tableau& tb, State s,
                               State yA, State yB, const KSet& ks, hipStream_t st);

// Escape runs of single spins (see kern_escape.hip): pulses k0 .. k1-1 of
// n_runs runs with state sx/sy/sz and times (negative = still running).
hipError_t launch_escape(const RepDev& R, const Tableau& tb, int precession, int64_t n_runs,
                         int64_t n, double dt, int64_t k0, int64_t k1, double h, double* sx,
                         double* sy, double* sz, double* times, unsigned int* active,
                         hipStream_t st);

// Fused RK4 step (one launch per step, z-marching LDS tiles).
struct FusedInfo {
    int bx, by, threads, lds_bytes;
};
int fused_variant_count(int prec);
bool fused_variant_info(int prec, int variant, FusedInfo* out);
// Event pair that a launch records at its own start and end (kernel timing).
struct LaunchEvents {
    hipEvent_t start, stop;
};
// kick != 0: apply kick number k to the step's output (epilogue), folding each
// tile's maximum of | |s'| - 1 | into one of the replica's kKickSlots slots
// of kickdev (integer atomic max); sigma_override >= 0
// replaces every replica's kick scale.  ev (optional, steps without kick only)
// times the launch.
// scheme: 0 one RK4 step, 1 two RK2-midpoint steps, 2 one RK2-midpoint step.
hipError_t launch_step_fused(int prec, int precession, int anis, int variant, int bz, int scheme,
                             const RepDev* reps, const int4* tiles, int ntiles, State in,
                             State out, int kick, uint64_t k, double sigma_override,
                             unsigned long long* kickdev, const LaunchEvents* ev, hipStream_t st);

// Fused Butcher RK5 step (Appendix) in two launches: stages 1-4 from in into
// the scratch states k[0] (Y5), k[1] (Q6), k[2] (R), then stages 5-6 into out,
// with kick number kp as the epilogue when kick != 0 (as launch_step_fused).
// The variant has the tile shape of the same RK4 variant.
hipError_t launch_step_rk5_fused(int prec, int precession, int anis, int variant, int bz,
                                 const RepDev* reps, const int4* tiles, int ntiles, State in,
                                 State out, const State* k, int kick, uint64_t kp, double so,
                                 unsigned long long* kd, hipStream_t st);

// Fused RK4 step from in to out (same bits as launch_step_fused without a
// kick) that also writes its stage inputs y2, y3, y4 into y[0..2].
hipError_t launch_step_fused_stages(int prec, int precession, int anis, int variant, int bz,
                                    const RepDev* reps, const int4* tiles, int ntiles, State in,
                                    State out, const State* y, hipStream_t st);

// RK4 step keeping the stage inputs y2, y3, y4 (per-stage launches).
hipError_t launch_rk4_stages(int prec, int precession, int anis, const RepDev* reps,
                             const int32_t* blk_rep, int nblk, State x, State y2, State y3,
                             State y4, State acc, State xnext, hipStream_t st);

// Adjoint kernels (256-site blocks, the same block table as the per-site kernels).
// part: [nblk][5] fp64 running partials {Hbar x3, Jbar, Dbar} (zeroed by the
// caller, added to by every pass, reduced in block order into acc[5] by
// launch_adj_finish); gD: per-site fp64 Dbar_i (per-site anisotropy) or unused.
// Adjoint launchers take the lattice's descriptor by value (host copy; the
// adjoint runs on one lattice).  Their per-site kernels run one wave per
// block, kAdjBlock sites: nblk = ceil(N / kAdjBlock) blocks, and as many rows
// of parameter partials.
constexpr int kAdjBlock = 64;
// cot: cotangent of s added to the loss's own (null pointers: none).
hipError_t launch_adj_loss(int prec, int anis, const RepDev& R, int nblk,
                           State s, State cot, State sbar, double wE, const double wm[3],
                           double* gD, double* part, hipStream_t st);
// Reverse of one RK4 step up to its last stage: pass A of stage 4 (unless a4
// is false: then a launch_adj_b1 of the step after has done it), then passes
// B + A of stages 4..2.  q[2], loc[2]: two scratch pairs used alternately;
// stage 4's q is q[0], stage 1's q[1].
hipError_t launch_adj_step(int prec, int precession, int anis, const RepDev& R, int nblk, const State y[4], double dt, State sbar,
                           State xbar, State kb, const State q[2], const State loc[2], double* gD,
                           double* part, bool a4, hipStream_t st);
// Pass B of stage 1, which finishes xbar; with y4prev (the stage-4 input of
// the step before) the same launch also does that step's pass A of stage 4.
hipError_t launch_adj_b1(int prec, int precession, int anis, const RepDev& R, int nblk, const State* y4prev, double dt, State sbar,
                         State xbar, State kb, const State q[2], const State loc[2], double* gD,
                         double* part, hipStream_t st);
hipError_t launch_adj_finish(const double* part, int nblk, double* acc, hipStream_t st);
hipError_t launch_adj_kick(int prec, const RepDev& R, int nblk, State spre,
                           State sbar, uint64_t k, double sigma_override, hipStream_t st);
}  // namespace lll
