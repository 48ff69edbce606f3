/*
 * lll.h -- C ABI of the MI355X (gfx950) pulse-noise Landau-Lifshitz-Langevin
 * library (D. A. Garanin, "Pulse-noise approach for classical spin systems",
 * arXiv:1610.04914).
 *
 * The library integrates a simple-cubic lattice of classical unit spins:
 *   - between noise pulses, the noise-free Landau-Lifshitz equation
 *     (Eq. (1) with zeta = 0, gamma = 1):
 *        ds_i/dt = s_i x h_i - lambda s_i x (s_i x h_i)
 *     (the slow equation of Sec. II drops the first term), with classical
 *     fourth-order Runge-Kutta steps of size dt;
 *   - the effective field h_i = J sum_{6 neighbours} s_j + H + 2 D_i (s_i.e_i) e_i
 *     belongs to E = -J sum_<ij> s_i.s_j - sum_i H.s_i - sum_i D_i (s_i.e_i)^2
 *     (each bond counted once; anisotropy convention of Eq. (12));
 *   - every Delta t = n dt a pulse-noise kick (Eqs. (5)-(6)): each spin is
 *     rotated by the vector angle phi = sqrt(2 lambda T Delta t) G, G a vector
 *     of three unit normals, and renormalised to unit length;
 *   - the kick sits in the middle of each interval (Eq. (7)): an interval is
 *     n1 = floor(n/2) steps, kick, n2 = n - n1 steps, measurement.
 * Units: gamma = mu_0 = k_B = 1.
 *
 * Memory: spins are stored structure-of-arrays (three arrays sx, sy, sz of N
 * elements each, site index i = x + Lx*(y + Ly*z)) in device memory, in fp64
 * (double) or fp32 (float).  Energies, magnetisation and the renormalisation
 * check are always computed in fp64.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with counter
 * (site i, pulse k mod 2^32, replica r, tag) and key (seed lo32, seed hi32);
 * tag 0 = kick, tag 1 = random-sphere initial state.  u = (w + 1/2) 2^-32;
 * normals by Box-Muller: G = (sqrt(-2 ln u0) cos 2pi u1,
 * sqrt(-2 ln u0) sin 2pi u1, sqrt(-2 ln u2) cos 2pi u3).
 *
 * Conventions for every entry point:
 *   - all functions return lll_status; 0 = success, < 0 = error (nothing was
 *     enqueued unless stated), > 0 = warning (the work was done);
 *   - after a non-zero status, lll_last_error() returns a message (per thread);
 *   - all GPU work is enqueued on the handle's HIP stream in call order; only
 *     calls that return host data (lll_observables, lll_run with a trace,
 *     lll_accumulators, lll_kick_norm_dev, batch observables, the adjoint)
 *     synchronise that stream;
 *   - a handle must not be used by two host threads at once.
 */
#ifndef LLL_H
#define LLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LLL_OK = 0,
    LLL_EINVAL = -1,        /* invalid argument (null pointer, bad size, non-integral Dt/dt, ...) */
    LLL_ENOMEM = -2,        /* device allocation failed */
    LLL_EDEVICE = -3,       /* a HIP runtime call failed */
    LLL_EUNSUPPORTED = -4,  /* valid request the library or the device does not support */
    LLL_ENONFINITE = -5,    /* a NaN/Inf was found in the state by a reduction */
    LLL_WARN_APPLICABILITY = 1, /* work done, but Eq. (8)/(9) or the step-size rule is violated */
    LLL_WARN_NORM = 2       /* work done, but a measured state has some | |s_i| - 1 | above
                               LLL_NORM_WARN_LEVEL: the spin length, conserved by Eq. (1), has
                               drifted that far within an interval (delta t too large for the
                               local fields); takes precedence over LLL_WARN_APPLICABILITY */
} lll_status;

/* Threshold of LLL_WARN_NORM on max_i | |s_i| - 1 | of a measured state. */
#define LLL_NORM_WARN_LEVEL 0.5

typedef enum { LLL_FP64 = 0, LLL_FP32 = 1 } lll_precision;
typedef enum { LLL_BC_PERIODIC = 0, LLL_BC_FREE = 1 } lll_bc;
typedef enum {
    LLL_INIT_RANDOM_SPHERE = 0, /* uniform on the sphere from Philox tag 1 */
    LLL_INIT_DIRECTION = 1,     /* every spin along dir (normalised) */
    LLL_INIT_KEEP = 2           /* the caller has filled the buffers it passes */
} lll_init;
/* Step integrators (Appendix).  LLL_RK4: classical fourth order, one fused
 * launch per step.  LLL_RK2MID: midpoint, K1 = dt f(x), K2 = dt f(x + K1/2),
 * x' = x + K2 (fused: two steps per launch).  LLL_RK5B: Butcher's six-stage
 * fifth-order method (the paper's main solver; fused: two launches per step,
 * stages 1-4 and stages 5-6).  With the unfused step configuration
 * (variant 0), RK2MID and RK5B run one launch per stage.  Neither is
 * available to the adjoint or the batch. */
typedef enum { LLL_RK4 = 0, LLL_RK2MID = 1, LLL_RK5B = 2 } lll_integrator;

/* Physical and numerical parameters, copied on every call.  Thresholds of the
 * applicability warning: 2 lambda T Dt > 0.2 (Eq. (8)); lambda h_max Dt > 0.2
 * (Eq. (9)); with precession, h_max dt > 0.25 (Sec. II, step-size rule), where
 * h_max = 6|J| + |H| + 2|D|. */
typedef struct {
    double J;             /* exchange constant */
    double H[3];          /* external field */
    double D;             /* uniform uniaxial anisotropy (ignored when D_site is set) */
    double e[3];          /* uniform easy axis, normalised by the library; (0,0,0) means z */
    const void* D_site;   /* optional device array [N] of the lattice precision: per-site D_i,
                             caller-owned, must stay valid while the handle uses it */
    const void* e_site;   /* optional device array [3*N] (x block, y block, z block) of the
                             lattice precision: per-site unit easy axes; needs D_site */
    double lambda;        /* damping, >= 0 */
    double T;             /* temperature, >= 0 (T = 0: the kick only renormalises) */
    double dt;            /* RK4 step, > 0 */
    double Dt;            /* pulse spacing; Dt/dt must be an integer n >= 1 (|Dt/dt - n| <= 1e-9 n) */
    int32_t precession;   /* 1: full Eq. (1); 0: slow equation (precession dropped) */
    int32_t integrator;   /* lll_integrator */
    uint64_t seed;        /* Philox key of the kicks */
    uint32_t replica;     /* Philox counter word 2 of the kicks: 0 for a lone lattice; set it to
                             a batch replica's index to draw that replica's noise */
    int32_t reserved;     /* set to 0 */
} lll_params;

/* Observables of one state, fp64. */
typedef struct {
    double E_total, E_exch, E_zeeman, E_anis; /* energies (sums over the lattice) */
    double m[3];                              /* magnetisation per site, sum_i s_i / N */
    double max_norm_dev;                      /* max_i | |s_i| - 1 | */
} lll_obs;

typedef struct lll_lattice lll_lattice;
typedef struct lll_batch lll_batch;

/* Creates a lattice of Lx*Ly*Lz sites on the current HIP device, with the
 * starting states of the paper's runs: spins uniformly distributed on the
 * sphere (the disordered start of the many-spin runs of Sec. IV), or all
 * along one direction (the ordered starts of Secs. III-IV).
 * sx, sy, sz: caller-owned device buffers of N elements of the precision
 * (all three or none); when NULL the library allocates and owns them.
 * hip_stream: the hipStream_t to enqueue on (NULL = the default stream).
 * mode/dir/seed: initial state (dir is read for LLL_INIT_DIRECTION only; the
 * seed keys the random sphere, replica 0).
 * On success *out receives the handle.  Errors: LLL_EINVAL (L < 1, null out,
 * partial buffers, dir zero, more than 2^31 - 1 sites), LLL_ENOMEM, LLL_EDEVICE. */
lll_status lll_init_lattice(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc, lll_precision prec,
                            lll_init mode, const double dir[3], uint64_t seed, void* sx, void* sy,
                            void* sz, void* hip_stream, lll_lattice** out);

/* n_steps >= 0 steps of size dt of the noise-free equation (Eq. (1) with
 * zeta = 0; no renormalisation), with the integrator params->integrator
 * (classical RK4 unless it names another).  Only params' physics, dt and
 * integrator are used. */
lll_status lll_step_conservative(lll_lattice* lat, const lll_params* params, int64_t n_steps);

/* One pulse-noise kick with pulse index pulse_index at temperature params->T
 * (Eqs. (5)-(6)) followed by renormalisation of every spin.  Stateless: the
 * noise depends only on (params->seed, site, pulse_index, params->replica). */
lll_status lll_noise_pulse(lll_lattice* lat, const lll_params* params, uint64_t pulse_index);

/* Observables of the current state into *out_host (synchronises the stream):
 * the energy of Eq. (1)'s Hamiltonian split into exchange, Zeeman and
 * anisotropy parts, the magnetisation per site and the largest spin-length
 * deviation, the quantities the paper measures at the end of each noise
 * interval (Sec. III.A) and averages over a run (Sec. IV).
 * LLL_ENONFINITE when the state holds a NaN or Inf; LLL_WARN_NORM when its
 * max_norm_dev exceeds LLL_NORM_WARN_LEVEL (out_host is filled in both cases). */
lll_status lll_observables(lll_lattice* lat, const lll_params* params, lll_obs* out_host);

/* n_pulses intervals (n1 steps, kick k, n2 steps) for k = first_pulse ...
 * first_pulse + n_pulses - 1.  T_per_pulse: optional host array [n_pulses] of
 * kick temperatures (NULL: params->T).  When obs_every > 0 and trace != NULL,
 * the observables after every obs_every-th interval are written to
 * trace[0 .. n_pulses/obs_every) (host memory; the call then synchronises).
 * Calling step(n1), pulse(k), step(n2) in order gives the same result bit for
 * bit.  Returns LLL_ENONFINITE when a traced measurement holds a NaN or Inf;
 * after doing the work, LLL_WARN_NORM (> 0) when a traced measurement's
 * max_norm_dev exceeds LLL_NORM_WARN_LEVEL, else LLL_WARN_APPLICABILITY (> 0)
 * when the parameters violate the applicability conditions. */
lll_status lll_run(lll_lattice* lat, const lll_params* params, uint64_t first_pulse,
                   int64_t n_pulses, const double* T_per_pulse, int32_t obs_every,
                   lll_obs* trace);

/* Device pointers of the current state (valid until lll_destroy). */
lll_status lll_get_state(lll_lattice* lat, void** sx, void** sy, void** sz);

/* Largest | |s'| - 1 | before renormalisation over all kicks since the last
 * reset, fp64 (synchronises).  reset != 0 clears it afterwards. */
lll_status lll_kick_norm_dev(lll_lattice* lat, double* out_host, int32_t reset);

/* FP64 running sums over measured intervals since the last reset, out_host[8] =
 * {count, sum E_total, sum E_total^2, sum |m|, sum |m|^2, sum m_x, sum m_y,
 * sum m_z}.  Synchronises; reset != 0 clears them afterwards. */
lll_status lll_accumulators(lll_lattice* lat, double* out_host, int32_t reset);

/* Kernel configuration of the RK4 step.  variant: 0 = unfused (one launch per
 * RK stage), 1..LLL_N_FUSED = fused tile shapes listed by
 * lll_step_variant_info; bz = z-chunk of the fused kernel (0 = automatic). */
lll_status lll_set_step_config(lll_lattice* lat, int32_t variant, int32_t bz);
lll_status lll_get_step_config(lll_lattice* lat, int32_t* variant, int32_t* bz);
/* Where the pulse-noise kick runs when the fused step is used: fused != 0 as
 * the epilogue of the step that precedes it (default), else as a launch of its
 * own.  Results are identical; only the timing differs.  No effect on the
 * unfused step. */
lll_status lll_set_kick_fusion(lll_lattice* lat, int32_t fused);
/* Kernel timing of the fused RK4 step (launches without kick epilogue).
 * enable != 0 starts a measurement: every 16th later launch records events
 * taken from its own dispatch into a ring of 64 pairs (a pair still in flight
 * is skipped), so the timed launches are a sample spread over the run.  A
 * launch that records its own events starts a few microseconds later, so
 * timing every launch would slow the run it measures.
 * enable == 0 synchronises the lattice's stream, ends the measurement and
 * returns the mean kernel duration *avg_ms over *n_timed launches (either
 * pointer may be NULL; 0 launches gives 0.0). */
lll_status lll_kernel_timing(lll_lattice* lat, int32_t enable, double* avg_ms, int64_t* n_timed);
/* Tile shape of a variant for a precision: out[0..3] = {bx, by, threads, lds_bytes};
 * LLL_EINVAL past the last variant. */
lll_status lll_step_variant_info(lll_precision prec, int32_t variant, int32_t* out4);

/* Times every step configuration on this lattice (RK4 steps with params,
 * restoring the state afterwards) and selects the fastest, then the faster
 * kick placement (lll_set_kick_fusion) over whole noise intervals.  The state
 * and the kick-deviation maximum are restored.  cache_path (optional) is a
 * text file of "key variant bz kick_fused" lines (a missing fourth field means
 * fused) that is read first and updated; the key is the shape, precision,
 * boundary, precession, anisotropy mode and integrator.  *chosen_variant and *chosen_bz
 * may be NULL. */
lll_status lll_autotune(lll_lattice* lat, const lll_params* params, const char* cache_path,
                        int32_t* chosen_variant, int32_t* chosen_bz);

/* Discrete adjoint (reverse mode) of lll_run.  The paper has no adjoint;
 * this differentiates its schedule (Eq. (7): n1 RK4 steps, the kick of
 * Eqs. (5)-(6), n2 steps, per interval) with the kicks held fixed by the seed,
 * for a loss L(s_T) of the final state plus the energy terms below.
 *
 * lll_adjoint_forward: runs n_pulses intervals from the current state exactly
 * as lll_run does (same kernels, same bits, no measurements; the kicks fold
 * into the lattice's kick-deviation maximum) and records a tape: the state
 * before every ckpt_every-th operation (one RK4 step or one kick) and the
 * final state s_T, which is also left in the lattice.  ckpt_every =
 * LLL_TAPE_FULL (0) records instead the stage inputs x, y2 = x + k1/2,
 * y3 = x + k2/2, y4 = x + k3 of every step (and the state before every
 * kick): 4 states per operation plus s_T, 3 N (4 n_ops + 1) elements of the
 * lattice precision, so that the backward recomputes nothing (the same
 * bits as the checkpointed tape).  Tape memory is device memory allocated
 * by the call (LLL_ENOMEM when it does not fit).  The tape keeps a copy
 * of params; params->D_site / e_site must stay valid until the tape is
 * destroyed.  Only LLL_RK4.  On success *tape receives the handle.
 *
 * lll_adjoint_backward: gradients of
 *     L = <cot, s_T> + wE * E(s_T) + wm . m(s_T)
 * with respect to the initial state and the parameters.  cot (optional,
 * NULL = 0) is a device array [3*N] of the lattice precision (x block, y
 * block, z block): the cotangent dL/ds_T of whatever loss the caller computes
 * from s_T itself.  Each call recomputes every checkpoint block (none for a
 * full tape), so a tape can be reversed any number of times.  Outputs: *loss (may be NULL) =
 * wE E(s_T) + wm . m(s_T) (the caller's own term is not included); g_H[3],
 * *g_J (host); g_D: host double[1] = dL/dD when the tape's D_site is NULL,
 * else a device fp64 array [N] of dL/dD_i; g_s0 (optional): device array
 * [3*N] of the lattice precision = dL/ds_0.  Synchronises the lattice's
 * stream.  The lattice's state and kick maximum are not touched.
 * LLL_EINVAL when the tape's lattice has been destroyed.
 *
 * lll_tape_destroy: frees the tape (its checkpoint buffer is handed back to
 * the lattice and reused by its next forward).  Tapes may be destroyed
 * before or after their lattice.
 *
 * lll_adjoint: forward, backward with cot = NULL, and the initial state
 * restored, in one call (the lattice's state and kick maximum are left as
 * they were).
 *
 * Work buffers of the backward pass (2 (4 ckpt_every + 1) + 8 states; 8 for
 * a full tape) stay with the lattice and are reused.  With checkpoints
 * the backward recomputes the next block on a second stream of the
 * lattice's (created on first use, default priority) while the current
 * block is reversed, ordered by events; all of it is complete when the call
 * returns.  ckpt_every < 0 is LLL_EINVAL. */
#define LLL_TAPE_FULL 0
typedef struct lll_tape lll_tape;
lll_status lll_adjoint_forward(lll_lattice* lat, const lll_params* params, uint64_t first_pulse,
                               int64_t n_pulses, int32_t ckpt_every, lll_tape** tape);
lll_status lll_adjoint_backward(lll_tape* tape, const void* cot, double wE, const double wm[3],
                                double* loss, double* g_H, double* g_J, void* g_D, void* g_s0);
void lll_tape_destroy(lll_tape* tape);
lll_status lll_adjoint(lll_lattice* lat, const lll_params* params, uint64_t first_pulse,
                       int64_t n_pulses, int32_t ckpt_every, double wE, const double wm[3],
                       double* loss, double* g_H, double* g_J, void* g_D, void* g_s0);

void lll_destroy(lll_lattice* lat);

/* ---------------------------------------------------------------- batch --
 * Many independent replicas (uneven sizes, own T, lambda, seed) advanced
 * together: every kernel of the schedule covers all replicas in one launch,
 * and a run is replayed from captured HIP graphs.  Spins of all replicas live in
 * one packed SoA allocation owned by the batch. */
typedef struct {
    int32_t Lx, Ly, Lz;
    int32_t bc;          /* lll_bc */
    double J, H[3], D, e[3];
    double lambda, T;
    uint64_t seed;       /* Philox key of this replica */
    uint32_t replica;    /* Philox counter word 2 of this replica */
    int32_t init;        /* lll_init: RANDOM_SPHERE (keyed by seed, replica) or DIRECTION (+z) */
} lll_replica_desc;

lll_status lll_batch_create(int32_t n_rep, const lll_replica_desc* reps, lll_precision prec,
                            double dt, double Dt, int32_t precession, void* hip_stream,
                            lll_batch** out);
/* Runs n_pulses intervals on every replica.  trace (optional, host):
 * [n_pulses/obs_every][n_rep] lll_obs; with a trace the call synchronises and
 * returns LLL_ENONFINITE or LLL_WARN_NORM as lll_run does, over all replicas.
 * The schedule is captured as a HIP graph on the first call with a given
 * (n_pulses, obs_every) and replayed by later calls with the same pair, for any
 * first_pulse (a long run made of equal chunks captures once).  A run longer
 * than 1000 pulses is done as chunks of at most 1000 (a whole number of
 * obs_every; with obs_every above 1000, each measurement period as unmeasured
 * chunks and a last one measured at its end), each a replay of one of three
 * graphs kept by the batch; the results are those of one run. */
lll_status lll_batch_run(lll_batch* b, uint64_t first_pulse, int64_t n_pulses, int32_t obs_every,
                         lll_obs* trace);
/* Observables of every replica's current state (synchronises); statuses as
 * lll_observables, over all replicas. */
lll_status lll_batch_observables(lll_batch* b, lll_obs* out_host /* [n_rep] */);
lll_status lll_batch_state(lll_batch* b, int32_t rep, void** sx, void** sy, void** sz);
/* FP64 running sums of every replica since creation: out_host[8*n_rep] as in lll_accumulators. */
lll_status lll_batch_accumulators(lll_batch* b, double* out_host, int32_t reset);
/* As lll_autotune, for the step kernel that advances all replicas together
 * (one tile shape for every replica); the states are restored. */
lll_status lll_batch_autotune(lll_batch* b, const char* cache_path, int32_t* chosen_variant,
                              int32_t* chosen_bz);
void lll_batch_destroy(lll_batch* b);

/* ------------------------------------------------------------- escape --- */
/* Thermally activated escape of a uniaxial spin in a transverse field
 * (Sec. III.B): E = -D s_z^2 - H s_x with h = H/(2D) in [0, 1), minima at
 * sin(theta) = h, saddle at s = (1, 0, 0), barrier D (1 - h)^2. */
typedef struct {
    double D;             /* uniaxial anisotropy along z, > 0 */
    double H;             /* transverse field along x, 0 <= H < 2D */
    double lambda;        /* damping, >= 0 */
    double T;             /* temperature, >= 0 */
    double dt;            /* integration step, > 0 */
    double Dt;            /* pulse spacing; Dt/dt an integer n >= 1 */
    int32_t precession;   /* 1: full Eq. (1); 0: slow equation */
    int32_t integrator;   /* lll_integrator (the paper used LLL_RK5B) */
    uint64_t seed;        /* Philox key of the kicks */
    uint32_t replica;     /* Philox counter word 2 */
    int32_t reserved;     /* set to 0 */
} lll_escape_params;

/* First-passage times of n_runs independent spins, each started at the bottom
 * of the well (phi = 0, sin theta = h: s = (h, 0, sqrt(1 - h^2))) and run
 * through the pulse-noise schedule (n1 = floor(n/2) steps, kick, n - n1 steps
 * per interval, pulses 0, 1, ...; run i draws the normals of pulse k from
 * counter (i, k, replica, 0)) until s_z < 0.  times_dev: caller-owned device
 * array of n_runs doubles (n_runs < 2^32); entry i receives the number of
 * completed steps times dt at the first step end or kick after which s_z < 0,
 * or -1 if that does not happen within max_pulses intervals.  The escape rate
 * is 1 / mean time (Sec. III.B).  Work is enqueued on hip_stream in bounded
 * launches of a few hundred pulses; the call synchronises the stream after
 * each one and returns once every run has escaped or max_pulses is reached.
 * Errors: LLL_EINVAL for invalid parameters or sizes, LLL_ENOMEM, LLL_EDEVICE. */
lll_status lll_escape_times(const lll_escape_params* p, int64_t n_runs, int64_t max_pulses,
                            double* times_dev, void* hip_stream);

/* ---------------------------------------------------------- no-alloc --- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of lll_observables for a state the caller holds, without a
 * handle and without allocating.  Lx, Ly, Lz, bc, prec describe the lattice
 * as for lll_init_lattice; params supplies J, H, D, e, D_site and e_site
 * (the rest is ignored); sx, sy, sz are the caller's device arrays of N
 * elements of the precision (read only).  out_dev: caller-owned device array
 * of 8 doubles receiving {E_total, E_exch, E_zeeman, E_anis, m_x, m_y, m_z,
 * max_norm_dev} (the lll_obs order), bit for bit what lll_observables reports
 * for the same state.  Work is enqueued on hip_stream (NULL = default
 * stream); the call does not synchronise, so it does not check the result
 * for NaN or Inf (the caller reads out_dev).  The call allocates nothing:
 * the kernels use a fixed 139,520-byte device array of the library (the
 * replica descriptor, its block table and at most 2048 blocks of partials;
 * every lattice size maps onto that many blocks), one copy per device, held
 * until the process ends, set up on the first call on each device.  Every
 * call on a device shares that device's array, so calls that overlap on one
 * device (different streams, or different host threads) race; calls on one
 * stream run one after another.  Errors (nothing enqueued): LLL_EINVAL for
 * NULL pointers, sizes < 1 or beyond 2^31 - 1 sites, invalid parameters;
 * LLL_EDEVICE when the device array cannot be located or a launch fails. */
lll_status lll_observables_noalloc(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc,
                                   lll_precision prec, const lll_params* params, const void* sx,
                                   const void* sy, const void* sz, double* out_dev,
                                   void* hip_stream);

/* ---------------------------------------------------------------- misc --- */
/* Philox4x32-10 words for counters (i0 + j, c1, c2, c3), j < n, key = seed,
 * into the device array out_dev[4*n] (enqueued on hip_stream). */
lll_status lll_philox4x32_10(uint64_t seed, uint32_t i0, int64_t n, uint32_t c1, uint32_t c2,
                             uint32_t c3, uint32_t* out_dev, void* hip_stream);

const char* lll_last_error(void);
const char* lll_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LLL_H */
