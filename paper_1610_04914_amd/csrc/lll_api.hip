// Host runtime and C ABI of liblll: lattice and batch handles, parameter
// validation, the interval schedule of the pulse-noise method (Eq. (7): n1
// steps, kick, n2 steps, measurement), graph capture of batched runs, and
// the autotuner of the RK4 step kernel.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/lll.h"
#include "lll_internal.hpp"
#include "tile_order.hpp"

using namespace lll;

// ------------------------------------------------------------- errors -----
static thread_local std::string g_err;

static lll_status set_err(lll_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_err(LLL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

extern "C" const char* lll_last_error(void) { return g_err.c_str(); }
extern "C" const char* lll_version(void) { return "lll-mi355x 0.1 (gfx950)"; }

// ------------------------------------------------------------- engine -----
namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Engine {
    int prec = 0;          // 0 fp64, 1 fp32
    size_t esz = 8;
    hipStream_t st = nullptr;
    int nrep = 0;
    int64_t nsites = 0;
    std::vector<RepDev> hreps;
    RepDev* dreps = nullptr;
    int precession = 1;
    int anis = ANIS_NONE;
    State s{};             // current state at API boundaries
    State alt{};           // second state buffer of the fused ping-pong
    State yA{}, yB{}, acc{};
    bool own_s = false;
    int32_t* d_blk_rep = nullptr;
    int nblk = 0;
    int32_t* d_oblk_rep = nullptr;
    int nobblk = 0;
    int4* d_tiles = nullptr;
    int ntiles = 0, tiles_variant = -1, tiles_bz = -1, tiles_cap = 0;
    double* d_partials = nullptr;
    double* d_result = nullptr;   // [nrep][8]
    double* d_accum = nullptr;    // [nrep][8]
    unsigned long long* d_kickdev = nullptr;  // [nrep][kKickSlots]
    bool kick_epilogue = true;     // kick as the fused step's epilogue (else its own launch)
    // With n = 1 (kick first in every interval) the next interval's kick can be
    // applied as the epilogue of this interval's step; carried_k then names
    // the pulse already applied, which the next interval skips.
    bool carried = false;
    uint64_t carried_k = 0;
    double* d_trace = nullptr;
    size_t trace_cap = 0;         // doubles
    // Measurements of a run are staged: each leaves its per-block partials in
    // d_obs_stage, and obs_fold reduces all staged ones in one launch (plus
    // the running sums), instead of one reduction launch per measurement.
    double* d_obs_stage = nullptr;  // [obs_cap][nobblk][8]
    double* d_obs_vals = nullptr;   // [obs_cap][nrep][8], values when no trace is kept
    int obs_cap = 0;
    int obs_n = 0;                  // staged and not yet reduced
    double* obs_out = nullptr;      // where the next reduced measurement goes (trace) or null
    int64_t obs_stride = 0;         // doubles between consecutive measurements in obs_out
    int variant = 0, bz = 0;      // step configuration (0 = unfused)
    int integrator = 0;           // lll_integrator; other than RK4 runs the per-stage tableau path
    State Kt[6]{};                // stage increments of the tableau path
    int cur = 0;                  // 0: state in s, 1: state in alt
    // kernel timing of fused steps without kick: a ring of event pairs that the
    // launches record themselves; a pair still in flight is skipped, so the
    // timed launches are a sample spread over the run
    bool kt_on = false;
    std::vector<LaunchEvents> kt_ev;
    std::vector<char> kt_busy;
    size_t kt_next = 0;
    uint64_t kt_seq = 0;  // fused launches since the measurement started
    double kt_ms = 0;
    int64_t kt_n = 0;

    ~Engine() {
        release();
        for (auto& e : kt_ev) {
            (void)hipEventDestroy(e.start);
            (void)hipEventDestroy(e.stop);
        }
    }

    void release() {
        auto fr = [](void* p) {
            if (p) (void)hipFree(p);
        };
        if (own_s) {
            fr(s.x); fr(s.y); fr(s.z);
        }
        fr(alt.x); fr(alt.y); fr(alt.z);
        fr(yA.x); fr(yA.y); fr(yA.z);
        fr(yB.x); fr(yB.y); fr(yB.z);
        fr(acc.x); fr(acc.y); fr(acc.z);
        for (State& k : Kt) {
            fr(k.x); fr(k.y); fr(k.z);
            k = State{};
        }
        fr(dreps); fr(d_blk_rep); fr(d_oblk_rep); fr(d_tiles); fr(d_partials); fr(d_result);
        fr(d_accum); fr(d_kickdev); fr(d_trace); fr(d_obs_stage); fr(d_obs_vals);
        s = alt = yA = yB = acc = State{};
        dreps = nullptr; d_blk_rep = d_oblk_rep = nullptr; d_tiles = nullptr;
        d_partials = d_result = d_accum = d_trace = nullptr; d_kickdev = nullptr;
        d_obs_stage = d_obs_vals = nullptr;
        obs_cap = obs_n = 0;
    }
};

lll_status alloc_state(Engine& E, State& S) {
    if (S.x) return LLL_OK;
    size_t bytes = (size_t)E.nsites * E.esz;
    void* p[3] = {nullptr, nullptr, nullptr};
    for (int c = 0; c < 3; ++c) {
        if (hipMalloc(&p[c], bytes) != hipSuccess) {
            for (int d = 0; d < c; ++d) (void)hipFree(p[d]);
            return set_err(LLL_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
    }
    S.x = p[0]; S.y = p[1]; S.z = p[2];
    return LLL_OK;
}

// Geometry-dependent tables: per-site blocks and observables blocks.
lll_status build_tables(Engine& E) {
    std::vector<int32_t> blk, oblk;
    int64_t off = 0;
    for (int r = 0; r < E.nrep; ++r) {
        RepDev& R = E.hreps[r];
        const int64_t N = (int64_t)R.Lx * R.Ly * R.Lz;
        R.off = off;
        off += N;
        R.sb0 = (int32_t)blk.size();
        R.nsb = (int32_t)((N + 255) / 256);
        for (int b = 0; b < R.nsb; ++b) blk.push_back(r);
        R.ob0 = (int32_t)oblk.size();
        R.nob = (int32_t)std::min<int64_t>(obs_item_count(R.Lx, R.Ly, R.Lz), 2048);
        for (int b = 0; b < R.nob; ++b) oblk.push_back(r);
    }
    E.nsites = off;
    E.nblk = (int)blk.size();
    E.nobblk = (int)oblk.size();
    HIP_TRY(hipMalloc(&E.d_blk_rep, sizeof(int32_t) * blk.size()));
    HIP_TRY(hipMemcpy(E.d_blk_rep, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&E.d_oblk_rep, sizeof(int32_t) * oblk.size()));
    HIP_TRY(hipMemcpy(E.d_oblk_rep, oblk.data(), sizeof(int32_t) * oblk.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&E.d_partials, sizeof(double) * 8 * oblk.size()));
    HIP_TRY(hipMalloc(&E.d_result, sizeof(double) * 8 * E.nrep));
    HIP_TRY(hipMalloc(&E.d_accum, sizeof(double) * 8 * E.nrep));
    HIP_TRY(hipMemset(E.d_accum, 0, sizeof(double) * 8 * E.nrep));
    HIP_TRY(hipMalloc(&E.d_kickdev, sizeof(unsigned long long) * kKickSlots * E.nrep));
    HIP_TRY(hipMemset(E.d_kickdev, 0, sizeof(unsigned long long) * kKickSlots * E.nrep));
    HIP_TRY(hipMalloc(&E.dreps, sizeof(RepDev) * E.nrep));
    return LLL_OK;
}

lll_status upload_reps(Engine& E) {
    HIP_TRY(hipStreamSynchronize(E.st));
    HIP_TRY(hipMemcpy(E.dreps, E.hreps.data(), sizeof(RepDev) * E.nrep, hipMemcpyHostToDevice));
    return LLL_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

struct Phys {
    double J, H[3], D, e[3], lambda, T;
    const void* D_site;
    const void* e_site;
};

// Stage coefficients and physics of one replica (see RepDev).
void fill_physics(RepDev& R, const Phys& p, double dt, double Dt, int precession, uint64_t seed,
                  uint32_t rid) {
    double en = sqrt(p.e[0] * p.e[0] + p.e[1] * p.e[1] + p.e[2] * p.e[2]);
    double e[3] = {0, 0, 1};
    if (en > 0) {
        e[0] = p.e[0] / en; e[1] = p.e[1] / en; e[2] = p.e[2] / en;
    }
    const double f = precession ? dt : -p.lambda * dt;
    R.cJ = f * p.J;
    for (int c = 0; c < 3; ++c) {
        R.cH[c] = f * p.H[c];
        R.e[c] = e[c];
        R.H[c] = p.H[c];
    }
    R.cD = p.D_site ? 2.0 * f : 2.0 * p.D * f;
    R.lam = precession ? p.lambda : 0.0;
    R.J = p.J;
    R.D = p.D;
    R.pad2 = 0;
    R.lambda = p.lambda;
    R.Dt = Dt;
    R.sigma = sqrt(2.0 * p.lambda * p.T * Dt);
    R.seed = seed;
    R.rid = rid;
    R.D_site = p.D_site;
    R.e_site = p.e_site;
}

int anis_mode_of(const Phys& p) {
    if (p.D_site) return ANIS_SITE;
    if (p.D == 0.0) return ANIS_NONE;
    double en = sqrt(p.e[0] * p.e[0] + p.e[1] * p.e[1] + p.e[2] * p.e[2]);
    if (en == 0.0 || (p.e[0] == 0.0 && p.e[1] == 0.0)) return ANIS_Z;
    return ANIS_AXIS;
}

lll_status steps_per_interval(double dt, double Dt, int64_t* n) {
    if (!(dt > 0) || !(Dt > 0) || !is_fin(dt) || !is_fin(Dt))
        return set_err(LLL_EINVAL, "dt and Dt must be positive and finite");
    double q = Dt / dt;
    double r = floor(q + 0.5);
    if (r < 1 || fabs(q - r) > 1e-9 * r)
        return set_err(LLL_EINVAL, "Dt/dt = %.17g is not a positive integer", q);
    *n = (int64_t)r;
    return LLL_OK;
}

lll_status check_phys(const Phys& p) {
    const double v[] = {p.J, p.H[0], p.H[1], p.H[2], p.D, p.e[0], p.e[1], p.e[2], p.lambda, p.T};
    for (double x : v)
        if (!is_fin(x)) return set_err(LLL_EINVAL, "non-finite parameter");
    if (p.lambda < 0) return set_err(LLL_EINVAL, "lambda must be >= 0");
    if (p.T < 0) return set_err(LLL_EINVAL, "T must be >= 0");
    if (p.e_site && !p.D_site) return set_err(LLL_EINVAL, "e_site needs D_site");
    return LLL_OK;
}

// Eq. (8): sqrt(Lambda_N Dt) small; Eq. (9): lambda h Dt small; step-size rule
// of Sec. II: h dt about 0.2-0.25 at most with precession.
bool applicability_warning(const Phys& p, double dt, double Dt, int precession, double Tmax) {
    const double hmax = 6 * fabs(p.J) +
                        sqrt(p.H[0] * p.H[0] + p.H[1] * p.H[1] + p.H[2] * p.H[2]) +
                        2 * fabs(p.D);
    if (2 * p.lambda * Tmax * Dt > 0.2) return true;
    if (p.lambda * hmax * Dt > 0.2) return true;
    if (precession && hmax * dt > 0.25) return true;
    return false;
}

// ----------------------------------------------------- step machinery -----
lll_status ensure_unfused_scratch(Engine& E) {
    lll_status s;
    if ((s = alloc_state(E, E.yA)) != LLL_OK) return s;
    if ((s = alloc_state(E, E.yB)) != LLL_OK) return s;
    if ((s = alloc_state(E, E.acc)) != LLL_OK) return s;
    return LLL_OK;
}

// Tableaus of the integrators of the Appendix: RK2 midpoint, Butcher's
// six-stage fifth-order method and classical RK4.
Tableau tableau_of(int integrator) {
    Tableau tb{};
    if (integrator == LLL_RK2MID) {
        tb.stages = 2;
        tb.a[1][0] = 0.5;
        tb.b[1] = 1.0;
    } else if (integrator == LLL_RK5B) {
        tb.stages = 6;
        tb.a[1][0] = 0.25;
        tb.a[2][0] = 0.125;
        tb.a[2][1] = 0.125;
        tb.a[3][1] = -0.5;
        tb.a[3][2] = 1.0;
        tb.a[4][0] = 3.0 / 16.0;
        tb.a[4][3] = 9.0 / 16.0;
        tb.a[5][0] = -3.0 / 7.0;
        tb.a[5][1] = 2.0 / 7.0;
        tb.a[5][2] = 12.0 / 7.0;
        tb.a[5][3] = -12.0 / 7.0;
        tb.a[5][4] = 8.0 / 7.0;
        tb.b[0] = 7.0 / 90.0;
        tb.b[2] = 32.0 / 90.0;
        tb.b[3] = 12.0 / 90.0;
        tb.b[4] = 32.0 / 90.0;
        tb.b[5] = 7.0 / 90.0;
    } else if (integrator == LLL_RK4) {  // used by the escape runs (lattices have fused RK4)
        tb.stages = 4;
        tb.a[1][0] = 0.5;
        tb.a[2][1] = 0.5;
        tb.a[3][2] = 1.0;
        tb.b[0] = 1.0 / 6.0;
        tb.b[1] = 1.0 / 3.0;
        tb.b[2] = 1.0 / 3.0;
        tb.b[3] = 1.0 / 6.0;
    }
    return tb;
}

lll_status ensure_tableau_scratch(Engine& E, int stages, KSet& ks) {
    lll_status s;
    if ((s = alloc_state(E, E.yA)) != LLL_OK) return s;
    if ((s = alloc_state(E, E.yB)) != LLL_OK) return s;
    ks = KSet{};
    for (int j = 0; j + 1 < stages; ++j) {
        if ((s = alloc_state(E, E.Kt[j])) != LLL_OK) return s;
        ks.K[j] = E.Kt[j];
    }
    return LLL_OK;
}

// z-chunk of the fused kernel: the configured one, else 16 planes (fp32) or
// 32 planes (fp64, whose tiles are smaller in x and y).
int eff_bz(const Engine& E) { return E.bz > 0 ? E.bz : (E.prec == 0 ? 32 : 16); }

// Tile list of the fused kernel: (replica, tile x, tile y, tile z) per
// workgroup, ordered so that the eight XCDs (workgroups are dealt out to them
// round-robin) each receive a contiguous z-major range of tiles, keeping halo
// re-reads inside one XCD's L2; a batch of replicas is first ordered by
// balance_tiles (tile_order.hpp).
lll_status ensure_tiles(Engine& E) {
    if (E.tiles_variant == E.variant && E.tiles_bz == E.bz && E.d_tiles) return LLL_OK;
    FusedInfo fi;
    if (!fused_variant_info(E.prec, E.variant, &fi))
        return set_err(LLL_EINVAL, "invalid step variant %d", E.variant);
    std::vector<int4> list;
    std::vector<int> bz_of(E.nrep);
    const int bz_eff = eff_bz(E);
    for (int r = 0; r < E.nrep; ++r) {
        RepDev& R = E.hreps[r];
        int bzr = bz_eff;
        if (bzr > R.Lz) bzr = R.Lz;
        bz_of[r] = bzr;
        R.tx = (R.Lx + fi.bx - 1) / fi.bx;
        R.ty = (R.Ly + fi.by - 1) / fi.by;
        R.tz = (R.Lz + bzr - 1) / bzr;
        R.tile0 = (int32_t)list.size();
        for (int tz = 0; tz < R.tz; ++tz)
            for (int ty = 0; ty < R.ty; ++ty)
                for (int tx = 0; tx < R.tx; ++tx) list.push_back(make_int4(r, tx, ty, tz));
    }
    if (E.nrep > 1) {
        std::vector<int> lz(E.nrep);
        for (int r = 0; r < E.nrep; ++r) lz[r] = E.hreps[r].Lz;
        list = tileord::balance_tiles(list, lz, bz_of);
    }
    // XCD-aware order: workgroup w runs on XCD w % 8.
    const int n = (int)list.size();
    std::vector<int4> ord(n);
    const std::vector<int> slot_of = tileord::xcd_slots(n);
    for (int p = 0; p < n; ++p) ord[slot_of[p]] = list[p];
    if (n > E.tiles_cap) {
        if (E.d_tiles) (void)hipFree(E.d_tiles);
        E.d_tiles = nullptr;
        HIP_TRY(hipMalloc(&E.d_tiles, sizeof(int4) * n));
        E.tiles_cap = n;
    }
    HIP_TRY(hipStreamSynchronize(E.st));
    HIP_TRY(hipMemcpy(E.d_tiles, ord.data(), sizeof(int4) * n, hipMemcpyHostToDevice));
    E.ntiles = n;
    E.tiles_variant = E.variant;
    E.tiles_bz = E.bz;
    lll_status st = upload_reps(E);
    return st;
}

State cur_state(Engine& E) { return E.cur ? E.alt : E.s; }

// n RK4 steps; when kick_last, kick k is applied right after the last step
// (as the fused kernel's epilogue, or as a separate launch).
void kt_harvest(Engine& E, size_t j) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, E.kt_ev[j].start, E.kt_ev[j].stop) == hipSuccess) {
        E.kt_ms += ms;
        E.kt_n += 1;
    }
    E.kt_busy[j] = 0;
}

// Every kKtStride-th fused launch of a measurement is timed: a launch that
// records events at its own dispatch starts a few microseconds later (about
// 6% of a 20-interval headline run when every launch was timed).
constexpr uint64_t kKtStride = 16;

const LaunchEvents* kt_take(Engine& E) {
    if (!E.kt_on || E.kt_ev.empty()) return nullptr;
    if (E.kt_seq++ % kKtStride != 0) return nullptr;
    const size_t j = E.kt_next++ % E.kt_ev.size();
    if (E.kt_busy[j]) {
        if (hipEventQuery(E.kt_ev[j].stop) != hipSuccess) return nullptr;
        kt_harvest(E, j);
    }
    E.kt_busy[j] = 1;
    return &E.kt_ev[j];
}

lll_status do_steps(Engine& E, int64_t n, bool kick_last, uint64_t k, double sigma_override) {
    if (n <= 0) return LLL_OK;
    const bool fused_ok = E.variant != 0;
    if (E.integrator == LLL_RK5B && fused_ok) {
        // two launches per step (stages 1-4, stages 5-6) through three scratch
        // states; the kick rides on the last step's second launch
        lll_status s = alloc_state(E, E.alt);
        for (int j = 0; j < 3 && s == LLL_OK; ++j) s = alloc_state(E, E.Kt[j]);
        if (s != LLL_OK) return s;
        if ((s = ensure_tiles(E)) != LLL_OK) return s;
        for (int64_t q = 0; q < n; ++q) {
            const bool kk = kick_last && q + 1 == n && E.kick_epilogue;
            State in = cur_state(E);
            State out = E.cur ? E.s : E.alt;
            HIP_TRY(launch_step_rk5_fused(E.prec, E.precession, E.anis, E.variant, eff_bz(E),
                                          E.dreps, E.d_tiles, E.ntiles, in, out, E.Kt, kk ? 1 : 0, k,
                                          sigma_override, E.d_kickdev, E.st));
            E.cur ^= 1;
        }
        if (kick_last && !E.kick_epilogue)
            HIP_TRY(launch_kick(E.prec, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), k,
                                sigma_override, E.d_kickdev, E.st));
        return LLL_OK;
    }
    if (E.integrator == LLL_RK5B || (E.integrator == LLL_RK2MID && !fused_ok)) {
        const Tableau tb = tableau_of(E.integrator);
        KSet ks;
        lll_status s = ensure_tableau_scratch(E, tb.stages, ks);
        if (s != LLL_OK) return s;
        for (int64_t q = 0; q < n; ++q)
            HIP_TRY(launch_step_tableau(E.prec, E.precession, E.anis, E.dreps, E.d_blk_rep, E.nblk,
                                        tb, cur_state(E), E.yA, E.yB, ks, E.st));
        if (kick_last)
            HIP_TRY(launch_kick(E.prec, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), k,
                                sigma_override, E.d_kickdev, E.st));
        return LLL_OK;
    }
    if (!fused_ok) {
        lll_status s = ensure_unfused_scratch(E);
        if (s != LLL_OK) return s;
        for (int64_t q = 0; q < n; ++q)
            HIP_TRY(launch_step_unfused(E.prec, E.precession, E.anis, E.dreps, E.d_blk_rep, E.nblk,
                                        cur_state(E), E.yA, E.yB, E.acc, E.st));
        if (kick_last)
            HIP_TRY(launch_kick(E.prec, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), k,
                                sigma_override, E.d_kickdev, E.st));
        return LLL_OK;
    }
    lll_status s = alloc_state(E, E.alt);
    if (s != LLL_OK) return s;
    if ((s = ensure_tiles(E)) != LLL_OK) return s;
    // RK4: one step per launch.  RK2 midpoint: two steps per launch, and one
    // single-step launch when the count is odd.
    for (int64_t q = 0; q < n;) {
        int scheme = 0, adv = 1;
        if (E.integrator == LLL_RK2MID) {
            scheme = n - q >= 2 ? 1 : 2;
            adv = n - q >= 2 ? 2 : 1;
        }
        const bool kk = kick_last && q + adv == n && E.kick_epilogue;
        State in = cur_state(E);
        State out = E.cur ? E.s : E.alt;
        HIP_TRY(launch_step_fused(E.prec, E.precession, E.anis, E.variant, eff_bz(E), scheme,
                                  E.dreps, E.d_tiles, E.ntiles, in, out, kk ? 1 : 0, k,
                                  sigma_override, E.d_kickdev, kk ? nullptr : kt_take(E), E.st));
        E.cur ^= 1;
        q += adv;
    }
    if (kick_last && !E.kick_epilogue)
        HIP_TRY(launch_kick(E.prec, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), k, sigma_override,
                            E.d_kickdev, E.st));
    return LLL_OK;
}

lll_status do_kick(Engine& E, uint64_t k, double sigma_override) {
    HIP_TRY(launch_kick(E.prec, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), k, sigma_override,
                        E.d_kickdev, E.st));
    return LLL_OK;
}

lll_status settle(Engine& E) {
    if (E.cur) {
        HIP_TRY(launch_copy(E.prec, E.s, E.alt, E.nsites, E.st));
        E.cur = 0;
    }
    return LLL_OK;
}

// One interval of Eq. (7): n1 steps, kick, n2 steps.
// look: the caller runs interval k_next (kick scale so_next) right after this
// one with no measurement in between; when that interval starts with its kick
// (n1 = 0), the kick is done here, as the epilogue of this interval's last step
// where the fused step is used (the same state at the same point of the
// schedule, so the same bits).
lll_status do_interval(Engine& E, int64_t n, uint64_t k, double sigma_override, bool look,
                       uint64_t k_next, double so_next) {
    const int64_t n1 = n / 2, n2 = n - n1;
    lll_status s;
    if (n1 > 0) {
        E.carried = false;
        if ((s = do_steps(E, n1, true, k, sigma_override)) != LLL_OK) return s;
    } else if (E.carried && E.carried_k == k) {
        E.carried = false;  // applied at the end of the previous interval
    } else {
        E.carried = false;
        if ((s = do_kick(E, k, sigma_override)) != LLL_OK) return s;
    }
    const bool carry = look && n1 == 0;
    if ((s = do_steps(E, n2, carry, k_next, so_next)) != LLL_OK) return s;
    if (carry) {
        E.carried = true;
        E.carried_k = k_next;
    }
    return LLL_OK;
}

lll_status do_interval(Engine& E, int64_t n, uint64_t k, double sigma_override) {
    E.carried = false;
    return do_interval(E, n, k, sigma_override, false, 0, -1.0);
}

// Observables into result (and the running sums when accumulate).
lll_status do_obs(Engine& E, double* result, int accumulate) {
    HIP_TRY(launch_obs(E.prec, E.anis, E.dreps, E.d_oblk_rep, E.nobblk, E.nrep, cur_state(E),
                       E.d_partials, result, E.d_accum, accumulate, E.st));
    return LLL_OK;
}

lll_status ensure_trace(Engine& E, size_t doubles) {
    if (doubles <= E.trace_cap) return LLL_OK;
    if (E.d_trace) (void)hipFree(E.d_trace);
    E.d_trace = nullptr;
    E.trace_cap = 0;
    HIP_TRY(hipMalloc(&E.d_trace, sizeof(double) * doubles));
    E.trace_cap = doubles;
    return LLL_OK;
}

// Staging buffers for the measurements of a run: up to 1024 measurements, and
// at most 32 MiB for the partials and for the values each.  Allocated once
// (a captured batch schedule keeps their addresses).
lll_status ensure_obs_stage(Engine& E) {
    if (E.d_obs_stage) return LLL_OK;
    const int64_t lim = (int64_t)32 << 20;
    const int64_t per_part = std::max<int64_t>(1, (int64_t)E.nobblk) * 8 * (int64_t)sizeof(double);
    const int64_t per_val = std::max<int64_t>(1, (int64_t)E.nrep) * 8 * (int64_t)sizeof(double);
    const int64_t cap = std::max<int64_t>(
        1, std::min<int64_t>(1024, std::min(lim / per_part, lim / per_val)));
    HIP_TRY(hipMalloc(&E.d_obs_stage, per_part * cap));
    HIP_TRY(hipMalloc(&E.d_obs_vals, per_val * cap));
    E.obs_cap = (int)cap;
    E.obs_n = 0;
    return LLL_OK;
}

// Starts staging: reduced measurements go to out, out + stride, ... (doubles;
// measurement of replica r at + 8 r), or, with out null, only the last one to
// d_result.
void obs_begin(Engine& E, double* out, int64_t stride) {
    E.obs_n = 0;
    E.obs_out = out;
    E.obs_stride = stride;
}

// Reduces the staged measurements, adds them to the running sums in order and
// leaves the last one in d_result.
lll_status obs_fold(Engine& E) {
    if (E.obs_n == 0) return LLL_OK;
    double* out = E.obs_out ? E.obs_out : E.d_obs_vals;
    const int64_t stride = E.obs_out ? E.obs_stride : (int64_t)8 * E.nrep;
    HIP_TRY(launch_obs_staged(E.anis, E.dreps, E.nrep, E.nobblk, E.obs_n, E.d_obs_stage, out,
                              stride, E.d_accum, E.d_result, E.st));
    if (E.obs_out) E.obs_out += (int64_t)E.obs_n * E.obs_stride;
    E.obs_n = 0;
    return LLL_OK;
}

// One measurement of the current state, staged.
lll_status obs_stage(Engine& E) {
    HIP_TRY(launch_obs_partials(E.prec, E.anis, E.dreps, E.d_oblk_rep, E.nobblk, cur_state(E),
                                E.d_obs_stage + (size_t)E.obs_n * E.nobblk * 8, E.st));
    if (++E.obs_n == E.obs_cap) return obs_fold(E);
    return LLL_OK;
}

void obs_from(const double* r, lll_obs* o) {
    o->E_total = r[0];
    o->E_exch = r[1];
    o->E_zeeman = r[2];
    o->E_anis = r[3];
    o->m[0] = r[4];
    o->m[1] = r[5];
    o->m[2] = r[6];
    o->max_norm_dev = r[7];
}

bool obs_finite(const double* r) {
    for (int j = 0; j < 8; ++j)
        if (!std::isfinite(r[j])) return false;
    return true;
}

// Largest | |s_i| - 1 | of n measured records (slot 7); NaN records are reported
// by obs_finite instead.
double max_norm_dev_of(const double* h, int64_t n) {
    double m = 0.0;
    for (int64_t j = 0; j < n; ++j)
        if (h[8 * j + 7] > m) m = h[8 * j + 7];
    return m;
}

lll_status norm_warning(double dev) {
    return set_err(LLL_WARN_NORM,
                   "spin length drifted: max | |s_i| - 1 | = %.3g exceeds %.2g (delta t too large "
                   "for the local fields)", dev, (double)LLL_NORM_WARN_LEVEL);
}

}  // namespace

// ------------------------------------------------------------- lattice ----
struct lll_tape;

struct lll_lattice {
    Engine E;
    int32_t Lx, Ly, Lz, bc;
    bool have_params = false;
    Phys phys{};
    double dt = 0, Dt = 0;
    int precession = 1;
    uint64_t seed = 0;
    uint32_t replica = 0;
    // adjoint: live tapes, a checkpoint buffer handed back by a destroyed
    // tape, and the backward pass's work buffers (grow-only, reused)
    std::vector<lll_tape*> tapes;
    void* ck_pool = nullptr;
    size_t ck_pool_bytes = 0;
    void* adj_bb = nullptr;
    size_t adj_bb_bytes = 0;
    void* adj_sc = nullptr;
    size_t adj_sc_bytes = 0;
    void* adj_small = nullptr;
    size_t adj_small_bytes = 0;
    // the backward pass recomputes the next checkpoint block on a second
    // stream while the current block is reversed: events 0 (work before the
    // backward), 1-2 (block buffer k recomputed), 3-4 (block buffer k reversed)
    hipStream_t adj_st2 = nullptr;
    hipEvent_t adj_ev[5] = {};
    ~lll_lattice();
};

static lll_status lattice_params(lll_lattice* L, const lll_params* p, bool need_schedule) {
    if (!p) return set_err(LLL_EINVAL, "params is NULL");
    Phys ph{};
    ph.J = p->J;
    for (int c = 0; c < 3; ++c) {
        ph.H[c] = p->H[c];
        ph.e[c] = p->e[c];
    }
    ph.D = p->D;
    ph.lambda = p->lambda;
    ph.T = p->T;
    ph.D_site = p->D_site;
    ph.e_site = p->e_site;
    lll_status s = check_phys(ph);
    if (s != LLL_OK) return s;
    if (p->integrator != LLL_RK4 && p->integrator != LLL_RK2MID && p->integrator != LLL_RK5B)
        return set_err(LLL_EINVAL, "unknown integrator %d", (int)p->integrator);
    if (!(p->dt > 0) || !is_fin(p->dt)) return set_err(LLL_EINVAL, "dt must be positive");
    double Dt = p->Dt;
    if (need_schedule) {
        int64_t n;
        if ((s = steps_per_interval(p->dt, p->Dt, &n)) != LLL_OK) return s;
    } else if (!(Dt > 0) || !is_fin(Dt)) {
        Dt = p->dt;
    }
    if (p->D_site && !p->e_site) return set_err(LLL_EINVAL, "D_site needs e_site");
    const int prec = p->precession ? 1 : 0;
    const bool same = L->have_params && memcmp(&ph, &L->phys, sizeof ph) == 0 && L->dt == p->dt &&
                      L->Dt == Dt && L->precession == prec && L->seed == p->seed &&
                      L->replica == p->replica && L->E.integrator == p->integrator;
    if (same) return LLL_OK;
    Engine& E = L->E;
    RepDev& R = E.hreps[0];
    fill_physics(R, ph, p->dt, Dt, prec, p->seed, p->replica);
    E.precession = prec;
    E.anis = anis_mode_of(ph);
    E.integrator = p->integrator;
    if ((s = upload_reps(E)) != LLL_OK) return s;
    L->phys = ph;
    L->dt = p->dt;
    L->Dt = Dt;
    L->precession = prec;
    L->seed = p->seed;
    L->replica = p->replica;
    L->have_params = true;
    return LLL_OK;
}

// Sites of an Lx x Ly x Lz lattice (sizes >= 1), or -1 beyond 2^31 - 1; the
// product is formed in two checked steps so that it cannot overflow.
static int64_t checked_sites(int32_t Lx, int32_t Ly, int32_t Lz) {
    const int64_t xy = (int64_t)Lx * Ly;  // < 2^62
    if (xy > 0x7FFFFFFFLL) return -1;
    const int64_t n = xy * Lz;            // < 2^62
    return n > 0x7FFFFFFFLL ? -1 : n;
}

// Parameter checks and the descriptor of a lone lattice for the
// allocation-free observables (lll_noalloc.hip).
lll_status noalloc_error(lll_status s, const char* msg, int code) {
    return code ? set_err(s, "%s (%d)", msg, code) : set_err(s, "%s", msg);
}

lll_status noalloc_describe(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc, const lll_params* p,
                            RepDev* R, int* anis) {
    if (!p) return set_err(LLL_EINVAL, "params is NULL");
    if (Lx < 1 || Ly < 1 || Lz < 1) return set_err(LLL_EINVAL, "lattice sizes must be >= 1");
    if (checked_sites(Lx, Ly, Lz) < 0) return set_err(LLL_EINVAL, "at most 2^31-1 sites");
    if (bc != LLL_BC_PERIODIC && bc != LLL_BC_FREE) return set_err(LLL_EINVAL, "bad boundary");
    Phys ph{};
    ph.J = p->J;
    for (int c = 0; c < 3; ++c) {
        ph.H[c] = p->H[c];
        ph.e[c] = p->e[c];
    }
    ph.D = p->D;
    ph.lambda = p->lambda;
    ph.T = p->T;
    ph.D_site = p->D_site;
    ph.e_site = p->e_site;
    lll_status s = check_phys(ph);
    if (s != LLL_OK) return s;
    if (p->D_site && !p->e_site) return set_err(LLL_EINVAL, "D_site needs e_site");
    memset(R, 0, sizeof *R);
    R->Lx = Lx;
    R->Ly = Ly;
    R->Lz = Lz;
    R->bc = bc;
    const double dt = (p->dt > 0 && is_fin(p->dt)) ? p->dt : 1.0;
    const double Dt = (p->Dt > 0 && is_fin(p->Dt)) ? p->Dt : dt;
    fill_physics(*R, ph, dt, Dt, p->precession ? 1 : 0, p->seed, p->replica);
    *anis = anis_mode_of(ph);
    return LLL_OK;
}

extern "C" lll_status lll_init_lattice(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc,
                                       lll_precision prec, lll_init mode, const double dir[3],
                                       uint64_t seed, void* sx, void* sy, void* sz,
                                       void* hip_stream, lll_lattice** out) {
    if (!out) return set_err(LLL_EINVAL, "out is NULL");
    *out = nullptr;
    if (Lx < 1 || Ly < 1 || Lz < 1) return set_err(LLL_EINVAL, "lattice sizes must be >= 1");
    const int64_t N = checked_sites(Lx, Ly, Lz);
    if (N < 0) return set_err(LLL_EINVAL, "at most 2^31-1 sites");
    if (bc != LLL_BC_PERIODIC && bc != LLL_BC_FREE) return set_err(LLL_EINVAL, "bad boundary");
    if (prec != LLL_FP64 && prec != LLL_FP32) return set_err(LLL_EINVAL, "bad precision");
    if (mode != LLL_INIT_RANDOM_SPHERE && mode != LLL_INIT_DIRECTION && mode != LLL_INIT_KEEP)
        return set_err(LLL_EINVAL, "bad init mode");
    const int nbuf = (sx != nullptr) + (sy != nullptr) + (sz != nullptr);
    if (nbuf != 0 && nbuf != 3) return set_err(LLL_EINVAL, "pass all three buffers or none");
    if (mode == LLL_INIT_KEEP && nbuf == 0)
        return set_err(LLL_EINVAL, "LLL_INIT_KEEP needs caller buffers");
    double d[3] = {0, 0, 1};
    if (mode == LLL_INIT_DIRECTION) {
        if (!dir) return set_err(LLL_EINVAL, "dir is NULL");
        double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        if (!(n > 0) || !is_fin(n)) return set_err(LLL_EINVAL, "dir must be a non-zero vector");
        d[0] = dir[0] / n; d[1] = dir[1] / n; d[2] = dir[2] / n;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_err(LLL_EDEVICE, "no HIP device");
    lll_lattice* L = new lll_lattice();
    L->Lx = Lx; L->Ly = Ly; L->Lz = Lz; L->bc = bc;
    Engine& E = L->E;
    E.prec = prec == LLL_FP64 ? 0 : 1;
    E.esz = E.prec == 0 ? 8 : 4;
    E.st = (hipStream_t)hip_stream;
    E.nrep = 1;
    E.hreps.assign(1, RepDev{});
    RepDev& R = E.hreps[0];
    memset(&R, 0, sizeof R);
    R.Lx = Lx; R.Ly = Ly; R.Lz = Lz; R.bc = bc;
    R.seed = seed;
    R.init = mode == LLL_INIT_RANDOM_SPHERE ? 0 : 1;
    lll_status s = build_tables(E);
    if (s != LLL_OK) { delete L; return s; }
    if (nbuf == 3) {
        E.s.x = sx; E.s.y = sy; E.s.z = sz;
        E.own_s = false;
    } else {
        E.own_s = true;
        if ((s = alloc_state(E, E.s)) != LLL_OK) { delete L; return s; }
    }
    if ((s = upload_reps(E)) != LLL_OK) { delete L; return s; }
    if (mode != LLL_INIT_KEEP) {
        hipError_t e = launch_init(E.prec, E.dreps, E.d_blk_rep, E.nblk, E.s, mode, d[0], d[1], d[2], E.st);
        if (e != hipSuccess) {
            delete L;
            return set_err(LLL_EDEVICE, "init launch failed: %s", hipGetErrorString(e));
        }
    }
    // default step configuration: fused when the lattice is large enough
    E.variant = 0;
    E.bz = 0;
    if (fused_variant_count(E.prec) > 0 && N >= 4096) E.variant = 1;
    *out = L;
    return LLL_OK;
}

extern "C" void lll_destroy(lll_lattice* L) {
    if (!L) return;
    if (L->E.st) (void)hipStreamSynchronize(L->E.st);
    else (void)hipDeviceSynchronize();
    delete L;
}

extern "C" lll_status lll_step_conservative(lll_lattice* L, const lll_params* p, int64_t n_steps) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    if (n_steps < 0) return set_err(LLL_EINVAL, "n_steps < 0");
    lll_status s = lattice_params(L, p, false);
    if (s != LLL_OK) return s;
    if ((s = do_steps(L->E, n_steps, false, 0, -1.0)) != LLL_OK) return s;
    return settle(L->E);
}

extern "C" lll_status lll_noise_pulse(lll_lattice* L, const lll_params* p, uint64_t pulse_index) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    lll_status s = lattice_params(L, p, true);
    if (s != LLL_OK) return s;
    if ((s = settle(L->E)) != LLL_OK) return s;
    return do_kick(L->E, pulse_index, -1.0);
}

extern "C" lll_status lll_observables(lll_lattice* L, const lll_params* p, lll_obs* out) {
    if (!L || !out) return set_err(LLL_EINVAL, "NULL argument");
    lll_status s = lattice_params(L, p, false);
    if (s != LLL_OK) return s;
    Engine& E = L->E;
    if ((s = settle(E)) != LLL_OK) return s;
    if ((s = do_obs(E, E.d_result, 0)) != LLL_OK) return s;
    double r[8];
    HIP_TRY(hipMemcpyAsync(r, E.d_result, sizeof r, hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipStreamSynchronize(E.st));
    obs_from(r, out);
    if (!obs_finite(r)) return set_err(LLL_ENONFINITE, "state contains NaN or Inf");
    if (r[7] > LLL_NORM_WARN_LEVEL) return norm_warning(r[7]);
    return LLL_OK;
}

extern "C" lll_status lll_run(lll_lattice* L, const lll_params* p, uint64_t first_pulse,
                              int64_t n_pulses, const double* T_per_pulse, int32_t obs_every,
                              lll_obs* trace) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    if (n_pulses < 0) return set_err(LLL_EINVAL, "n_pulses < 0");
    if (obs_every < 0) return set_err(LLL_EINVAL, "obs_every < 0");
    lll_status s = lattice_params(L, p, true);
    if (s != LLL_OK) return s;
    Engine& E = L->E;
    int64_t n;
    if ((s = steps_per_interval(p->dt, p->Dt, &n)) != LLL_OK) return s;
    double Tmax = p->T;
    if (T_per_pulse) {
        Tmax = 0;
        for (int64_t q = 0; q < n_pulses; ++q) {
            if (!(T_per_pulse[q] >= 0) || !is_fin(T_per_pulse[q]))
                return set_err(LLL_EINVAL, "T_per_pulse[%lld] invalid", (long long)q);
            Tmax = std::max(Tmax, T_per_pulse[q]);
        }
    }
    const int64_t nmeas = obs_every > 0 ? n_pulses / obs_every : 0;
    const bool want_trace = trace && nmeas > 0;
    if (want_trace && (s = ensure_trace(E, (size_t)nmeas * 8)) != LLL_OK) return s;
    if (nmeas > 0 && (s = ensure_obs_stage(E)) != LLL_OK) return s;
    if ((s = settle(E)) != LLL_OK) return s;
    obs_begin(E, want_trace ? E.d_trace : nullptr, 8);
    E.carried = false;
    for (int64_t q = 0; q < n_pulses; ++q) {
        const uint64_t k = first_pulse + (uint64_t)q;
        const double so = T_per_pulse ? sqrt(2.0 * p->lambda * T_per_pulse[q] * L->Dt) : -1.0;
        const bool measure = obs_every > 0 && (q + 1) % obs_every == 0;
        const bool look = q + 1 < n_pulses && !measure;
        const double so_next =
            look && T_per_pulse ? sqrt(2.0 * p->lambda * T_per_pulse[q + 1] * L->Dt) : -1.0;
        if ((s = do_interval(E, n, k, so, look, k + 1, so_next)) != LLL_OK) return s;
        if (measure && (s = obs_stage(E)) != LLL_OK) return s;
    }
    if ((s = obs_fold(E)) != LLL_OK) return s;
    if ((s = settle(E)) != LLL_OK) return s;
    if (want_trace) {
        std::vector<double> h((size_t)nmeas * 8);
        HIP_TRY(hipMemcpyAsync(h.data(), E.d_trace, sizeof(double) * h.size(),
                               hipMemcpyDeviceToHost, E.st));
        HIP_TRY(hipStreamSynchronize(E.st));
        bool fin = true;
        for (int64_t j = 0; j < nmeas; ++j) {
            obs_from(&h[8 * j], &trace[j]);
            fin = fin && obs_finite(&h[8 * j]);
        }
        if (!fin) return set_err(LLL_ENONFINITE, "state became NaN or Inf during the run");
        const double dev = max_norm_dev_of(h.data(), nmeas);
        if (dev > LLL_NORM_WARN_LEVEL) return norm_warning(dev);
    }
    if (applicability_warning(L->phys, p->dt, p->Dt, L->precession, Tmax))
        return set_err(LLL_WARN_APPLICABILITY,
                       "applicability: 2 lambda T Dt, lambda h Dt or h dt exceeds its bound");
    return LLL_OK;
}

extern "C" lll_status lll_get_state(lll_lattice* L, void** sx, void** sy, void** sz) {
    if (!L || !sx || !sy || !sz) return set_err(LLL_EINVAL, "NULL argument");
    *sx = L->E.s.x;
    *sy = L->E.s.y;
    *sz = L->E.s.z;
    return LLL_OK;
}

extern "C" lll_status lll_kick_norm_dev(lll_lattice* L, double* out, int32_t reset) {
    if (!L || !out) return set_err(LLL_EINVAL, "NULL argument");
    // the running maximum is the largest slot (bit patterns of doubles >= 0)
    unsigned long long slots[kKickSlots];
    HIP_TRY(hipMemcpyAsync(slots, L->E.d_kickdev, sizeof slots, hipMemcpyDeviceToHost, L->E.st));
    HIP_TRY(hipStreamSynchronize(L->E.st));
    unsigned long long v = 0;
    for (unsigned long long x : slots) v = std::max(v, x);
    memcpy(out, &v, sizeof v);
    if (reset) {
        HIP_TRY(hipMemsetAsync(L->E.d_kickdev, 0, sizeof slots, L->E.st));
        HIP_TRY(hipStreamSynchronize(L->E.st));
    }
    return LLL_OK;
}

extern "C" lll_status lll_accumulators(lll_lattice* L, double* out, int32_t reset) {
    if (!L || !out) return set_err(LLL_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(out, L->E.d_accum, sizeof(double) * 8, hipMemcpyDeviceToHost, L->E.st));
    HIP_TRY(hipStreamSynchronize(L->E.st));
    if (reset) {
        HIP_TRY(hipMemsetAsync(L->E.d_accum, 0, sizeof(double) * 8, L->E.st));
        HIP_TRY(hipStreamSynchronize(L->E.st));
    }
    return LLL_OK;
}

extern "C" lll_status lll_step_variant_info(lll_precision prec, int32_t variant, int32_t* out4) {
    if (!out4) return set_err(LLL_EINVAL, "NULL argument");
    const int pr = prec == LLL_FP64 ? 0 : 1;
    if (variant == 0) {
        out4[0] = 1; out4[1] = 1; out4[2] = 256; out4[3] = 0;
        return LLL_OK;
    }
    FusedInfo fi;
    if (!fused_variant_info(pr, variant, &fi)) return set_err(LLL_EINVAL, "no such variant");
    out4[0] = fi.bx; out4[1] = fi.by; out4[2] = fi.threads; out4[3] = fi.lds_bytes;
    return LLL_OK;
}

extern "C" lll_status lll_set_step_config(lll_lattice* L, int32_t variant, int32_t bz) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    if (variant < 0 || variant > fused_variant_count(L->E.prec))
        return set_err(LLL_EINVAL, "variant %d out of range", variant);
    if (bz < 0) return set_err(LLL_EINVAL, "bz < 0");
    lll_status s = settle(L->E);
    if (s != LLL_OK) return s;
    L->E.variant = variant;
    L->E.bz = bz;
    return LLL_OK;
}

extern "C" lll_status lll_set_kick_fusion(lll_lattice* L, int32_t fused) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    lll_status s = settle(L->E);
    if (s != LLL_OK) return s;
    L->E.kick_epilogue = fused != 0;
    return LLL_OK;
}

extern "C" lll_status lll_kernel_timing(lll_lattice* L, int32_t enable, double* avg_ms,
                                        int64_t* n_timed) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    Engine& E = L->E;
    if (enable) {
        if (E.kt_ev.empty()) {
            E.kt_ev.resize(64);
            E.kt_busy.assign(64, 0);
            // timestamps only: no system-scope fence (cache writeback and
            // invalidation) when the events complete, which would otherwise
            // lengthen the timed launch and delay the next one
            for (auto& e : E.kt_ev) {
                e.start = e.stop = nullptr;
                HIP_TRY(hipEventCreateWithFlags(&e.start, hipEventDisableSystemFence));
                HIP_TRY(hipEventCreateWithFlags(&e.stop, hipEventDisableSystemFence));
            }
        }
        for (size_t j = 0; j < E.kt_ev.size(); ++j) E.kt_busy[j] = 0;
        E.kt_ms = 0;
        E.kt_n = 0;
        E.kt_next = 0;
        E.kt_seq = 0;
        E.kt_on = true;
        return LLL_OK;
    }
    HIP_TRY(hipStreamSynchronize(E.st));
    for (size_t j = 0; j < E.kt_ev.size(); ++j)
        if (E.kt_busy[j]) kt_harvest(E, j);
    E.kt_on = false;
    if (avg_ms) *avg_ms = E.kt_n > 0 ? E.kt_ms / (double)E.kt_n : 0.0;
    if (n_timed) *n_timed = E.kt_n;
    return LLL_OK;
}

extern "C" lll_status lll_get_step_config(lll_lattice* L, int32_t* variant, int32_t* bz) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    if (variant) *variant = L->E.variant;
    if (bz) *bz = L->E.bz;
    return LLL_OK;
}

extern "C" lll_status lll_philox4x32_10(uint64_t seed, uint32_t i0, int64_t n, uint32_t c1,
                                        uint32_t c2, uint32_t c3, uint32_t* out_dev,
                                        void* hip_stream) {
    if (n < 0) return set_err(LLL_EINVAL, "n < 0");
    if (n > 0 && !out_dev) return set_err(LLL_EINVAL, "out_dev is NULL");
    HIP_TRY(launch_philox_words(seed, i0, n, c1, c2, c3, out_dev, (hipStream_t)hip_stream));
    return LLL_OK;
}

// ------------------------------------------------------------- autotune ---
// Times every step configuration (unfused, and each fused tile shape with
// z-chunks of 4..64 planes) on the engine's own state and keeps the fastest,
// then times whole noise intervals with the kick as the fused step's epilogue
// and as a launch of its own (both give identical results).  The state and the
// kick-deviation maxima are restored afterwards.  The optional cache file holds
// "key variant bz kick_fused" lines; a cached key is used without timing.
namespace {
lll_status engine_autotune(Engine& E, const std::string& key, int maxLz, int64_t n_interval,
                           const char* cache_path, int32_t* chosen_variant, int32_t* chosen_bz) {
    lll_status s;
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            char line[320], k[200];
            int v, b, kf;
            bool found = false;
            while (fgets(line, sizeof line, f)) {
                const int got = sscanf(line, "%199s %d %d %d", k, &v, &b, &kf);
                if (got >= 3 && key == k && v >= 0 && v <= fused_variant_count(E.prec) && b >= 0) {
                    E.variant = v;
                    E.bz = b;
                    E.kick_epilogue = got < 4 || kf != 0;
                    found = true;
                }
            }
            fclose(f);
            if (found) {
                if (chosen_variant) *chosen_variant = E.variant;
                if (chosen_bz) *chosen_bz = E.bz;
                return LLL_OK;
            }
        }
    }
    if ((s = settle(E)) != LLL_OK) return s;
    State save{};
    if ((s = alloc_state(E, save)) != LLL_OK) return s;
    HIP_TRY(launch_copy(E.prec, save, E.s, E.nsites, E.st));
    std::vector<unsigned long long> kd_save((size_t)kKickSlots * E.nrep);
    HIP_TRY(hipMemcpyAsync(kd_save.data(), E.d_kickdev, sizeof(unsigned long long) * kd_save.size(),
                           hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipStreamSynchronize(E.st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<std::pair<int, int>> cands;
    cands.push_back({0, 0});
    {
        for (int v = 1; v <= fused_variant_count(E.prec); ++v) {
            const int bzs[] = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 512, 1024};
            for (int b : bzs)
                if (b <= std::max(maxLz, 4)) cands.push_back({v, b});
        }
    }
    double best = 1e30;
    int bv = E.variant, bb = E.bz;
    const int reps = 20;
    // bring the clocks up before timing anything
    if ((s = do_steps(E, 40, false, 0, -1.0)) == LLL_OK) s = settle(E);
    for (int trial = 0; trial < 2 && s == LLL_OK; ++trial) {
        for (auto& c : cands) {
            E.variant = c.first;
            E.bz = c.second;
            if ((s = do_steps(E, 2, false, 0, -1.0)) != LLL_OK) break;  // warm-up
            if ((s = settle(E)) != LLL_OK) break;
            HIP_TRY(hipEventRecord(e0, E.st));
            if ((s = do_steps(E, reps, false, 0, -1.0)) != LLL_OK) break;
            HIP_TRY(hipEventRecord(e1, E.st));
            if ((s = settle(E)) != LLL_OK) break;
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bv = c.first;
                bb = c.second;
            }
        }
    }
    E.variant = bv;
    E.bz = bb;
    // kick placement: epilogue of the fused step, or its own launch (whole intervals timed;
    // the two differ by a few per cent of an interval, so three alternating trials of six)
    bool bk = true;
    if (s == LLL_OK && bv != 0 && n_interval >= 2) {
        double tk[2] = {1e30, 1e30};
        for (int trial = 0; trial < 3 && s == LLL_OK; ++trial)
            for (int mode = 0; mode < 2 && s == LLL_OK; ++mode) {
                E.kick_epilogue = mode == 1;
                if ((s = do_interval(E, n_interval, 0, -1.0)) != LLL_OK) break;
                HIP_TRY(hipEventRecord(e0, E.st));
                for (int q = 0; q < 6 && s == LLL_OK; ++q) s = do_interval(E, n_interval, 1 + q, -1.0);
                HIP_TRY(hipEventRecord(e1, E.st));
                if (s == LLL_OK) s = settle(E);
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                tk[mode] = std::min(tk[mode], (double)ms);
            }
        bk = tk[1] <= tk[0];
    }
    E.kick_epilogue = bk;
    // maxima of the timing runs are dropped: kickdev is restored below
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipError_t ce = launch_copy(E.prec, E.s, save, E.nsites, E.st);
    if (ce == hipSuccess)
        ce = hipMemcpyAsync(E.d_kickdev, kd_save.data(), sizeof(unsigned long long) * kd_save.size(),
                            hipMemcpyHostToDevice, E.st);
    (void)hipStreamSynchronize(E.st);
    (void)hipFree(save.x);
    (void)hipFree(save.y);
    (void)hipFree(save.z);
    if (s != LLL_OK) return s;
    if (ce != hipSuccess) return set_err(LLL_EDEVICE, "restore failed");
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d\n", key.c_str(), bv, bb, bk ? 1 : 0);
            fclose(f);
        }
    }
    if (chosen_variant) *chosen_variant = bv;
    if (chosen_bz) *chosen_bz = bb;
    return LLL_OK;
}
}  // namespace

extern "C" lll_status lll_autotune(lll_lattice* L, const lll_params* p, const char* cache_path,
                                   int32_t* chosen_variant, int32_t* chosen_bz) {
    if (!L) return set_err(LLL_EINVAL, "lattice is NULL");
    lll_status s = lattice_params(L, p, false);
    if (s != LLL_OK) return s;
    char buf[200];
    snprintf(buf, sizeof buf, "L%dx%dx%d_bc%d_%s_prec%d_anis%d%s", L->Lx, L->Ly, L->Lz, L->bc,
             L->E.prec == 0 ? "fp64" : "fp32", L->E.precession, L->E.anis,
             L->E.integrator == LLL_RK2MID ? "_rk2" : L->E.integrator == LLL_RK5B ? "_rk5" : "");
    int64_t n = 0;
    if (steps_per_interval(L->dt, L->Dt, &n) != LLL_OK) n = 0;
    return engine_autotune(L->E, buf, L->Lz, n, cache_path, chosen_variant, chosen_bz);
}

// ------------------------------------------------------------- adjoint ----
// Reverse mode of the schedule, split into a forward call that records a
// tape and a backward call that takes the cotangent of the final state.  The
// forward pass advances the lattice like lll_run and stores the state before
// every ckpt_every-th operation (an operation is one RK4 step or one kick)
// and the final state; the backward pass walks the checkpoint blocks in
// reverse, recomputes each block while keeping the stage inputs of every
// step, and runs the reverse stages and kick reverses.  With ckpt_every = 0
// (full tape) the forward itself keeps the stage inputs of every step, in
// the same slot layout as a recomputed block that spans the whole run, and
// the backward recomputes nothing: a trade of memory (four states per
// operation) for one forward pass, cheap where the run fits in HBM many
// times over.  Work buffers of the backward pass live in the lattice's
// engine and are reused by later calls; a destroyed tape hands its
// checkpoint buffer back to the lattice, so a forward/backward cycle of the
// same length allocates nothing after the first.
namespace {
struct TmpAlloc {
    std::vector<void*> ptrs;
    ~TmpAlloc() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    void* get(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

State state_at(void* base, size_t comp_bytes, int64_t idx) {
    char* b = (char*)base + (size_t)idx * 3 * comp_bytes;
    return State{b, b + comp_bytes, b + 2 * comp_bytes};
}

// Grow-only device buffer.
lll_status ensure_buf(void** p, size_t* have, size_t bytes) {
    if (*p && *have >= bytes) return LLL_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return set_err(LLL_ENOMEM, "hipMalloc of %zu bytes failed (adjoint buffers)", bytes);
    }
    *have = bytes;
    return LLL_OK;
}
}  // namespace

struct lll_tape {
    lll_lattice* lat = nullptr;
    lll_params p{};
    std::vector<int8_t> op;        // 0 = RK4 step, 1 = kick
    std::vector<uint64_t> opk;     // pulse index of each operation
    int64_t K = 1, nblocks = 0;
    bool full = false;             // ckpt_every = 0: every step's stage inputs kept
    void* ck = nullptr;            // [nblocks + 1][3][N]: checkpoints, then s_T; full
                                   // tape: [4 nops + 1][3][N], x y2 y3 y4 per operation
    size_t ck_bytes = 0;
};

lll_lattice::~lll_lattice() {
    // tapes may outlive their lattice: their backward calls then fail cleanly,
    // and destroying them still frees their checkpoints
    for (lll_tape* T : tapes) T->lat = nullptr;
    if (adj_st2) {
        (void)hipStreamSynchronize(adj_st2);
        (void)hipStreamDestroy(adj_st2);
    }
    for (hipEvent_t e : adj_ev)
        if (e) (void)hipEventDestroy(e);
    for (void* p : {ck_pool, adj_bb, adj_sc, adj_small})
        if (p) (void)hipFree(p);
}

// Scratch states of the backward pass: the RK4 accumulator of a per-stage
// recompute (slot 0), the cotangents of the step output and input, the stage
// cotangent, and the two (q, loc) pairs of the reverse passes.
constexpr int kAdjScratch = 8;
constexpr int kAdjAcc = 0;

// Blocks of the adjoint's per-site kernels (one wave each).
static int adj_blocks(const Engine& E) { return (int)((E.nsites + kAdjBlock - 1) / kAdjBlock); }

// Adjoint work buffers of an engine: two block buffers of 4K + 1 states each
// (none for a full tape, K = 0), eight scratch states, parameter partials, their
// sum, the loss observables and the kick maxima of recomputed kicks (kept
// apart from the lattice's own); with checkpoints, the second stream and its
// events.
static lll_status ensure_adj_work(lll_lattice* L, int64_t K) {
    Engine& E = L->E;
    const size_t cb = (size_t)E.nsites * E.esz;
    lll_status s;
    if (K > 0 &&
        (s = ensure_buf(&L->adj_bb, &L->adj_bb_bytes, 3 * cb * 2 * (size_t)(4 * K + 1))) != LLL_OK)
        return s;
    if (K > 0 && !L->adj_st2) {
        // default priority, like every stream of the library
        HIP_TRY(hipStreamCreateWithFlags(&L->adj_st2, hipStreamNonBlocking));
        for (hipEvent_t& e : L->adj_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    if ((s = ensure_buf(&L->adj_sc, &L->adj_sc_bytes, 3 * cb * kAdjScratch)) != LLL_OK) return s;
    const size_t small = sizeof(double) * (5 * (size_t)adj_blocks(E) + 5 + 8) +
                         sizeof(unsigned long long) * kKickSlots;
    return ensure_buf(&L->adj_small, &L->adj_small_bytes, small);
}

static void tape_release_ck(lll_tape* T) {
    if (!T->ck) return;
    lll_lattice* L = T->lat;
    if (L && (!L->ck_pool || L->ck_pool_bytes < T->ck_bytes)) {
        if (L->ck_pool) (void)hipFree(L->ck_pool);
        L->ck_pool = T->ck;
        L->ck_pool_bytes = T->ck_bytes;
    } else {
        (void)hipFree(T->ck);
    }
    T->ck = nullptr;
    T->ck_bytes = 0;
}

// Forward pass with checkpoints; kicks fold their deviation into kd.
static lll_status tape_forward(lll_lattice* L, lll_tape* T, uint64_t first_pulse,
                               int64_t n_pulses, unsigned long long* kd) {
    Engine& E = L->E;
    int64_t n;
    lll_status s = steps_per_interval(T->p.dt, T->p.Dt, &n);
    if (s != LLL_OK) return s;
    const int64_t n1 = n / 2, n2 = n - n1;
    T->op.clear();
    T->opk.clear();
    for (int64_t q = 0; q < n_pulses; ++q) {
        const uint64_t k = first_pulse + (uint64_t)q;
        for (int64_t a = 0; a < n1; ++a) { T->op.push_back(0); T->opk.push_back(k); }
        T->op.push_back(1); T->opk.push_back(k);
        for (int64_t a = 0; a < n2; ++a) { T->op.push_back(0); T->opk.push_back(k); }
    }
    const int64_t nops = (int64_t)T->op.size();
    T->nblocks = T->full ? 1 : (nops + T->K - 1) / T->K;
    const size_t cb = (size_t)E.nsites * E.esz;
    const size_t need = 3 * cb * (size_t)(T->full ? 4 * nops + 1 : T->nblocks + 1);
    if (L->ck_pool && L->ck_pool_bytes >= need) {
        T->ck = L->ck_pool;
        T->ck_bytes = L->ck_pool_bytes;
        L->ck_pool = nullptr;
        L->ck_pool_bytes = 0;
    } else {
        if (hipMalloc(&T->ck, need) != hipSuccess) {
            T->ck = nullptr;
            return set_err(LLL_ENOMEM, "hipMalloc of %zu bytes failed (adjoint checkpoints)", need);
        }
        T->ck_bytes = need;
    }
    if ((s = settle(E)) != LLL_OK) return s;
    E.carried = false;
    const int pr = E.prec;
    if (T->full) {
        // slot j holds x, y2, y3, y4 of operation j; slot nops holds s_T
        auto slot = [&](int64_t j, int c) { return state_at(T->ck, cb, 4 * j + c); };
        if (E.variant != 0 && (s = ensure_tiles(E)) != LLL_OK) return s;
        if (E.variant == 0 && (s = ensure_adj_work(L, 0)) != LLL_OK) return s;
        const int pc = E.precession, an = E.anis;
        HIP_TRY(launch_copy(pr, slot(0, 0), E.s, E.nsites, E.st));
        for (int64_t j = 0; j < nops; ++j) {
            const State nx = slot(j + 1, 0);
            if (T->op[j] == 0 && E.variant != 0) {
                const State ys[3] = {slot(j, 1), slot(j, 2), slot(j, 3)};
                HIP_TRY(launch_step_fused_stages(pr, pc, an, E.variant, eff_bz(E), E.dreps,
                                                 E.d_tiles, E.ntiles, slot(j, 0), nx, ys, E.st));
            } else if (T->op[j] == 0) {
                HIP_TRY(launch_rk4_stages(pr, pc, an, E.dreps, E.d_blk_rep, E.nblk, slot(j, 0),
                                          slot(j, 1), slot(j, 2), slot(j, 3),
                                          state_at(L->adj_sc, cb, kAdjAcc), nx, E.st));
            } else {
                HIP_TRY(launch_copy(pr, nx, slot(j, 0), E.nsites, E.st));
                HIP_TRY(launch_kick(pr, E.dreps, E.d_blk_rep, E.nblk, nx, T->opk[j], -1.0, kd,
                                    E.st));
            }
        }
        HIP_TRY(launch_copy(pr, E.s, slot(nops, 0), E.nsites, E.st));
        return LLL_OK;
    }
    for (int64_t j = 0; j < nops;) {
        if (j % T->K == 0)
            HIP_TRY(launch_copy(pr, state_at(T->ck, cb, j / T->K), cur_state(E), E.nsites, E.st));
        if (T->op[j] == 1) {
            HIP_TRY(launch_kick(pr, E.dreps, E.d_blk_rep, E.nblk, cur_state(E), T->opk[j], -1.0, kd,
                                E.st));
            ++j;
            continue;
        }
        // consecutive steps up to the next kick or checkpoint
        int64_t e = j + 1;
        while (e < nops && T->op[e] == 0 && e % T->K != 0) ++e;
        if ((s = do_steps(E, e - j, false, 0, -1.0)) != LLL_OK) return s;
        j = e;
    }
    if ((s = settle(E)) != LLL_OK) return s;
    HIP_TRY(launch_copy(pr, state_at(T->ck, cb, T->nblocks), E.s, E.nsites, E.st));
    return LLL_OK;
}

// Backward pass for L = <cot, s_T> + wE E(s_T) + wm . m(s_T).
static lll_status tape_backward(lll_tape* T, const void* cot, double wE, const double wm[3],
                                double* loss, double* g_H, double* g_J, void* g_D, void* g_s0) {
    lll_lattice* L = T->lat;
    if (!L) return set_err(LLL_EINVAL, "the tape's lattice has been destroyed");
    lll_status s = lattice_params(L, &T->p, true);
    if (s != LLL_OK) return s;
    Engine& E = L->E;
    if ((s = ensure_adj_work(L, T->full ? 0 : T->K)) != LLL_OK) return s;
    if (E.variant != 0 && (s = ensure_tiles(E)) != LLL_OK) return s;
    const size_t cb = (size_t)E.nsites * E.esz;
    const int64_t nops = (int64_t)T->op.size();
    const int64_t K = T->full ? nops : T->K;
    double* part = (double*)L->adj_small;
    const int anb = adj_blocks(E);
    double* acc5 = part + 5 * (size_t)anb;
    double* res8 = acc5 + 5;
    unsigned long long* kd = (unsigned long long*)(res8 + 8);
    State accb = state_at(L->adj_sc, cb, kAdjAcc);
    State sbar = state_at(L->adj_sc, cb, 1), xbar = state_at(L->adj_sc, cb, 2);
    State kb = state_at(L->adj_sc, cb, 3);
    const State q2[2] = {state_at(L->adj_sc, cb, 4), state_at(L->adj_sc, cb, 6)};
    const State loc2[2] = {state_at(L->adj_sc, cb, 5), state_at(L->adj_sc, cb, 7)};
    // block buffer k (k = b & 1 for block b): slot j holds x, y2, y3, y4 of
    // operation j of the block (the full tape is one block that the forward
    // has already filled)
    void* const bb = T->full ? T->ck : L->adj_bb;
    const int64_t bstride = 4 * K + 1;
    auto slot_of = [&](int64_t b, int64_t j, int c) {
        return state_at(bb, cb, (T->full ? 0 : (b & 1) * bstride) + 4 * j + c);
    };
    const bool site = T->p.D_site != nullptr;
    double* gD = site ? (double*)g_D : nullptr;
    HIP_TRY(hipMemsetAsync(L->adj_small, 0, sizeof(double) * (5 * (size_t)anb + 5), E.st));
    if (site) HIP_TRY(hipMemsetAsync(gD, 0, sizeof(double) * E.nsites, E.st));
    const int pr = E.prec, pc = E.precession, an = E.anis;
    const State sT = T->full ? slot_of(0, nops, 0) : state_at(T->ck, cb, T->nblocks);
    const State cs = cot ? State{const_cast<void*>(cot), (char*)cot + cb, (char*)cot + 2 * cb}
                         : State{};
    HIP_TRY(launch_obs(pr, an, E.dreps, E.d_oblk_rep, E.nobblk, 1, sT, E.d_partials, res8, nullptr,
                       0, E.st));
    HIP_TRY(launch_adj_loss(pr, an, E.hreps[0], anb, sT, cs, sbar, wE, wm, gD, part,
                            E.st));
    const double dt = T->p.dt;
    // Recompute of checkpoint block b into buffer b & 1, on the second stream:
    // it runs while the block after it is reversed on the lattice's stream
    // (both are small, latency-bound launches that leave most CUs idle).  It
    // waits for the reverse that last read its buffer; the reverse of block b
    // waits for it.
    hipStream_t const s2 = L->adj_st2;
    bool reversed[2] = {false, false};
    auto recompute = [&](int64_t b) -> lll_status {
        const int64_t j0 = b * K, j1 = std::min(j0 + K, nops);
        if (reversed[b & 1]) HIP_TRY(hipStreamWaitEvent(s2, L->adj_ev[3 + (b & 1)], 0));
        HIP_TRY(launch_copy(pr, slot_of(b, 0, 0), state_at(T->ck, cb, b), E.nsites, s2));
        for (int64_t j = j0; j < j1; ++j) {
            const int64_t sl = j - j0;
            const State x = slot_of(b, sl, 0), nx = slot_of(b, sl + 1, 0);
            if (T->op[j] == 0 && E.variant != 0) {  // one fused launch: x', y2, y3, y4
                const State ys[3] = {slot_of(b, sl, 1), slot_of(b, sl, 2), slot_of(b, sl, 3)};
                HIP_TRY(launch_step_fused_stages(pr, pc, an, E.variant, eff_bz(E), E.dreps,
                                                 E.d_tiles, E.ntiles, x, nx, ys, s2));
            } else if (T->op[j] == 0) {
                HIP_TRY(launch_rk4_stages(pr, pc, an, E.dreps, E.d_blk_rep, E.nblk, x,
                                          slot_of(b, sl, 1), slot_of(b, sl, 2), slot_of(b, sl, 3),
                                          accb, nx, s2));
            } else {
                HIP_TRY(launch_copy(pr, nx, x, E.nsites, s2));
                HIP_TRY(launch_kick(pr, E.dreps, E.d_blk_rep, E.nblk, nx, T->opk[j], -1.0, kd, s2));
            }
        }
        HIP_TRY(hipEventRecord(L->adj_ev[1 + (b & 1)], s2));
        return LLL_OK;
    };
    // Stage 1's pass B of the last reversed step waits for the next operation
    // to reverse: when that is a step, one launch also does its stage-4 pass A
    // (pointwise in the finished cotangent), after its block is recomputed.
    bool pend_b1 = false;
    auto finish_b1 = [&](const State* y4prev) -> lll_status {
        HIP_TRY(launch_adj_b1(pr, pc, an, E.hreps[0], anb, y4prev, dt, sbar, xbar,
                              kb, q2, loc2, gD, part, E.st));
        std::swap(sbar, xbar);
        pend_b1 = false;
        return LLL_OK;
    };
    if (!T->full) {
        // the second stream starts after everything queued on the lattice's
        // stream so far (the forward that wrote the checkpoints included)
        HIP_TRY(hipEventRecord(L->adj_ev[0], E.st));
        HIP_TRY(hipStreamWaitEvent(s2, L->adj_ev[0], 0));
        if ((s = recompute(T->nblocks - 1)) != LLL_OK) return s;
    }
    for (int64_t b = T->nblocks - 1; b >= 0; --b) {
        const int64_t j0 = b * K, j1 = std::min(j0 + K, nops);
        if (!T->full) {
            if (b >= 1 && (s = recompute(b - 1)) != LLL_OK) return s;
            HIP_TRY(hipStreamWaitEvent(E.st, L->adj_ev[1 + (b & 1)], 0));
        }
        for (int64_t j = j1 - 1; j >= j0; --j) {
            const int64_t sl = j - j0;
            if (T->op[j] == 0) {
                const State y[4] = {slot_of(b, sl, 0), slot_of(b, sl, 1), slot_of(b, sl, 2),
                                    slot_of(b, sl, 3)};
                const bool a4 = !pend_b1;
                if (pend_b1 && (s = finish_b1(&y[3])) != LLL_OK) return s;
                HIP_TRY(launch_adj_step(pr, pc, an, E.hreps[0], anb, y, dt, sbar, xbar,
                                        kb, q2, loc2, gD, part, a4, E.st));
                pend_b1 = true;
            } else {
                if (pend_b1 && (s = finish_b1(nullptr)) != LLL_OK) return s;
                HIP_TRY(launch_adj_kick(pr, E.hreps[0], anb, slot_of(b, sl, 0), sbar,
                                        T->opk[j], -1.0, E.st));
            }
        }
        if (!T->full) {
            HIP_TRY(hipEventRecord(L->adj_ev[3 + (b & 1)], E.st));
            reversed[b & 1] = true;
        }
    }
    if (pend_b1 && (s = finish_b1(nullptr)) != LLL_OK) return s;
    HIP_TRY(launch_adj_finish(part, anb, acc5, E.st));
    if (g_s0) {
        State dst{g_s0, (char*)g_s0 + cb, (char*)g_s0 + 2 * cb};
        HIP_TRY(launch_copy(pr, dst, sbar, E.nsites, E.st));
    }
    double h5[5], r[8];
    HIP_TRY(hipMemcpyAsync(h5, acc5, sizeof h5, hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipMemcpyAsync(r, res8, sizeof r, hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipStreamSynchronize(E.st));
    if (loss) *loss = wE * r[0] + wm[0] * r[4] + wm[1] * r[5] + wm[2] * r[6];
    g_H[0] = h5[0];
    g_H[1] = h5[1];
    g_H[2] = h5[2];
    *g_J = h5[3];
    if (!site) *(double*)g_D = h5[4];
    if (!obs_finite(r)) return set_err(LLL_ENONFINITE, "forward state became NaN or Inf");
    return LLL_OK;
}

static lll_status tape_check_args(lll_lattice* L, const lll_params* p, int64_t n_pulses,
                                  int32_t ckpt_every) {
    if (!L || !p) return set_err(LLL_EINVAL, "NULL argument");
    if (n_pulses < 0 || ckpt_every < 0) return set_err(LLL_EINVAL, "bad n_pulses or ckpt_every");
    if (p->integrator != LLL_RK4)
        return set_err(LLL_EUNSUPPORTED, "the adjoint is implemented for LLL_RK4 only");
    return lattice_params(L, p, true);
}

extern "C" lll_status lll_adjoint_forward(lll_lattice* L, const lll_params* p, uint64_t first_pulse,
                                          int64_t n_pulses, int32_t ckpt_every, lll_tape** out) {
    if (!out) return set_err(LLL_EINVAL, "out is NULL");
    *out = nullptr;
    lll_status s = tape_check_args(L, p, n_pulses, ckpt_every);
    if (s != LLL_OK) return s;
    lll_tape* T = new lll_tape();
    T->lat = L;
    T->p = *p;
    T->K = ckpt_every > 0 ? ckpt_every : 1;
    T->full = ckpt_every == 0;
    if ((s = tape_forward(L, T, first_pulse, n_pulses, L->E.d_kickdev)) != LLL_OK) {
        tape_release_ck(T);
        delete T;
        return s;
    }
    L->tapes.push_back(T);
    *out = T;
    return LLL_OK;
}

extern "C" lll_status lll_adjoint_backward(lll_tape* T, const void* cot, double wE,
                                           const double wm[3], double* loss, double* g_H,
                                           double* g_J, void* g_D, void* g_s0) {
    if (!T || !wm || !g_H || !g_J || !g_D) return set_err(LLL_EINVAL, "NULL argument");
    return tape_backward(T, cot, wE, wm, loss, g_H, g_J, g_D, g_s0);
}

extern "C" void lll_tape_destroy(lll_tape* T) {
    if (!T) return;
    lll_lattice* L = T->lat;
    if (L) {
        if (L->E.st) (void)hipStreamSynchronize(L->E.st);
        else (void)hipDeviceSynchronize();
        if (L->adj_st2) (void)hipStreamSynchronize(L->adj_st2);
        auto& v = L->tapes;
        v.erase(std::remove(v.begin(), v.end(), T), v.end());
    }
    tape_release_ck(T);
    delete T;
}

extern "C" lll_status lll_adjoint(lll_lattice* L, const lll_params* p, uint64_t first_pulse,
                                  int64_t n_pulses, int32_t ckpt_every, double wE,
                                  const double wm[3], double* loss, double* g_H, double* g_J,
                                  void* g_D, void* g_s0) {
    if (!loss || !g_H || !g_J || !g_D || !wm) return set_err(LLL_EINVAL, "NULL argument");
    lll_status s = tape_check_args(L, p, n_pulses, ckpt_every);
    if (s != LLL_OK) return s;
    if ((s = ensure_adj_work(L, ckpt_every)) != LLL_OK) return s;
    lll_tape T;
    T.lat = L;
    T.p = *p;
    T.K = ckpt_every > 0 ? ckpt_every : 1;
    T.full = ckpt_every == 0;
    // the forward's kicks go to the scratch maxima: the state is restored
    unsigned long long* kd =
        (unsigned long long*)((double*)L->adj_small + 5 * (size_t)adj_blocks(L->E) + 5 + 8);
    s = tape_forward(L, &T, first_pulse, n_pulses, kd);
    if (s == LLL_OK) s = tape_backward(&T, nullptr, wE, wm, loss, g_H, g_J, g_D, g_s0);
    Engine& E = L->E;
    if (T.ck) {
        const hipError_t e = launch_copy(E.prec, E.s, state_at(T.ck, (size_t)E.nsites * E.esz, 0),
                                         E.nsites, E.st);
        E.cur = 0;
        (void)hipStreamSynchronize(E.st);
        if (s == LLL_OK && e != hipSuccess) s = set_err(LLL_EDEVICE, "state restore failed");
    }
    tape_release_ck(&T);
    return s;
}

// --------------------------------------------------------------- batch -----
// A captured run schedule of a batch: n_pulses intervals measured every
// obs_every, replayable for any first pulse.
struct BatchGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t npulses = -1;
    int32_t obs_every = -1;
    uint64_t used = 0;  // recency, for replacing the older of the two
    void clear() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        npulses = -1;
        obs_every = -1;
    }
};

// Pulses captured in one graph at most: a longer run replays graphs of chunks
// of at most this length (see lll_batch_run), up to three kept side by side.
// A single graph of tens of thousands of intervals (hundreds of thousands of
// kernel nodes) is not built.
constexpr int64_t kBatchGraphPulses = 1000;
constexpr int kBatchGraphs = 3;

struct lll_batch {
    Engine E;
    double dt = 0, Dt = 0;
    int64_t n = 0;
    BatchGraph g[kBatchGraphs];
    uint64_t uses = 0;
    void clear_graphs() {
        for (BatchGraph& c : g) c.clear();
    }
    ~lll_batch() { clear_graphs(); }
};

extern "C" lll_status lll_batch_create(int32_t n_rep, const lll_replica_desc* reps,
                                       lll_precision prec, double dt, double Dt,
                                       int32_t precession, void* hip_stream, lll_batch** out) {
    if (!out) return set_err(LLL_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_rep < 1 || !reps) return set_err(LLL_EINVAL, "need at least one replica");
    if (prec != LLL_FP64 && prec != LLL_FP32) return set_err(LLL_EINVAL, "bad precision");
    int64_t n;
    lll_status s = steps_per_interval(dt, Dt, &n);
    if (s != LLL_OK) return s;
    lll_batch* B = new lll_batch();
    Engine& E = B->E;
    E.prec = prec == LLL_FP64 ? 0 : 1;
    E.esz = E.prec == 0 ? 8 : 4;
    E.st = (hipStream_t)hip_stream;
    E.nrep = n_rep;
    E.hreps.assign(n_rep, RepDev{});
    E.precession = precession ? 1 : 0;
    int anis = ANIS_NONE;
    int64_t total = 0;
    for (int r = 0; r < n_rep; ++r) {
        const lll_replica_desc& d = reps[r];
        if (d.Lx < 1 || d.Ly < 1 || d.Lz < 1) { delete B; return set_err(LLL_EINVAL, "replica %d: bad size", r); }
        if (d.bc != LLL_BC_PERIODIC && d.bc != LLL_BC_FREE) { delete B; return set_err(LLL_EINVAL, "replica %d: bad bc", r); }
        const int64_t nr = checked_sites(d.Lx, d.Ly, d.Lz);
        if (nr < 0) { delete B; return set_err(LLL_EINVAL, "replica %d: at most 2^31-1 sites", r); }
        total += nr;  // at most n_rep * 2^31, no overflow
        Phys ph{};
        ph.J = d.J;
        for (int c = 0; c < 3; ++c) { ph.H[c] = d.H[c]; ph.e[c] = d.e[c]; }
        ph.D = d.D;
        ph.lambda = d.lambda;
        ph.T = d.T;
        if ((s = check_phys(ph)) != LLL_OK) { delete B; return s; }
        RepDev& R = E.hreps[r];
        memset(&R, 0, sizeof R);
        R.Lx = d.Lx; R.Ly = d.Ly; R.Lz = d.Lz; R.bc = d.bc;
        R.init = d.init == LLL_INIT_DIRECTION ? 1 : 0;
        fill_physics(R, ph, dt, Dt, E.precession, d.seed, d.replica);
        const int a = anis_mode_of(ph);
        if (a == ANIS_AXIS || (a == ANIS_Z && anis == ANIS_NONE)) anis = std::max(anis, a);
    }
    if (total > 0x7FFFFFFFLL) { delete B; return set_err(LLL_EINVAL, "too many sites in the batch"); }
    E.anis = anis;
    B->dt = dt;
    B->Dt = Dt;
    B->n = n;
    if ((s = build_tables(E)) != LLL_OK) { delete B; return s; }
    E.own_s = true;
    if ((s = alloc_state(E, E.s)) != LLL_OK) { delete B; return s; }
    if ((s = upload_reps(E)) != LLL_OK) { delete B; return s; }
    hipError_t e = launch_init(E.prec, E.dreps, E.d_blk_rep, E.nblk, E.s, 0, 0.0, 0.0, 1.0, E.st);
    if (e != hipSuccess) { delete B; return set_err(LLL_EDEVICE, "init failed"); }
    E.variant = fused_variant_count(E.prec) > 0 ? 1 : 0;
    E.bz = 0;
    *out = B;
    return LLL_OK;
}

// One captured (or replayed) schedule of at most kBatchGraphPulses intervals.
static lll_status batch_run_chunk(lll_batch* B, uint64_t first_pulse, int64_t n_pulses,
                                  int32_t obs_every, lll_obs* trace) {
    Engine& E = B->E;
    const int64_t nmeas = obs_every > 0 ? n_pulses / obs_every : 0;
    lll_status s;
    if (nmeas > 0 && (s = ensure_trace(E, (size_t)nmeas * 8 * E.nrep)) != LLL_OK) return s;
    if (nmeas > 0 && (s = ensure_obs_stage(E)) != LLL_OK) return s;
    if ((s = settle(E)) != LLL_OK) return s;
    // Tables and buffers must exist before capture (their uploads synchronise).
    if (E.variant == 0 || E.anis == ANIS_SITE) {
        if ((s = ensure_unfused_scratch(E)) != LLL_OK) return s;
    } else {
        if ((s = alloc_state(E, E.alt)) != LLL_OK) return s;
        if ((s = ensure_tiles(E)) != LLL_OK) return s;
    }
    // The captured schedule carries pulse indices relative to the first pulse
    // (the kernels add the descriptors' kbase), so it replays for any first
    // pulse with the same length and measurement spacing.
    BatchGraph* G = nullptr;
    for (BatchGraph& c : B->g)
        if (c.exec && c.npulses == n_pulses && c.obs_every == obs_every) G = &c;
    if (!G) {
        G = &B->g[0];  // the least recently used
        for (BatchGraph& c : B->g)
            if (c.used < G->used) G = &c;
        G->clear();
        hipStream_t cs = E.st;
        bool made_stream = false;
        if (!cs) {
            HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            made_stream = true;
        }
        hipStream_t saved = E.st;
        E.st = cs;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        lll_status cap = LLL_OK;
        E.carried = false;
        obs_begin(E, E.d_trace, (int64_t)8 * E.nrep);
        for (int64_t q = 0; q < n_pulses && cap == LLL_OK; ++q) {
            const uint64_t k = (uint64_t)q;  // relative to the first pulse
            const bool measure = obs_every > 0 && (q + 1) % obs_every == 0;
            cap = do_interval(E, B->n, k, -1.0, q + 1 < n_pulses && !measure, k + 1, -1.0);
            if (cap == LLL_OK && measure) cap = obs_stage(E);
        }
        if (cap == LLL_OK) cap = obs_fold(E);  // every replay ends with nothing staged
        if (cap == LLL_OK) cap = settle(E);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(cs, &g);
        E.st = saved;
        if (cap != LLL_OK) {
            if (g) (void)hipGraphDestroy(g);
            if (made_stream) (void)hipStreamDestroy(cs);
            return cap;
        }
        if (ee != hipSuccess) {
            if (made_stream) (void)hipStreamDestroy(cs);
            return set_err(LLL_EDEVICE, "graph capture failed: %s", hipGetErrorString(ee));
        }
        if (made_stream) (void)hipStreamDestroy(cs);
        G->graph = g;
        HIP_TRY(hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0));
        G->npulses = n_pulses;
        G->obs_every = obs_every;
    }
    G->used = ++B->uses;
    HIP_TRY(launch_set_pulse_base(E.dreps, E.nrep, first_pulse, E.st));
    HIP_TRY(hipGraphLaunch(G->exec, E.st));
    if (trace && nmeas > 0) {
        std::vector<double> h((size_t)nmeas * 8 * E.nrep);
        HIP_TRY(hipMemcpyAsync(h.data(), E.d_trace, sizeof(double) * h.size(),
                               hipMemcpyDeviceToHost, E.st));
        HIP_TRY(hipStreamSynchronize(E.st));
        bool fin = true;
        for (size_t j = 0; j < (size_t)nmeas * E.nrep; ++j) {
            obs_from(&h[8 * j], &trace[j]);
            fin = fin && obs_finite(&h[8 * j]);
        }
        if (!fin) return set_err(LLL_ENONFINITE, "a replica became NaN or Inf");
        const double dev = max_norm_dev_of(h.data(), (int64_t)nmeas * E.nrep);
        if (dev > LLL_NORM_WARN_LEVEL) return norm_warning(dev);
    }
    return LLL_OK;
}

extern "C" lll_status lll_batch_run(lll_batch* B, uint64_t first_pulse, int64_t n_pulses,
                                    int32_t obs_every, lll_obs* trace) {
    if (!B) return set_err(LLL_EINVAL, "batch is NULL");
    if (n_pulses < 0 || obs_every < 0) return set_err(LLL_EINVAL, "bad counts");
    if (n_pulses <= kBatchGraphPulses)
        return batch_run_chunk(B, first_pulse, n_pulses, obs_every, trace);
    // Chunks whose measurements fall where one run would take them: with a
    // spacing of at most kBatchGraphPulses, chunks of a whole number of
    // spacings; with a longer spacing, each measurement period as unmeasured
    // chunks of kBatchGraphPulses and a last chunk measured at its end.  The
    // intervals, kicks and measurements are those of one run (a kick is
    // applied with the same bits whether it rides on the step before it or
    // not), and the running sums are added in measurement order.
    lll_status warn = LLL_OK;
    auto part = [&](uint64_t done, int64_t len, int32_t every, int64_t meas_before) {
        lll_obs* tr = trace && every > 0 ? trace + meas_before * B->E.nrep : nullptr;
        const lll_status s = batch_run_chunk(B, first_pulse + done, len, every, tr);
        if (s > 0) warn = s;  // a warning: the work was done; report it at the end
        return s;
    };
    if (obs_every == 0 || obs_every <= kBatchGraphPulses) {
        int64_t chunk = kBatchGraphPulses;
        if (obs_every > 0) chunk = chunk / obs_every * obs_every;
        for (int64_t done = 0; done < n_pulses;) {
            const int64_t len = std::min(chunk, n_pulses - done);
            const lll_status s = part((uint64_t)done, len, obs_every,
                                      obs_every > 0 ? done / obs_every : 0);
            if (s < 0) return s;
            done += len;
        }
        return warn;
    }
    int64_t done = 0, meas = 0;
    for (; done + obs_every <= n_pulses; ++meas) {
        int64_t left = obs_every;
        while (left > kBatchGraphPulses) {
            const lll_status s = part((uint64_t)done, kBatchGraphPulses, 0, 0);
            if (s < 0) return s;
            done += kBatchGraphPulses;
            left -= kBatchGraphPulses;
        }
        const lll_status s = part((uint64_t)done, left, (int32_t)left, meas);
        if (s < 0) return s;
        done += left;
    }
    while (done < n_pulses) {
        const int64_t len = std::min(kBatchGraphPulses, n_pulses - done);
        const lll_status s = part((uint64_t)done, len, 0, 0);
        if (s < 0) return s;
        done += len;
    }
    return warn;
}

extern "C" lll_status lll_batch_observables(lll_batch* B, lll_obs* out) {
    if (!B || !out) return set_err(LLL_EINVAL, "NULL argument");
    Engine& E = B->E;
    lll_status s;
    if ((s = settle(E)) != LLL_OK) return s;
    if ((s = do_obs(E, E.d_result, 0)) != LLL_OK) return s;
    std::vector<double> h((size_t)8 * E.nrep);
    HIP_TRY(hipMemcpyAsync(h.data(), E.d_result, sizeof(double) * h.size(), hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipStreamSynchronize(E.st));
    bool fin = true;
    for (int r = 0; r < E.nrep; ++r) {
        obs_from(&h[8 * r], &out[r]);
        fin = fin && obs_finite(&h[8 * r]);
    }
    if (!fin) return set_err(LLL_ENONFINITE, "a replica holds NaN or Inf");
    const double dev = max_norm_dev_of(h.data(), E.nrep);
    if (dev > LLL_NORM_WARN_LEVEL) return norm_warning(dev);
    return LLL_OK;
}

extern "C" lll_status lll_batch_state(lll_batch* B, int32_t rep, void** sx, void** sy, void** sz) {
    if (!B || !sx || !sy || !sz) return set_err(LLL_EINVAL, "NULL argument");
    if (rep < 0 || rep >= B->E.nrep) return set_err(LLL_EINVAL, "replica out of range");
    const int64_t off = B->E.hreps[rep].off;
    *sx = (char*)B->E.s.x + off * B->E.esz;
    *sy = (char*)B->E.s.y + off * B->E.esz;
    *sz = (char*)B->E.s.z + off * B->E.esz;
    return LLL_OK;
}

extern "C" lll_status lll_batch_accumulators(lll_batch* B, double* out, int32_t reset) {
    if (!B || !out) return set_err(LLL_EINVAL, "NULL argument");
    Engine& E = B->E;
    HIP_TRY(hipMemcpyAsync(out, E.d_accum, sizeof(double) * 8 * E.nrep, hipMemcpyDeviceToHost, E.st));
    HIP_TRY(hipStreamSynchronize(E.st));
    if (reset) {
        HIP_TRY(hipMemsetAsync(E.d_accum, 0, sizeof(double) * 8 * E.nrep, E.st));
        HIP_TRY(hipStreamSynchronize(E.st));
    }
    return LLL_OK;
}

extern "C" lll_status lll_batch_autotune(lll_batch* B, const char* cache_path,
                                         int32_t* chosen_variant, int32_t* chosen_bz) {
    if (!B) return set_err(LLL_EINVAL, "batch is NULL");
    Engine& E = B->E;
    // key: replica count, total sites, largest z extent, precision, equation, anisotropy
    int maxLz = 1;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the replica shapes
    for (int r = 0; r < E.nrep; ++r) {
        maxLz = std::max(maxLz, E.hreps[r].Lz);
        const int32_t dims[4] = {E.hreps[r].Lx, E.hreps[r].Ly, E.hreps[r].Lz, E.hreps[r].bc};
        for (int q = 0; q < 4; ++q) {
            h ^= (uint64_t)(uint32_t)dims[q];
            h *= 1099511628211ull;
        }
    }
    char buf[200];
    snprintf(buf, sizeof buf, "B%d_%lld_%016llx_%s_prec%d_anis%d", E.nrep, (long long)E.nsites,
             (unsigned long long)h, E.prec == 0 ? "fp64" : "fp32", E.precession, E.anis);
    lll_status s = engine_autotune(E, buf, maxLz, B->n, cache_path, chosen_variant, chosen_bz);
    B->clear_graphs();
    return s;
}

extern "C" void lll_batch_destroy(lll_batch* B) {
    if (!B) return;
    if (B->E.st) (void)hipStreamSynchronize(B->E.st);
    else (void)hipDeviceSynchronize();
    delete B;
}

// ------------------------------------------------------------- escape -----
extern "C" lll_status lll_escape_times(const lll_escape_params* p, int64_t n_runs,
                                       int64_t max_pulses, double* times_dev, void* hip_stream) {
    if (!p) return set_err(LLL_EINVAL, "params is NULL");
    if (n_runs < 0 || n_runs > 0xFFFFFFFFLL) return set_err(LLL_EINVAL, "n_runs out of range");
    if (max_pulses < 1) return set_err(LLL_EINVAL, "max_pulses < 1");
    if (n_runs > 0 && !times_dev) return set_err(LLL_EINVAL, "times_dev is NULL");
    if (!(p->D > 0) || !is_fin(p->D)) return set_err(LLL_EINVAL, "D must be positive");
    const double h = p->H / (2.0 * p->D);
    if (!(h >= 0.0 && h < 1.0)) return set_err(LLL_EINVAL, "need 0 <= H/(2D) < 1");
    if (!(p->lambda >= 0) || !is_fin(p->lambda) || !(p->T >= 0) || !is_fin(p->T))
        return set_err(LLL_EINVAL, "lambda and T must be finite and >= 0");
    if (!(p->dt > 0) || !is_fin(p->dt)) return set_err(LLL_EINVAL, "dt must be positive");
    if (p->integrator != LLL_RK4 && p->integrator != LLL_RK2MID && p->integrator != LLL_RK5B)
        return set_err(LLL_EINVAL, "unknown integrator %d", (int)p->integrator);
    int64_t n;
    lll_status s = steps_per_interval(p->dt, p->Dt, &n);
    if (s != LLL_OK) return s;
    if (n_runs == 0) return LLL_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    Phys ph{};
    ph.J = 0.0;
    ph.H[0] = p->H;
    ph.D = p->D;
    ph.e[2] = 1.0;
    ph.lambda = p->lambda;
    ph.T = p->T;
    RepDev R{};
    R.Lx = R.Ly = R.Lz = 1;
    R.bc = 1;
    fill_physics(R, ph, p->dt, p->Dt, p->precession ? 1 : 0, p->seed, p->replica);
    const Tableau tb = tableau_of(p->integrator);
    TmpAlloc tmp;
    double* st3 = (double*)tmp.get(sizeof(double) * 3 * (size_t)n_runs);
    unsigned int* act = (unsigned int*)tmp.get(sizeof(unsigned int));
    if (!st3 || !act) return set_err(LLL_ENOMEM, "escape scratch allocation failed");
    {
        std::vector<double> neg((size_t)n_runs, -1.0);
        HIP_TRY(hipMemcpyAsync(times_dev, neg.data(), sizeof(double) * neg.size(),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    // bounded launches: a chunk of pulses each, until every run has escaped
    const int64_t chunk = std::max<int64_t>(1, 6000 / (n * tb.stages));
    for (int64_t k0 = 0; k0 < max_pulses; k0 += chunk) {
        const int64_t k1 = std::min(max_pulses, k0 + chunk);
        HIP_TRY(hipMemsetAsync(act, 0, sizeof(unsigned int), st));
        HIP_TRY(launch_escape(R, tb, p->precession ? 1 : 0, n_runs, n, p->dt, k0, k1, h, st3,
                              st3 + n_runs, st3 + 2 * n_runs, times_dev, act, st));
        unsigned int left = 0;
        HIP_TRY(hipMemcpyAsync(&left, act, sizeof left, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (left == 0) break;
    }
    return LLL_OK;
}
