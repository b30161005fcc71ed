// C ABI of the moment-pass least-squares fit (declared in include/lsefit.h).
//
// Host side only: argument validation, workspace carving, the launch schedule,
// plans (tuned schedule + own workspace + captured HIP graph) and the order of
// kernel launches for each call.  Every step of the computation runs in the
// kernels of kernels_impl.hpp and dispatch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lsefit.h"
#include "tune_cache.hpp"

using namespace lsefit;

namespace lsefit {
TimingSlot& timing_slot() {
    static thread_local TimingSlot slot;
    return slot;
}
}  // namespace lsefit

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultWavesPerCU = 8;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t tile_start, pstatus, rec, part, block_tot, total;
};

Layout layout(int64_t B, int maxM, int64_t W) {
    Layout L{};
    size_t off = 0;
    L.tile_start = off;
    off = align_up(off + sizeof(int64_t) * (size_t)(B + 2));
    L.pstatus = off;
    off = align_up(off + sizeof(int32_t) * (size_t)B);
    L.rec = off;
    off = align_up(off + sizeof(double) * (size_t)B * rec_len(maxM));
    L.part = off;
    // the slots may also hold streaming QR factors (fit_qr, degree <= LSEFIT_MAX_DEGREE)
    const int per = (maxM <= LSEFIT_MAX_DEGREE && qr_len(maxM) > nacc(maxM)) ? qr_len(maxM) : nacc(maxM);
    off = align_up(off + sizeof(double) * (size_t)(W + B) * per);
    L.block_tot = off;
    off = align_up(off + sizeof(int64_t) * (size_t)((B + kPlanThreads - 1) / kPlanThreads));
    L.total = off + kAlign;   // slack for aligning the caller's base pointer
    return L;
}

Work carve(void* ws, const Layout& L) {
    uintptr_t base = ((uintptr_t)ws + kAlign - 1) / kAlign * kAlign;
    Work w;
    w.tile_start = (int64_t*)(base + L.tile_start);
    w.pstatus = (int32_t*)(base + L.pstatus);
    w.rec = (double*)(base + L.rec);
    w.part = (double*)(base + L.part);
    w.block_tot = (int64_t*)(base + L.block_tot);
    w.clock = nullptr;   // armed per launch by launch_timed only
    return w;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

lsefit_schedule initial_schedule() {
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    lsefit_schedule s;
    s.waves = cus * kDefaultWavesPerCU;
    s.waves_per_block = 4;
    s.tile = 2048;
    s.unroll = 2;
    return s;
}

std::mutex g_sched_mu;
bool g_sched_set = false;
bool g_sched_user = false;   // set by lsefit_set_default_schedule (not the initial one)
lsefit_schedule g_sched;

lsefit_schedule current_default(bool* user = nullptr) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    if (!g_sched_set) {
        g_sched = initial_schedule();
        g_sched_set = true;
    }
    if (user) *user = g_sched_user;
    return g_sched;
}

// The launch shape of the adjoint passes (fit_backward): they keep no per-wave
// partial sums (tiles go to blocks, and a block streams each segment with all
// its waves), so their grid need not be the forward's.  Unless the caller set a
// default schedule, they run 16 waves per compute unit, 2 per block, 1 vector
// in flight per lane: on the MI355X, 4,096 fits x 4,096 float32 points,
// 46 us against 54.6 us with the forward's default shape (bit for bit the same
// gradients under every shape).
lsefit_schedule adjoint_schedule() {
    bool user = false;
    lsefit_schedule s = current_default(&user);
    if (user) return s;
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    s.waves = cus * 16;
    s.waves_per_block = 2;
    s.unroll = 1;
    return s;
}

// Below this many bytes of points a single fit's power-sum or refinement pass
// runs the small-fit grid.
constexpr int64_t kSmallFitBytes = (int64_t)32 << 20;

// The launch shape of a single fit's power-sum, refinement and residual
// passes: the default schedule, except that while the default is the initial
// one, a power-basis fit of fewer than kSmallFitBytes of points runs 4 waves
// per compute unit instead of 8, with 4 vectors in flight per lane for
// float64 points (2 for float32): fewer block partials for the finish to sum,
// and more bytes in flight per wave.  Measured on the MI355X for 1e6 float64
// points (16 MB); at 1e7 float32 points (80 MB) and above the default grid is
// as fast or faster.
lsefit_schedule single_schedule(int64_t n, int dt, const lsefit_options* o) {
    bool user = false;
    lsefit_schedule s = current_default(&user);
    if (user || o->basis != LSEFIT_BASIS_MONOMIAL) return s;
    const int64_t bytes = n * 2 * (dt == LSEFIT_F32 ? 4 : 8);
    if (bytes >= kSmallFitBytes) return s;
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    s.waves = cus * 4;
    s.unroll = dt == LSEFIT_F64 ? 4 : 2;
    return s;
}

bool schedule_ok(const lsefit_schedule& s) {
    const int wpb = s.waves_per_block;
    return s.waves >= 1 && s.waves <= (1 << 22) && (wpb == 1 || wpb == 2 || wpb == 4) && s.tile >= 64 &&
           (s.unroll == 1 || s.unroll == 2 || s.unroll == 4);
}

Launch to_launch(const lsefit_schedule& s) {
    Launch L;
    L.wpb = s.waves_per_block;
    L.waves = (int64_t)(s.waves + L.wpb - 1) / L.wpb * L.wpb;   // whole blocks
    L.tile = s.tile;
    L.unroll = s.unroll;
    return L;
}

// common misalignment (elements modulo the 16-byte vector width) of the given
// pointers, or -1 when they differ or are not element-aligned
int common_mis(int dt, std::initializer_list<const void*> ptrs) {
    const uintptr_t es = dt == LSEFIT_F32 ? 4 : 8;
    const uintptr_t vw = 16 / es;
    int mis = -1;
    for (const void* p : ptrs) {
        if (!p) continue;
        const uintptr_t a = (uintptr_t)p;
        if (a % es) return -1;
        const int m = (int)((a / es) % vw);
        if (mis < 0) mis = m;
        else if (mis != m) return -1;
    }
    return mis;
}

bool chebyshev(const lsefit_options* o) { return o->basis == LSEFIT_BASIS_CHEBYSHEV; }

bool opts_ok(const lsefit_options* o, int dt, bool batched) {
    if (!o) return false;
    if (o->basis != LSEFIT_BASIS_MONOMIAL && o->basis != LSEFIT_BASIS_CHEBYSHEV) return false;
    if (o->degree < 1 || o->degree > (chebyshev(o) ? LSEFIT_MAX_DEGREE_CHEBYSHEV : LSEFIT_MAX_DEGREE)) return false;
    if (o->precision != LSEFIT_PREC_F64 && o->precision != LSEFIT_PREC_F32C) return false;
    if (o->refine_steps < 0 || o->refine_steps > 1) return false;
    if (o->range_mode != LSEFIT_RANGE_GIVEN && o->range_mode != LSEFIT_RANGE_AUTO) return false;
    if (o->range_mode == LSEFIT_RANGE_GIVEN && !(std::isfinite(o->center) && std::isfinite(o->scale) && o->scale > 0))
        return false;
    if (dt != LSEFIT_F32 && dt != LSEFIT_F64) return false;
    if (o->solver != LSEFIT_SOLVER_GEPP && o->solver != LSEFIT_SOLVER_CHOLESKY) return false;
    if (o->output_basis != LSEFIT_OUTPUT_X && o->output_basis != LSEFIT_OUTPUT_X_AND_T) return false;
    (void)batched;
    return true;
}

// batched monomial fits that also return b and (c, s)
bool t_output(const lsefit_options* o) { return o->output_basis == LSEFIT_OUTPUT_X_AND_T && !chebyshev(o); }

// the coefficient row of a batched call holds what the options ask for
bool stride_ok(const lsefit_options* o, int32_t coef_stride) {
    return coef_stride >= (t_output(o) ? 2 * o->degree + 4 : o->degree + 1);
}

bool refining(const lsefit_options* o) {
    return o->precision == LSEFIT_PREC_F32C && o->refine_steps > 0 && !chebyshev(o);
}

// combinations the kernels do not implement
bool unsupported(const lsefit_options* o, int dt) {
    if (o->precision == LSEFIT_PREC_F32C && dt != LSEFIT_F32) return true;
    if (chebyshev(o) && o->precision != LSEFIT_PREC_F64) return true;
    return false;
}

#define LSEFIT_TRY(expr)                                   \
    do {                                                   \
        if ((expr) != hipSuccess) return LSEFIT_ERR_DEVICE; \
    } while (0)

// ---------------------------------------------------------------------------
// optional kernel timing: the first kernel of a timed launcher carries a pair
// of events that record its own dispatch's start and end (launch_timed)
// ---------------------------------------------------------------------------
enum TimedKind {
    kTimeMoments = 0,
    kTimeRefine = 1,
    kTimeAdjoint = 2,
    kTimeCombine = 3,
    kTimeProbe = 4,
    kTimeResidual = 5,
    kTimeRange = 6,
    kTimePlan = 7,
    kTimeKinds = 8
};

// the launches of each kind get one clock slot each (kClockWords uint64
// words: the start, and the last end of each group of waves) from a device
// pool taken when timing is first enabled; reading copies the used slots back
// and turns their spans into milliseconds at the device's wall-clock rate
constexpr int kClockSlots = 1 << 14;

struct Timing {
    std::mutex mu;
    bool enabled = false;
    uint64_t* slots = nullptr;   // device [kClockWords * kClockSlots]
    double khz = 0.0;            // wall-clock rate
    int used = 0;                // slots handed out since the last reset
    std::vector<std::pair<int, int>> pending;   // (kind, slot) not read yet
    double total_ms[kTimeKinds] = {};
    int64_t launches[kTimeKinds] = {};
};
Timing g_timing;

// while a NoTiming guard lives on a host thread, its launches are never timed
thread_local bool t_no_timing = false;
struct NoTiming {
    bool prev;
    NoTiming() : prev(t_no_timing) { t_no_timing = true; }
    ~NoTiming() { t_no_timing = prev; }
};

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// slots [lo, hi) back to (start = max, ends = 0), so that an unwritten start
// is seen and the kernels' atomic maxima take their first values; the device
// is idle when called
hipError_t clear_slots(int lo, int hi) {
    if (hi <= lo) return hipSuccess;
    std::vector<uint64_t> init(kClockWords * (size_t)(hi - lo), 0);
    for (size_t i = 0; i < init.size(); i += kClockWords) init[i] = ~(uint64_t)0;
    return hipMemcpy(g_timing.slots + kClockWords * (size_t)lo, init.data(), init.size() * sizeof(uint64_t),
                     hipMemcpyHostToDevice);
}

// runs `launch` on `st`; when timing is on, its first kernel started through
// launch_timed stamps its start and end into a fresh clock slot
template <class F>
hipError_t timed(int kind, hipStream_t st, F&& launch) {
    int idx = -1;
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        if (g_timing.enabled && g_timing.slots && !t_no_timing && g_timing.used < kClockSlots) idx = g_timing.used;
    }
    if (idx < 0 || capturing(st)) return launch();
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        idx = g_timing.used++;
    }
    TimingSlot& slot = timing_slot();
    slot.slot = g_timing.slots + kClockWords * (size_t)idx;
    slot.used = false;
    const hipError_t e = launch();
    const bool used = slot.used;
    slot = TimingSlot{};
    if (e == hipSuccess && used) {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.pending.push_back({kind, idx});
    }
    return e;
}

// the whole batched forward on one stream
lsefit_status enqueue_batched(const FitDesc& d, const Work& w, const lsefit_options* o, int dt, const void* x,
                              const void* y, double* coef, int32_t coef_stride, int32_t* status,
                              const lsefit_schedule& sched, hipStream_t st) {
    const Launch L = to_launch(sched);
    const int maxM = o->degree;
    const bool given = o->range_mode == LSEFIT_RANGE_GIVEN;
    const int mis = common_mis(dt, {x, y});
    const bool by_block = L.waves >= 64 * d.batch;
    Finish solve{kSolve, coef, coef_stride, 0, status, nullptr, o->solver};
    if (t_output(o)) {
        solve.b_at = maxM + 1;
        solve.cs_at = 2 * maxM + 2;
    }
    Finish refine = solve;
    refine.mode = kRefine;
    if (chebyshev(o)) {
        // the plan takes the given (c, s), or a placeholder the range pass replaces
        LSEFIT_TRY(timed(kTimePlan, st, [&] {
            return launch_plan(d, w, maxM, L.tile, true, given ? o->center : 0.0, given ? o->scale : 1.0, dt, x,
                               w.block_tot, st);
        }));
        if (!given)
            LSEFIT_TRY(timed(kTimeRange, st, [&] { return launch_range_cheb(d, w, maxM, dt, x, L, mis, st); }));
        const RangeArg ra{LSEFIT_RANGE_GIVEN, 0.0, 1.0};
        LSEFIT_TRY(timed(kTimeMoments, st,
                         [&] { return launch_moments_cheb(d, w, maxM, dt, x, y, L, mis, ra, st); }));
        LSEFIT_TRY(timed(kTimeCombine, st, [&] { return launch_finish_cheb(d, w, maxM, L.waves, solve, st); }));
        return LSEFIT_OK;
    }
    LSEFIT_TRY(timed(kTimePlan, st,
                     [&] { return launch_plan(d, w, maxM, L.tile, given, o->center, o->scale, dt, x, w.block_tot, st); }));
    const RangeArg ra{LSEFIT_RANGE_GIVEN, 0.0, 1.0};   // per-fit (c, s) are in the records
    LSEFIT_TRY(timed(kTimeMoments, st,
                     [&] { return launch_moments(d, w, maxM, o->precision, dt, x, y, L, mis, ra, st); }));
    LSEFIT_TRY(timed(kTimeCombine, st, [&] { return launch_combine(d, w, maxM, L, by_block, solve, st); }));
    if (refining(o)) {
        LSEFIT_TRY(timed(kTimeRefine, st, [&] { return launch_refine(d, w, maxM, dt, x, y, L, mis, st); }));
        LSEFIT_TRY(timed(kTimeCombine, st, [&] { return launch_combine(d, w, maxM, L, by_block, refine, st); }));
    }
    return LSEFIT_OK;
}

// validation shared by the single-fit entry points
lsefit_status check_single(const void* x, const void* y, int64_t n, int dt, const lsefit_options* opt, void* ws,
                           size_t ws_bytes, Layout* lay, lsefit_schedule* sched, bool power_sums = true) {
    if (!x || !y || !ws || !opts_ok(opt, dt, false)) return LSEFIT_ERR_INVALID_ARG;
    if (n < (int64_t)opt->degree + 1) return LSEFIT_ERR_INVALID_ARG;
    if (unsupported(opt, dt)) return LSEFIT_ERR_UNSUPPORTED;
    *sched = power_sums ? single_schedule(n, dt, opt) : current_default();
    *lay = layout(1, opt->degree, to_launch(*sched).waves);
    if (ws_bytes < lay->total) return LSEFIT_ERR_WORKSPACE;
    return LSEFIT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
struct lsefit_plan {
    int64_t batch = 0;
    int32_t max_degree = 0;
    int32_t dtype = 0;
    int32_t precision = 0;
    int device = 0;
    int64_t max_waves = 0;
    lsefit_schedule sched{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool graph_enabled = true;
    bool graph_user = false;   // the form was set by fit_plan_set_graph: tuning keeps it
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        const void *x, *y;
        const int64_t* offsets;
        const int32_t* degrees;
        int64_t batch;
        int32_t dt;
        lsefit_options opt;
        double* coef;
        int32_t coef_stride;
        int32_t* status;
    } key{};
    bool have_key = false;
    std::string tune_cache;   // schedule cache file of fit_plan_tune ("" = none)

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        have_key = false;
    }
};

namespace {

// ---------------------------------------------------------------------------
// schedule cache of fit_plan_tune (file format and parsing in tune_cache.hpp)
// ---------------------------------------------------------------------------
std::string tune_key(const lsefit_options* opt, int32_t dt, int64_t batch, int64_t points) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    return tune_cache::key(arch, device_cus(), opt, dt, batch, points);
}

bool same_key(const lsefit_plan::Key& a, const lsefit_plan::Key& b) {
    return a.x == b.x && a.y == b.y && a.offsets == b.offsets && a.degrees == b.degrees && a.batch == b.batch &&
           a.dt == b.dt && a.coef == b.coef && a.coef_stride == b.coef_stride && a.status == b.status &&
           std::memcmp(&a.opt, &b.opt, sizeof(lsefit_options)) == 0;
}

}  // namespace

extern "C" {

const char* lsefit_status_string(int32_t s) {
    switch (s) {   // an int: a value outside the enumeration is no lsefit_status
        case LSEFIT_OK: return "ok";
        case LSEFIT_ERR_INVALID_ARG: return "invalid argument";
        case LSEFIT_ERR_SINGULAR: return "singular normal system";
        case LSEFIT_ERR_NONFINITE: return "non-finite value";
        case LSEFIT_ERR_WORKSPACE: return "workspace too small";
        case LSEFIT_ERR_DEVICE: return "device or launch error";
        case LSEFIT_ERR_UNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

int32_t lsefit_device_cus(void) { return device_cus(); }

lsefit_status lsefit_default_schedule(lsefit_schedule* out) {
    if (!out) return LSEFIT_ERR_INVALID_ARG;
    *out = current_default();
    return LSEFIT_OK;
}

lsefit_status lsefit_set_default_schedule(const lsefit_schedule* s) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    if (!s) {
        g_sched = initial_schedule();
        g_sched_set = true;
        g_sched_user = false;
        return LSEFIT_OK;
    }
    if (!schedule_ok(*s)) return LSEFIT_ERR_INVALID_ARG;
    g_sched = *s;
    g_sched_set = true;
    g_sched_user = true;
    return LSEFIT_OK;
}

size_t lsefit_workspace_bytes(int64_t batch, int32_t max_degree, const lsefit_schedule* schedule) {
    if (batch < 1 || max_degree < 1 || max_degree > LSEFIT_MAX_DEGREE_CHEBYSHEV) return 0;
    const lsefit_schedule s = schedule ? *schedule : current_default();
    if (!schedule_ok(s)) return 0;
    return layout(batch, max_degree, to_launch(s).waves).total;
}

int64_t grid_blocks(const Launch& L) { return L.waves / L.wpb; }

// one streaming pass of a single fit (power sums or refinement), then the
// one-block kernel that sums the block partials and finishes the fit
lsefit_status single_pass(bool refine_pass, const FitDesc& d, const Work& w, const lsefit_options* opt, int dt,
                          const void* x, const void* y, const Launch& L, int mis, const Finish& fz, hipStream_t st) {
    const RangeArg ra{opt->range_mode, opt->center, opt->scale};
    if (chebyshev(opt)) {
        RangeArg rc = ra;
        if (opt->range_mode == LSEFIT_RANGE_AUTO) {
            LSEFIT_TRY(timed(kTimeRange, st,
                             [&] { return launch_range_cheb(d, w, opt->degree, dt, x, L, mis, st); }));
            rc.mode = kRangeFromRecord;
        }
        LSEFIT_TRY(timed(kTimeMoments, st,
                         [&] { return launch_moments_cheb(d, w, opt->degree, dt, x, y, L, mis, rc, st); }));
        LSEFIT_TRY(timed(kTimeCombine, st,
                         [&] { return launch_finish_cheb(d, w, opt->degree, grid_blocks(L), fz, st); }));
        return LSEFIT_OK;
    }
    if (refine_pass)
        LSEFIT_TRY(timed(kTimeRefine, st, [&] { return launch_refine(d, w, opt->degree, dt, x, y, L, mis, st); }));
    else
        LSEFIT_TRY(timed(kTimeMoments, st, [&] {
            return launch_moments(d, w, opt->degree, opt->precision, dt, x, y, L, mis, ra, st);
        }));
    LSEFIT_TRY(timed(kTimeCombine, st,
                     [&] { return launch_finish_single(d, w, opt->degree, grid_blocks(L), fz, st); }));
    return LSEFIT_OK;
}

lsefit_status fit_moments(const void* x, const void* y, int64_t n, int32_t dt, const lsefit_options* opt,
                          void* ws, size_t ws_bytes, double* moments, void* stream) {
    if (!moments) return LSEFIT_ERR_INVALID_ARG;
    Layout lay;
    lsefit_schedule sched;
    const lsefit_status v = check_single(x, y, n, dt, opt, ws, ws_bytes, &lay, &sched);
    if (v != LSEFIT_OK) return v;
    const FitDesc d{nullptr, nullptr, n, 1, opt->degree};
    const Finish fz{kMomentsOnly, nullptr, 0, 0, nullptr, moments, opt->solver};
    return single_pass(false, d, carve(ws, lay), opt, dt, x, y, to_launch(sched), common_mis(dt, {x, y}), fz,
                       (hipStream_t)stream);
}

lsefit_status fit_solve(const double* moments, const lsefit_options* opt, const void* x, const void* y, int64_t n,
                        int32_t dt, void* ws, size_t ws_bytes, double* coef, int32_t* status, void* stream) {
    if (!moments || !ws || !coef || !status || !opts_ok(opt, dt, false)) return LSEFIT_ERR_INVALID_ARG;
    if (chebyshev(opt) && opt->precision != LSEFIT_PREC_F64) return LSEFIT_ERR_UNSUPPORTED;
    const bool refine = refining(opt);
    if (refine) {
        if (!x || !y || n < (int64_t)opt->degree + 1) return LSEFIT_ERR_INVALID_ARG;
        if (dt != LSEFIT_F32) return LSEFIT_ERR_UNSUPPORTED;
    }
    const lsefit_schedule sched = refine ? single_schedule(n, dt, opt) : current_default();
    const Layout lay = layout(1, opt->degree, to_launch(sched).waves);
    if (ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{nullptr, nullptr, refine ? n : 0, 1, opt->degree};
    const Work w = carve(ws, lay);
    if (chebyshev(opt)) {
        const Finish fz{kSolve, coef, 2 * (opt->degree + 1), 1, status, nullptr, opt->solver};
        LSEFIT_TRY(timed(kTimeCombine, st, [&] { return launch_solve_cheb_moments(moments, w, opt->degree, fz, st); }));
        return LSEFIT_OK;
    }
    LSEFIT_TRY(timed(kTimeCombine, st, [&] {
        return launch_solve_moments(moments, w, opt->degree, opt->degree, opt->solver, coef, status, st);
    }));
    if (!refine) return LSEFIT_OK;
    const Finish fz{kRefine, coef, 2 * (opt->degree + 1), 1, status, nullptr, opt->solver};
    return single_pass(true, d, w, opt, dt, x, y, to_launch(sched), common_mis(dt, {x, y}), fz, st);
}

namespace {

// the launches of one single fit (fit_single, fit_single_noalloc) on a
// validated workspace
lsefit_status enqueue_single(const void* x, const void* y, int64_t n, int dt, const lsefit_options* opt, void* ws,
                             const Layout& lay, const lsefit_schedule& sched, double* coef, int32_t* status,
                             double* moments, hipStream_t st) {
    const FitDesc d{nullptr, nullptr, n, 1, opt->degree};
    const Work w = carve(ws, lay);
    const Launch L = to_launch(sched);
    const int mis = common_mis(dt, {x, y});
    const int stride = 2 * (opt->degree + 1);
    const Finish solve{kSolve, coef, stride, 1, status, moments, opt->solver};
    lsefit_status r = single_pass(false, d, w, opt, dt, x, y, L, mis, solve, st);
    if (r != LSEFIT_OK || !refining(opt)) return r;
    const Finish fz{kRefine, coef, stride, 1, status, nullptr, opt->solver};
    return single_pass(true, d, w, opt, dt, x, y, L, mis, fz, st);
}

}  // namespace

lsefit_status fit_single(const void* x, const void* y, int64_t n, int32_t dt, const lsefit_options* opt,
                         void* ws, size_t ws_bytes, double* coef, int32_t* status, double* moments, void* stream) {
    if (!coef || !status) return LSEFIT_ERR_INVALID_ARG;
    Layout lay;
    lsefit_schedule sched;
    const lsefit_status v = check_single(x, y, n, dt, opt, ws, ws_bytes, &lay, &sched);
    if (v != LSEFIT_OK) return v;
    return enqueue_single(x, y, n, dt, opt, ws, lay, sched, coef, status, moments, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// fit_single_noalloc: the workspace of fit_single in a static device array.
// Each GPU the library runs on holds its own copy (a module global is
// instantiated per device); its address on the current device is taken once,
// with hipGetSymbolAddress, and kept per device ordinal.  The array's name is
// a host-side stand-in and is never passed to a kernel or a copy.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LSEFIT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the scratch array's device address on the current device (taken on the first
// call there), or nullptr when the device or the symbol cannot be resolved
void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

lsefit_status fit_single_noalloc(const void* x, const void* y, int64_t n, int32_t dt,
                                 const lsefit_options* opt, double* coef, int32_t* status, double* moments,
                                 void* stream) {
    if (!coef || !status || !x || !y || !opts_ok(opt, dt, false)) return LSEFIT_ERR_INVALID_ARG;
    if (n < (int64_t)opt->degree + 1) return LSEFIT_ERR_INVALID_ARG;
    if (unsupported(opt, dt)) return LSEFIT_ERR_UNSUPPORTED;
    const lsefit_schedule sched = single_schedule(n, dt, opt);
    const Layout lay = layout(1, opt->degree, to_launch(sched).waves);
    if (lay.total > (size_t)LSEFIT_NOALLOC_SCRATCH_BYTES) return LSEFIT_ERR_WORKSPACE;
    void* ws = scratch_on_current_device();
    if (!ws) return LSEFIT_ERR_DEVICE;
    NoTiming quiet;   // the timing events of lsefit_timing_* may be created on demand: not here
    return enqueue_single(x, y, n, dt, opt, ws, lay, sched, coef, status, moments, (hipStream_t)stream);
}

lsefit_status fit_qr(const void* x, const void* y, int64_t n, int32_t dt, const lsefit_options* opt, void* ws,
                     size_t ws_bytes, double* coef, int32_t* status, double* info, void* stream) {
    if (!coef || !status) return LSEFIT_ERR_INVALID_ARG;
    Layout lay;
    lsefit_schedule sched;
    const lsefit_status v = check_single(x, y, n, dt, opt, ws, ws_bytes, &lay, &sched, false);
    if (v != LSEFIT_OK) return v;
    if (opt->precision != LSEFIT_PREC_F64 || chebyshev(opt)) return LSEFIT_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{nullptr, nullptr, n, 1, opt->degree};
    const Work w = carve(ws, lay);
    const Launch L = to_launch(sched);
    const int mis = common_mis(dt, {x, y});
    const RangeArg ra{opt->range_mode, opt->center, opt->scale};
    LSEFIT_TRY(timed(kTimeMoments, st, [&] { return launch_qr_single(d, w, dt, x, y, L, mis, ra, st); }));
    LSEFIT_TRY(timed(kTimeCombine, st,
                     [&] { return launch_qr_finish(d, w, grid_blocks(L), coef, status, info, st); }));
    return LSEFIT_OK;
}

lsefit_status fit_qr_batched(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                             int64_t batch, int32_t dt, const lsefit_options* opt, void* ws, size_t ws_bytes,
                             double* coef, int32_t coef_stride, int32_t* status, double* sse, void* stream) {
    if (batch < 0 || !opts_ok(opt, dt, true)) return LSEFIT_ERR_INVALID_ARG;
    if (batch == 0) return LSEFIT_OK;
    if (!x || !y || !offsets || !degrees || !coef || !status) return LSEFIT_ERR_INVALID_ARG;
    if (coef_stride < opt->degree + 1) return LSEFIT_ERR_INVALID_ARG;
    if (opt->precision != LSEFIT_PREC_F64 || chebyshev(opt)) return LSEFIT_ERR_UNSUPPORTED;
    const lsefit_schedule sched = current_default();
    const Launch L = to_launch(sched);
    const Layout lay = layout(batch, opt->degree, L.waves);
    if (!ws || ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{offsets, degrees, 0, batch, opt->degree};
    const Work w = carve(ws, lay);
    const bool given = opt->range_mode == LSEFIT_RANGE_GIVEN;
    const int mis = common_mis(dt, {x, y});
    LSEFIT_TRY(timed(kTimePlan, st, [&] {
        return launch_plan(d, w, opt->degree, L.tile, given, opt->center, opt->scale, dt, x, w.block_tot, st);
    }));
    LSEFIT_TRY(timed(kTimeMoments, st, [&] { return launch_qr_batch(d, w, opt->degree, dt, x, y, L, mis, st); }));
    LSEFIT_TRY(timed(kTimeCombine, st, [&] {
        return launch_qr_combine(d, w, opt->degree, L.waves, coef, coef_stride, status, sse, st);
    }));
    return LSEFIT_OK;
}

extern "C++" {
namespace {

// One call of a plan through its captured graph: capture (on the plan's own
// stream) when the arguments differ from the captured call's, then replay.
lsefit_status plan_graph_call(lsefit_plan* plan, const FitDesc& d, const Work& w, const lsefit_options* opt,
                              int32_t dt, const void* x, const void* y, double* coef, int32_t coef_stride,
                              int32_t* status, hipStream_t st) {
    lsefit_plan::Key key{x, y, d.offsets, d.degrees, d.batch, dt, *opt, coef, coef_stride, status};
    if (!(plan->exec && plan->have_key && same_key(plan->key, key))) {
        plan->drop_graph();
        if (!plan->cap_stream) LSEFIT_TRY(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
        LSEFIT_TRY(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
        const lsefit_status s =
            enqueue_batched(d, w, opt, dt, x, y, coef, coef_stride, status, plan->sched, plan->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(plan->cap_stream, &graph);
        if (s != LSEFIT_OK || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return s != LSEFIT_OK ? s : LSEFIT_ERR_DEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            plan->exec = nullptr;
            return LSEFIT_ERR_DEVICE;
        }
        plan->key = key;
        plan->have_key = true;
    }
    LSEFIT_TRY(hipGraphLaunch(plan->exec, st));
    return LSEFIT_OK;
}

// Time `reps` calls of fn (each returning an lsefit_status) on stream st, after
// one untimed call: milliseconds per call.
template <class F>
lsefit_status time_calls(hipStream_t st, int reps, F&& fn, double* ms_per_call) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return LSEFIT_ERR_DEVICE;
    }
    lsefit_status r = fn();
    if (r == LSEFIT_OK && hipEventRecord(e0, st) != hipSuccess) r = LSEFIT_ERR_DEVICE;
    for (int i = 0; i < reps && r == LSEFIT_OK; ++i) r = fn();
    float ms = 0.f;
    if (r == LSEFIT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        r = LSEFIT_ERR_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r == LSEFIT_OK) *ms_per_call = (double)ms / reps;
    return r;
}

// The replay form of a tuned plan: eager launches of its schedule against
// replays of the captured graph, timed on the same call; the faster is kept
// (*graph_out = 1 for the graph).  A form set with fit_plan_set_graph is kept.
// The eager launches have just run with these arguments, so a graph that
// cannot be captured or replayed here leaves the plan eager, not failed.
lsefit_status choose_replay_form(lsefit_plan* plan, const FitDesc& d, const Work& w, const lsefit_options* opt,
                                 const void* x, const void* y, double* coef, int32_t coef_stride, int32_t* status,
                                 hipStream_t st, int reps, int* graph_out) {
    *graph_out = -1;
    if (plan->graph_user) return LSEFIT_OK;
    const int32_t dt = plan->dtype;
    double te = 0.0, tg = 0.0;
    lsefit_status r = time_calls(st, reps, [&] {
        return enqueue_batched(d, w, opt, dt, x, y, coef, coef_stride, status, plan->sched, st);
    }, &te);
    if (r != LSEFIT_OK) return r;
    r = time_calls(st, reps, [&] { return plan_graph_call(plan, d, w, opt, dt, x, y, coef, coef_stride, status, st); },
                   &tg);
    if (r != LSEFIT_OK) {
        (void)hipGetLastError();   // the failed capture or launch, not the caller's
        if (hipStreamSynchronize(st) != hipSuccess) return LSEFIT_ERR_DEVICE;
        plan->graph_enabled = false;
        plan->drop_graph();
        *graph_out = 0;
        return LSEFIT_OK;
    }
    plan->graph_enabled = tg < te;
    if (!plan->graph_enabled) plan->drop_graph();
    *graph_out = plan->graph_enabled ? 1 : 0;
    return LSEFIT_OK;
}

}  // namespace
}  // extern "C++"

lsefit_status fit_batched(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                          int64_t batch, int32_t dt, const lsefit_options* opt, lsefit_plan* plan, void* ws,
                          size_t ws_bytes, double* coef, int32_t coef_stride, int32_t* status, void* stream) {
    if (batch < 0 || !opts_ok(opt, dt, true)) return LSEFIT_ERR_INVALID_ARG;
    if (batch == 0) return LSEFIT_OK;
    if (!x || !y || !offsets || !degrees || !coef || !status) return LSEFIT_ERR_INVALID_ARG;
    if (!stride_ok(opt, coef_stride)) return LSEFIT_ERR_INVALID_ARG;
    if (unsupported(opt, dt)) return LSEFIT_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{offsets, degrees, 0, batch, opt->degree};
    if (!plan) {
        const lsefit_schedule sched = current_default();
        const Layout lay = layout(batch, opt->degree, to_launch(sched).waves);
        if (!ws || ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
        return enqueue_batched(d, carve(ws, lay), opt, dt, x, y, coef, coef_stride, status, sched, st);
    }
    if (batch > plan->batch || opt->degree > plan->max_degree || dt != plan->dtype) return LSEFIT_ERR_INVALID_ARG;
    const Layout lay = layout(plan->batch, plan->max_degree, plan->max_waves);
    const Work w = carve(plan->ws, lay);
    if (!plan->graph_enabled)
        return enqueue_batched(d, w, opt, dt, x, y, coef, coef_stride, status, plan->sched, st);
    return plan_graph_call(plan, d, w, opt, dt, x, y, coef, coef_stride, status, st);
}

lsefit_status fit_backward(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                           int64_t batch, int32_t dt, const lsefit_options* opt, lsefit_plan* plan, void* ws,
                           size_t ws_bytes, const double* grad_coef, int32_t coef_stride, void* grad_x,
                           void* grad_y, void* stream) {
    if (batch < 0 || !opts_ok(opt, dt, true)) return LSEFIT_ERR_INVALID_ARG;
    if (batch == 0) return LSEFIT_OK;
    if (!x || !y || !offsets || !degrees || !grad_coef || !grad_x || !grad_y) return LSEFIT_ERR_INVALID_ARG;
    if (coef_stride < opt->degree + 1) return LSEFIT_ERR_INVALID_ARG;
    // the Chebyshev coefficients depend on (c, s); with the automatic range
    // those follow the extreme x, which this adjoint holds fixed
    if (chebyshev(opt) && opt->range_mode != LSEFIT_RANGE_GIVEN) return LSEFIT_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{offsets, degrees, 0, batch, opt->degree};
    Work w;
    lsefit_schedule sched;
    if (plan) {
        if (batch > plan->batch || opt->degree > plan->max_degree || dt != plan->dtype) return LSEFIT_ERR_INVALID_ARG;
        w = carve(plan->ws, layout(plan->batch, plan->max_degree, plan->max_waves));
        sched = plan->sched;
    } else {
        sched = current_default();
        const Layout lay = layout(batch, opt->degree, to_launch(sched).waves);
        if (!ws || ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
        w = carve(ws, lay);
    }
    const int mis = common_mis(dt, {x, y, grad_x, grad_y});
    const Launch La = to_launch(adjoint_schedule());
    if (chebyshev(opt)) {
        LSEFIT_TRY(timed(kTimeAdjoint, st, [&] {
            return launch_adjoint_cheb(d, w, opt->degree, opt->solver, dt, x, y, grad_coef, coef_stride, grad_x,
                                       grad_y, La, mis, st);
        }));
        return LSEFIT_OK;
    }
    LSEFIT_TRY(timed(kTimeAdjoint, st, [&] {
        return launch_adjoint(d, w, opt->degree, opt->solver, dt, x, y, grad_coef, coef_stride, grad_x, grad_y,
                              La, mis, st);
    }));
    return LSEFIT_OK;
}

lsefit_status fit_residuals(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                            int64_t batch, int64_t n, int32_t dt, const lsefit_options* opt, lsefit_plan* plan,
                            void* ws, size_t ws_bytes, double* sse, void* residuals, void* stream) {
    if (!x || !y || !sse || !opts_ok(opt, dt, offsets != nullptr)) return LSEFIT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int mis = common_mis(dt, {x, y, residuals});
    if (!offsets) {
        if (n < (int64_t)opt->degree + 1 || !ws) return LSEFIT_ERR_INVALID_ARG;
        const lsefit_schedule sched = single_schedule(n, dt, opt);
        const Layout lay = layout(1, opt->degree, to_launch(sched).waves);
        if (ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
        const FitDesc d{nullptr, nullptr, n, 1, opt->degree};
        const Work w = carve(ws, lay);
        const Launch L = to_launch(sched);
        if (chebyshev(opt)) {
            LSEFIT_TRY(timed(kTimeResidual, st, [&] {
                return launch_residual_cheb(d, w, opt->degree, dt, x, y, residuals, sse, L, mis, st);
            }));
            return LSEFIT_OK;
        }
        const Finish fz{kSSE, sse, 1, 0, nullptr, nullptr, opt->solver};
        LSEFIT_TRY(timed(kTimeResidual, st,
                         [&] { return launch_residual(d, w, opt->degree, dt, x, y, residuals, L, mis, st); }));
        LSEFIT_TRY(launch_finish_single(d, w, opt->degree, grid_blocks(L), fz, st));
        return LSEFIT_OK;
    }
    if (batch < 0 || !degrees) return LSEFIT_ERR_INVALID_ARG;
    if (batch == 0) return LSEFIT_OK;
    const FitDesc d{offsets, degrees, 0, batch, opt->degree};
    Work w;
    lsefit_schedule sched;
    if (plan) {
        if (batch > plan->batch || opt->degree > plan->max_degree || dt != plan->dtype) return LSEFIT_ERR_INVALID_ARG;
        w = carve(plan->ws, layout(plan->batch, plan->max_degree, plan->max_waves));
        sched = plan->sched;
    } else {
        sched = current_default();
        const Layout lay = layout(batch, opt->degree, to_launch(sched).waves);
        if (!ws || ws_bytes < lay.total) return LSEFIT_ERR_WORKSPACE;
        w = carve(ws, lay);
    }
    const Launch L = to_launch(sched);
    if (chebyshev(opt)) {
        LSEFIT_TRY(timed(kTimeResidual, st, [&] {
            return launch_residual_cheb(d, w, opt->degree, dt, x, y, residuals, sse, L, mis, st);
        }));
        return LSEFIT_OK;
    }
    const Finish fz{kSSE, sse, 1, 0, nullptr, nullptr, opt->solver};
    LSEFIT_TRY(timed(kTimeResidual, st,
                     [&] { return launch_residual(d, w, opt->degree, dt, x, y, residuals, L, mis, st); }));
    LSEFIT_TRY(launch_combine(d, w, opt->degree, L, L.waves >= 64 * d.batch, fz, st));
    return LSEFIT_OK;
}

lsefit_status fit_plan_create(lsefit_plan** out, int64_t batch, int32_t max_degree, int32_t dt,
                              int32_t precision) {
    if (!out || batch < 1 || max_degree < 1 || max_degree > LSEFIT_MAX_DEGREE_CHEBYSHEV) return LSEFIT_ERR_INVALID_ARG;
    if (dt != LSEFIT_F32 && dt != LSEFIT_F64) return LSEFIT_ERR_INVALID_ARG;
    if (precision != LSEFIT_PREC_F64 && precision != LSEFIT_PREC_F32C) return LSEFIT_ERR_INVALID_ARG;
    lsefit_plan* p = new (std::nothrow) lsefit_plan();
    if (!p) return LSEFIT_ERR_DEVICE;
    p->batch = batch;
    p->max_degree = max_degree;
    p->dtype = dt;
    p->precision = precision;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return LSEFIT_ERR_DEVICE;
    }
    p->sched = current_default();
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    p->max_waves = (int64_t)cus * 64;
    if (to_launch(p->sched).waves > p->max_waves) p->max_waves = to_launch(p->sched).waves;
    const Layout lay = layout(batch, max_degree, p->max_waves);
    if (hipMalloc(&p->ws, lay.total) != hipSuccess) {
        delete p;
        return LSEFIT_ERR_DEVICE;
    }
    p->ws_bytes = lay.total;
    *out = p;
    return LSEFIT_OK;
}

lsefit_status fit_plan_set_schedule(lsefit_plan* plan, const lsefit_schedule* s) {
    if (!plan || !s || !schedule_ok(*s) || to_launch(*s).waves > plan->max_waves) return LSEFIT_ERR_INVALID_ARG;
    plan->sched = *s;
    plan->drop_graph();
    return LSEFIT_OK;
}

lsefit_status fit_plan_get_schedule(const lsefit_plan* plan, lsefit_schedule* out) {
    if (!plan || !out) return LSEFIT_ERR_INVALID_ARG;
    *out = plan->sched;
    return LSEFIT_OK;
}

lsefit_status fit_plan_set_graph(lsefit_plan* plan, int32_t enable) {
    if (!plan) return LSEFIT_ERR_INVALID_ARG;
    plan->graph_enabled = enable != 0;
    plan->graph_user = true;
    plan->drop_graph();
    return LSEFIT_OK;
}

lsefit_status fit_plan_get_graph(const lsefit_plan* plan, int32_t* enabled) {
    if (!plan || !enabled) return LSEFIT_ERR_INVALID_ARG;
    *enabled = plan->graph_enabled ? 1 : 0;
    return LSEFIT_OK;
}

lsefit_status fit_plan_tune(lsefit_plan* plan, const void* x, const void* y, const int64_t* offsets,
                            const int32_t* degrees, int64_t batch, const lsefit_options* opt, double* coef,
                            int32_t coef_stride, int32_t* status, void* stream, int32_t reps, double* best_ms_out) {
    if (!plan || !opts_ok(opt, plan->dtype, true) || batch < 1 || batch > plan->batch) return LSEFIT_ERR_INVALID_ARG;
    if (!x || !y || !offsets || !degrees || !coef || !status) return LSEFIT_ERR_INVALID_ARG;
    if (opt->degree > plan->max_degree || !stride_ok(opt, coef_stride)) return LSEFIT_ERR_INVALID_ARG;
    if (unsupported(opt, plan->dtype)) return LSEFIT_ERR_UNSUPPORTED;
    if (reps < 1) reps = 3;
    hipStream_t st = (hipStream_t)stream;
    const FitDesc d{offsets, degrees, 0, batch, opt->degree};
    const Work w = carve(plan->ws, layout(plan->batch, plan->max_degree, plan->max_waves));
    std::string key;
    if (!plan->tune_cache.empty()) {
        int64_t ends[2] = {0, 0};
        if (hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&ends[1], offsets + batch, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return LSEFIT_ERR_DEVICE;
        key = tune_key(opt, plan->dtype, batch, ends[1] - ends[0]);
        lsefit_schedule cs{};
        double cms = 0.0;
        int cgraph = -1;
        if (tune_cache::lookup(plan->tune_cache, key, &cs, &cms, &cgraph) && schedule_ok(cs) &&
            to_launch(cs).waves <= plan->max_waves) {
            // a cached shape: one run with its schedule, no timing; the cached
            // replay form unless the caller set one
            const lsefit_status r = enqueue_batched(d, w, opt, plan->dtype, x, y, coef, coef_stride, status, cs, st);
            if (r != LSEFIT_OK) return r;
            if (hipStreamSynchronize(st) != hipSuccess) return LSEFIT_ERR_DEVICE;
            plan->sched = cs;
            plan->drop_graph();
            if (cgraph >= 0 && !plan->graph_user) plan->graph_enabled = cgraph == 1;
            if (best_ms_out) *best_ms_out = cms;
            return LSEFIT_OK;
        }
    }
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    std::vector<lsefit_schedule> cands;
    for (int wpc : {4, 8, 16, 32})
        for (int wpb : {2, 4})
            for (int tile : {256, 2048})
                for (int unroll : {1, 2, 4}) {
                    lsefit_schedule s{cus * wpc, wpb, tile, unroll};
                    if (to_launch(s).waves <= plan->max_waves) cands.push_back(s);
                }
    // first round: every candidate, `reps` timed calls each; second round: the
    // kTuneFinalists fastest again with 3 * reps calls each (one round's timing
    // moves by a few percent from run to run, about the gap between the leaders)
    constexpr size_t kTuneFinalists = 4;
    std::vector<std::pair<double, size_t>> first;
    lsefit_status r = LSEFIT_OK;
    for (size_t i = 0; i < cands.size(); ++i) {
        double per = 0.0;
        r = time_calls(st, reps, [&] {
            return enqueue_batched(d, w, opt, plan->dtype, x, y, coef, coef_stride, status, cands[i], st);
        }, &per);
        if (r != LSEFIT_OK) return r;
        first.emplace_back(per, i);
    }
    std::sort(first.begin(), first.end());
    double best = 1e300;
    lsefit_schedule best_s = plan->sched;
    for (size_t j = 0; j < first.size() && j < kTuneFinalists; ++j) {
        const lsefit_schedule& s = cands[first[j].second];
        double per = 0.0;
        r = time_calls(st, 3 * reps, [&] {
            return enqueue_batched(d, w, opt, plan->dtype, x, y, coef, coef_stride, status, s, st);
        }, &per);
        if (r != LSEFIT_OK) return r;
        if (per < best) {
            best = per;
            best_s = s;
        }
    }
    plan->sched = best_s;
    plan->drop_graph();
    int form = -1;
    r = choose_replay_form(plan, d, w, opt, x, y, coef, coef_stride, status, st, reps, &form);
    if (r != LSEFIT_OK) return r;
    if (best_ms_out) *best_ms_out = best;
    if (!key.empty()) tune_cache::store(plan->tune_cache, key, best_s, best, form);
    return LSEFIT_OK;
}

lsefit_status fit_plan_set_tune_cache(lsefit_plan* plan, const char* path) {
    if (!plan) return LSEFIT_ERR_INVALID_ARG;
    plan->tune_cache = path ? path : "";
    return LSEFIT_OK;
}

lsefit_status lsefit_read_probe(const float* x, const float* y, int64_t n, const lsefit_schedule* schedule,
                                int32_t pattern, int32_t nontemporal, float* out, size_t out_count, void* stream) {
    if (!x || !y || !out || n < 4 || pattern < 0 || pattern > 2) return LSEFIT_ERR_INVALID_ARG;
    if (((uintptr_t)x | (uintptr_t)y) % 16) return LSEFIT_ERR_INVALID_ARG;
    const lsefit_schedule s = schedule ? *schedule : current_default();
    if (!schedule_ok(s)) return LSEFIT_ERR_INVALID_ARG;
    const Launch L = to_launch(s);
    if (out_count < (size_t)(L.waves / L.wpb)) return LSEFIT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    LSEFIT_TRY(timed(kTimeProbe, st,
                     [&] { return launch_read_probe(x, y, n / 4, L, pattern, nontemporal != 0, out, st); }));
    return LSEFIT_OK;
}

lsefit_status lsefit_copy_probe(const float* x, const float* y, float* ox, float* oy, int64_t n,
                               const lsefit_schedule* schedule, int32_t pattern, int32_t nontemporal, void* stream) {
    if (!x || !y || !ox || !oy || n < 4 || pattern < 0 || pattern > 2) return LSEFIT_ERR_INVALID_ARG;
    if (((uintptr_t)x | (uintptr_t)y | (uintptr_t)ox | (uintptr_t)oy) % 16) return LSEFIT_ERR_INVALID_ARG;
    const lsefit_schedule s = schedule ? *schedule : current_default();
    if (!schedule_ok(s)) return LSEFIT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    LSEFIT_TRY(timed(kTimeProbe, st, [&] {
        return launch_copy_probe(x, y, ox, oy, n / 4, to_launch(s), pattern, nontemporal != 0, st);
    }));
    return LSEFIT_OK;
}

lsefit_status lsefit_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (enable && !g_timing.slots) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess) return LSEFIT_ERR_DEVICE;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            return LSEFIT_ERR_DEVICE;
        void* p = nullptr;
        if (hipMalloc(&p, kClockWords * sizeof(uint64_t) * (size_t)kClockSlots) != hipSuccess)
            return LSEFIT_ERR_DEVICE;
        g_timing.slots = (uint64_t*)p;
        g_timing.khz = (double)khz;
        g_timing.used = 0;
        if (hipDeviceSynchronize() != hipSuccess || clear_slots(0, kClockSlots) != hipSuccess) return LSEFIT_ERR_DEVICE;
    }
    g_timing.enabled = enable != 0;
    return LSEFIT_OK;
}

namespace {

// spans of the pending slots into the per-kind totals (waits for the device)
lsefit_status collect_pending() {
    if (g_timing.pending.empty()) return LSEFIT_OK;
    if (hipDeviceSynchronize() != hipSuccess) return LSEFIT_ERR_DEVICE;
    std::vector<uint64_t> host(kClockWords * (size_t)g_timing.used);
    if (hipMemcpy(host.data(), g_timing.slots, host.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return LSEFIT_ERR_DEVICE;
    for (const auto& p : g_timing.pending) {
        const uint64_t* sl = host.data() + kClockWords * (size_t)p.second;
        uint64_t end = 0;
        for (int j = 0; j < kClockLines; ++j) end = sl[8 * j + 1] > end ? sl[8 * j + 1] : end;
        if (sl[0] == ~(uint64_t)0 || end < sl[0]) continue;   // the kernel never ran
        g_timing.total_ms[p.first] += (double)(end - sl[0]) / g_timing.khz;
        g_timing.launches[p.first] += 1;
    }
    g_timing.pending.clear();
    return LSEFIT_OK;
}

}  // namespace

lsefit_status lsefit_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.pending.clear();
    for (int k = 0; k < kTimeKinds; ++k) {
        g_timing.total_ms[k] = 0.0;
        g_timing.launches[k] = 0;
    }
    if (g_timing.slots && g_timing.used > 0) {
        if (hipDeviceSynchronize() != hipSuccess || clear_slots(0, g_timing.used) != hipSuccess)
            return LSEFIT_ERR_DEVICE;
    }
    g_timing.used = 0;
    return LSEFIT_OK;
}

lsefit_status lsefit_timing_read(int32_t kind, double* total_ms, int64_t* launches) {
    if (kind < 0 || kind >= kTimeKinds || !total_ms || !launches) return LSEFIT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    const lsefit_status st = collect_pending();
    if (st != LSEFIT_OK) return st;
    *total_ms = g_timing.total_ms[kind];
    *launches = g_timing.launches[kind];
    return LSEFIT_OK;
}

void fit_plan_destroy(lsefit_plan* plan) {
    if (!plan) return;
    plan->drop_graph();
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    if (plan->ws) (void)hipFree(plan->ws);
    delete plan;
}

}  // extern "C"
