// Host-side launchers of the streaming and solve kernels (monomial basis: kernels_m1..8.hip through
// dispatch.hip; Chebyshev basis: cheb.hip; streaming QR: tsqr.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace lsefit {

// Kernel timing (lsefit_timing_*).  The host side arms a clock slot on its
// thread before it calls a launcher; the first kernel that launcher starts
// through launch_timed gets the slot in its workspace argument (Work::clock,
// or KClock for the probes), and the kernel itself stamps its start and end
// there (KernelClock).  Nothing else is enqueued, so timed launches run back
// to back as untimed ones do.  With nothing armed, launch_timed is a plain
// launch.
struct TimingSlot {
    uint64_t* slot = nullptr;
    bool used = false;
};
TimingSlot& timing_slot();   // this host thread's slot (api.hip)

template <typename T>
inline T with_clock(const T& v, uint64_t*) {
    return v;
}
inline Work with_clock(const Work& w, uint64_t* slot) {
    Work c = w;
    c.clock = slot;
    return c;
}
inline KClock with_clock(const KClock&, uint64_t* slot) { return KClock{slot}; }

template <typename K, typename... Args>
inline void launch_timed(K kernel, const dim3& grid, const dim3& block, hipStream_t st, Args... args) {
    TimingSlot& t = timing_slot();
    if (t.slot && !t.used) {
        t.used = true;
        hipLaunchKernelGGL(kernel, grid, block, 0, st, with_clock(args, t.slot)...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    }
}

struct Launch {
    int64_t waves;        // total waves of the persistent grid
    int32_t wpb;          // waves per block
    int64_t tile;         // points per tile
    int32_t unroll;       // vector loads in flight per lane and array
};

enum CombineMode { kNoFinish = -1, kMomentsOnly = 0, kSolve = 1, kRefine = 2, kSSE = 3 };

// What happens once the partial sums of a fit are complete: write its power
// sums (kMomentsOnly), solve (kSolve), apply the refinement correction
// (kRefine), or store the sum of squared residuals (kSSE, into coef[f]).
// Passed to the combine and finish kernels.
struct Finish {
    int mode;
    double* coef;          // [B * coef_stride] x-basis coefficients (kSSE: [B] sums)
    int32_t coef_stride;
    int write_b;           // also write the t-basis solution after a_0..a_m
    int32_t* status;       // [B]
    double* moments_out;   // nullable: [3m+4] = c, s, S_0..S_2m, T_0..T_m
    int solver;            // lsefit_solver
    int32_t b_at = -1;     // >= 0: batched t-basis output, b_0..b_m of fit f from
                           // coef[f * coef_stride + b_at] on
    int32_t cs_at = -1;    // >= 0: the fit's c and s at coef[f * coef_stride + cs_at] and + 1
};

// Range of a single fit: given (c, s), or derived by the streaming kernel itself.
struct RangeArg {
    int mode;   // lsefit_range_mode, or kRangeFromRecord
    double c, s;
};
// (c, s) already in the fit's record (written by an earlier range pass)
constexpr int kRangeFromRecord = 2;

// Batched: tile table, plan status and (c, s) of every fit (given, or from a
// sample of the fit's x), in two launches (one for at most 32 blocks of fits and
// a power-of-two tile); block_tot holds plan_blocks(B) int64.
int64_t plan_blocks(int64_t batch);
hipError_t launch_plan(const FitDesc& d, const Work& w, int maxM, int64_t tile, bool range_given, double c,
                       double s, int dtype, const void* x, int64_t* block_tot, hipStream_t st);

// The power-sum pass: per-(wave, fit) partial sums (batched) or per-block
// partial sums (single fit) into w.part.
hipError_t launch_moments(const FitDesc& d, const Work& w, int maxM, int prec, int dtype, const void* x,
                          const void* y, const Launch& L, int mis, const RangeArg& ra, hipStream_t st);

// Single fit: sum the block partials and finish (mode of fz).
hipError_t launch_finish_single(const FitDesc& d, const Work& w, int maxM, int64_t blocks, const Finish& fz,
                                hipStream_t st);

// Fixed-order sum of the partial slots of each fit, then (mode) write the power
// sums, solve, or apply the refinement correction.  by_block: one block per fit
// (few fits), else one thread per fit.
hipError_t launch_combine(const FitDesc& d, const Work& w, int maxM, const Launch& L, bool by_block,
                          const Finish& fz, hipStream_t st);

// Solve one fit from caller-provided power sums [c, s, S_0..S_2m, T_0..T_m].
hipError_t launch_solve_moments(const double* moments, const Work& w, int m, int maxM, int solver, double* coef,
                                int32_t* status, hipStream_t st);

// Refinement pass: per-(wave, fit) partial sums of t^j (y - f(t)) into w.part.
hipError_t launch_refine(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                         const Launch& L, int mis, hipStream_t st);

// Adjoint: lambda per fit, then dL/dx, dL/dy per point.
hipError_t launch_adjoint(const FitDesc& d, const Work& w, int maxM, int solver, int dtype, const void* x,
                          const void* y, const double* grad_coef, int32_t coef_stride, void* gx, void* gy,
                          const Launch& L, int mis, hipStream_t st);

// Residual pass: e = y - f(t) per point (optionally stored) and partial sums of
// e^2 (per block for a single fit, per wave and fit for a batch) into w.part.
hipError_t launch_residual(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                           void* resid, const Launch& L, int mis, hipStream_t st);

// Read-bandwidth probe over two float32 arrays of nvec 16-byte vectors each;
// one float per block into out.
hipError_t launch_read_probe(const float* x, const float* y, int64_t nvec, const Launch& L, int pattern, bool nt,
                             float* out, hipStream_t st);
// Copy probe: x, y -> ox, oy over nvec 16-byte vectors each (8 B read and 8 B
// written per float32 point, the traffic of the adjoint pass).
hipError_t launch_copy_probe(const float* x, const float* y, float* ox, float* oy, int64_t nvec, const Launch& L,
                             int pattern, bool nt, hipStream_t st);

// Chebyshev basis (degree up to LSEFIT_MAX_DEGREE_CHEBYSHEV, float64 sums):
// streaming pass, per-fit finish (single fit: W = number of block partials),
// and a solve from caller-provided sums.
// exact extent of the finite x of every fit -> (c, s) of the Chebyshev basis in
// its record (a streaming pass over x with per-block / per-slot min and max,
// then a per-fit fold)
hipError_t launch_range_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const Launch& L,
                             int mis, hipStream_t st);
hipError_t launch_moments_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                               const Launch& L, int mis, const RangeArg& ra, hipStream_t st);
hipError_t launch_finish_cheb(const FitDesc& d, const Work& w, int maxm, int64_t W, const Finish& fz,
                              hipStream_t st);
hipError_t launch_solve_cheb_moments(const double* moments, const Work& w, int m, const Finish& fz,
                                    hipStream_t st);
// residuals of Chebyshev-basis fits: e = y - sum_j c_j T_j(t) per point
// (optionally stored) and sse[f] = sum e^2 (NaN for fits whose status is not OK)
hipError_t launch_residual_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                                void* resid, double* sse, const Launch& L, int mis, hipStream_t st);
// adjoint of a Chebyshev-basis batch with a given range: lambda = G^-1 dL/dc per
// fit, then dL/dx and dL/dy per point (NaN for fits whose status is not OK)
hipError_t launch_adjoint_cheb(const FitDesc& d, const Work& w, int maxm, int solver, int dtype, const void* x,
                               const void* y, const double* grad_coef, int32_t coef_stride, void* gx, void* gy,
                               const Launch& L, int mis, hipStream_t st);

// Streaming QR of one fit (degree d.degree): per-block factors into w.part,
// then one block merges them, solves and writes [a | b], the status and info.
hipError_t launch_qr_single(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y,
                            const Launch& L, int mis, const RangeArg& ra, hipStream_t st);
hipError_t launch_qr_finish(const FitDesc& d, const Work& w, int64_t G, double* coef, int32_t* status, double* info,
                            hipStream_t st);
// Streaming QR of a batch: per-(wave, fit) factors into w.part (after the tile
// table), then one thread per fit merges, solves and writes a, status, sse.
hipError_t launch_qr_batch(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                           const Launch& L, int mis, hipStream_t st);
hipError_t launch_qr_combine(const FitDesc& d, const Work& w, int maxm, int64_t W, double* coef, int32_t coef_stride,
                             int32_t* status, double* sse, hipStream_t st);

}  // namespace lsefit
