// Degree dispatch of the launchers, and the kernels that do not depend on the
// degree: the tile table and the sampled range.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launchers.hpp"

namespace lsefit {

// ---------------------------------------------------------------------------
// tile table: fit f gets ceil(L_f / tile) tiles; one block scans all fits.
// Also writes the plan status of each fit and, for a given range, (c, s).
// ---------------------------------------------------------------------------
constexpr int kPlanThreads = 1024;

__device__ inline int64_t plan_tiles(const FitDesc& d, int64_t f, int64_t tile) {
    const int64_t L = fit_hi(d, f) - fit_lo(d, f);
    return L <= 0 ? 0 : (L + tile - 1) / tile;
}

__global__ void __launch_bounds__(kPlanThreads)
    k_plan(FitDesc d, Work w, int maxM, int64_t tile, int range_given, double c, double s) {
    __shared__ int64_t sh[kPlanThreads];
    const int tid = threadIdx.x;
    const int64_t B = d.batch;
    const int64_t per = (B + kPlanThreads - 1) / kPlanThreads;
    int64_t f0 = (int64_t)tid * per;
    if (f0 > B) f0 = B;
    int64_t f1 = f0 + per;
    if (f1 > B) f1 = B;
    int64_t cnt = 0;
    for (int64_t f = f0; f < f1; ++f) cnt += plan_tiles(d, f, tile);
    sh[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const int64_t v = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    int64_t base = sh[tid] - cnt;
    const int rl = rec_len(maxM);
    for (int64_t f = f0; f < f1; ++f) {
        w.tile_start[f] = base;
        base += plan_tiles(d, f, tile);
        const int64_t L = fit_hi(d, f) - fit_lo(d, f);
        const int m = fit_deg(d, f);
        int st = LSEFIT_OK;
        if (m < 1 || m > maxM || L < 0) st = LSEFIT_ERR_INVALID_ARG;
        else if (L < m + 1) st = LSEFIT_ERR_SINGULAR;
        w.pstatus[f] = st;
        if (range_given) {
            w.rec[f * rl + 0] = c;
            w.rec[f * rl + 1] = s;
        }
    }
    if (tid == kPlanThreads - 1) w.tile_start[B] = sh[tid];
}

// ---------------------------------------------------------------------------
// sampled range
// ---------------------------------------------------------------------------
constexpr int kRangeBatchSamples = 16;

template <typename In>
__global__ void __launch_bounds__(256) k_range_batched(FitDesc d, Work w, int maxM, const In* __restrict__ x) {
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int lane = lane_id();
    const int rl = rec_len(maxM);
    for (int64_t f = wave0; f < d.batch; f += nw) {
        const int64_t base = fit_lo(d, f);
        const int64_t L = fit_hi(d, f) - base;
        const int64_t K = L < kRangeBatchSamples ? L : kRangeBatchSamples;
        double lo = INFINITY, hi = -INFINITY;
        if (lane < K) {
            const int64_t idx = K == 1 ? 0 : (int64_t)lane * (L - 1) / (K - 1);
            const double v = (double)x[base + idx];
            if (isfinite(v)) lo = hi = v;
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane == 0) {
            double c, s;
            snap_range(lo, hi, &c, &s);
            w.rec[f * rl + 0] = c;
            w.rec[f * rl + 1] = s;
        }
    }
}


// ---------------------------------------------------------------------------
// dispatch on the largest degree of the call
// ---------------------------------------------------------------------------
#define LSEFIT_SWITCH_MAXM(maxM, CALL)                   \
    switch (maxM) {                                      \
        case 1: { constexpr int MM = 1; CALL; } break; \
        case 2: { constexpr int MM = 2; CALL; } break; \
        case 3: { constexpr int MM = 3; CALL; } break; \
        case 4: { constexpr int MM = 4; CALL; } break; \
        case 5: { constexpr int MM = 5; CALL; } break; \
        case 6: { constexpr int MM = 6; CALL; } break; \
        case 7: { constexpr int MM = 7; CALL; } break; \
        case 8: { constexpr int MM = 8; CALL; } break; \
        default: break;                                  \
    }                                                    \
    return hipErrorInvalidValue;

hipError_t launch_plan(const FitDesc& d, const Work& w, int maxM, int64_t tile, bool range_given, double c,
                       double s, hipStream_t st) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, st, d, w, maxM, tile, range_given ? 1 : 0, c, s);
    return hipGetLastError();
}

hipError_t launch_range(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, hipStream_t st) {
    int64_t blocks = (d.batch + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (dtype == LSEFIT_F32)
        hipLaunchKernelGGL(k_range_batched<float>, dim3(blocks), dim3(256), 0, st, d, w, maxM, (const float*)x);
    else
        hipLaunchKernelGGL(k_range_batched<double>, dim3(blocks), dim3(256), 0, st, d, w, maxM, (const double*)x);
    return hipGetLastError();
}

hipError_t launch_moments(const FitDesc& d, const Work& w, int maxM, int prec, int dtype, const void* x,
                          const void* y, const Launch& L, int mis, const RangeArg& ra, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::moments(d, w, prec, dtype, x, y, L, mis, ra, st));
}

hipError_t launch_finish_single(const FitDesc& d, const Work& w, int maxM, int64_t blocks, const Finish& fz,
                                hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::finish_single(d, w, blocks, fz, st));
}

hipError_t launch_combine(const FitDesc& d, const Work& w, int maxM, const Launch& L, bool by_block,
                          const Finish& fz, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::combine(d, w, L, by_block, fz, st));
}

hipError_t launch_solve_moments(const double* moments, const Work& w, int m, int maxM, double* coef,
                                int32_t* status, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::solve_moments(moments, w, m, coef, status, st));
}

hipError_t launch_refine(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                         const Launch& L, int mis, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::refine(d, w, dtype, x, y, L, mis, st));
}

hipError_t launch_adjoint(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                          const double* grad_coef, int32_t coef_stride, void* gx, void* gy, const Launch& L,
                          int mis, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::adjoint(d, w, dtype, x, y, grad_coef, coef_stride, gx, gy, L,
                                                           mis, st));
}

}  // namespace lsefit
