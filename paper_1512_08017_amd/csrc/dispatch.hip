// Degree dispatch of the launchers, and the kernels that do not depend on the
// degree: the tile table and the sampled range.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launchers.hpp"

namespace lsefit {

// ---------------------------------------------------------------------------
// tile table of a batch, in two launches.  Pass A: one thread per fit counts
// its tiles (ceil(L / tile), every point of every fit is in exactly one tile),
// sets its plan status (bad degree or segment -> INVALID_ARG, fewer than m+1
// points -> SINGULAR), writes (c, s) (given, or from the first 8 and the last
// 8 points of its x, all of a shorter fit, loaded in one round), and
// scans the tile counts of its block.  Pass B adds the tile totals of the
// blocks before it and stores the number of tiles and the tile size after the
// last fit's entry.  Integer sums: the result does not depend on the order.
//
// A batch of at most kPlanFusedBlocks blocks with a power-of-two tile takes
// one launch (FUSED): every block also counts the tiles of all the fits before
// its own (at most NPREV per thread, the number of blocks before the last one
// rounded up to 2^k - 1, a shift each, loaded
// together with its own fits' data) and writes the final table itself.
// ---------------------------------------------------------------------------
constexpr int kRangeBatchSamples = 16;
constexpr int kPlanFusedBlocks = 32;
constexpr int kPlanWaves = kPlanThreads / kWave;

template <typename In, bool FUSED, int NPREV>
__global__ void __launch_bounds__(kPlanThreads)
    k_plan_count(FitDesc d, Work w, int maxM, int64_t tile, int range_given, double c, double s,
                 const In* __restrict__ x, int64_t* __restrict__ block_tot, int tile_shift) {
    const KernelClock kclock_(w.clock);
    const int tid = threadIdx.x;
    const int64_t f = (int64_t)blockIdx.x * kPlanThreads + tid;
    const int rl = rec_len(maxM);
    // this thread's fit; a thread past the last fit loads the last one and
    // drops it, so that no load sits behind a branch of its own
    const int64_t fc = f < d.batch ? f : d.batch - 1;
    const int64_t lo = fit_lo(d, fc);
    const int64_t L = fit_hi(d, fc) - lo;
    const int m = fit_deg(d, fc);
    // FUSED: the tiles of fits tid, tid + 256, ... below this block's first fit;
    // a thread past the end reads the last such fit again and drops it.  A
    // block with fits before it belongs to a batch, which has offsets: read
    // directly (not through the null check of fit_lo / fit_hi), the two
    // offsets of a fit come in one 16-byte load, half the load instructions
    int64_t prev = 0;
    if constexpr (FUSED) {
        const int64_t nprev = (int64_t)blockIdx.x * kPlanThreads;
        if (nprev > 0) {
#pragma unroll
            for (int i = 0; i < NPREV; ++i) {
                const int64_t j = tid + (int64_t)i * kPlanThreads;
                const int64_t jc = j < nprev ? j : nprev - 1;
                const int64_t Lj = d.offsets[jc + 1] - d.offsets[jc];
                const int64_t t = Lj <= 0 ? 0 : (Lj + tile - 1) >> tile_shift;
                prev += j < nprev ? t : 0;
            }
        }
    }
    double cc = c, ss = s;
    if (!range_given) {
        // the first and the last kRangeBatchSamples / 2 points (all of a
        // shorter fit, whose last point is read again in place of the missing
        // ones): two cache lines per fit, the exact extent of sorted data, and
        // one round of loads
        constexpr int H = kRangeBatchSamples / 2;
        double v[kRangeBatchSamples];
        if (L > 0) {
#pragma unroll
            for (int i = 0; i < kRangeBatchSamples; ++i) {
                const int64_t k = L <= kRangeBatchSamples ? (i < L ? i : L - 1)
                                                          : (i < H ? i : L - kRangeBatchSamples + i);
                v[i] = (double)x[lo + k];
            }
        } else {
#pragma unroll
            for (int i = 0; i < kRangeBatchSamples; ++i) v[i] = NAN;
        }
        double mn = INFINITY, mx = -INFINITY;
#pragma unroll
        for (int i = 0; i < kRangeBatchSamples; ++i) {
            if (isfinite(v[i])) {
                mn = fmin(mn, v[i]);
                mx = fmax(mx, v[i]);
            }
        }
        snap_range(mn, mx, &cc, &ss);
    }
    int64_t tiles = 0;
    if (f < d.batch) {
        tiles = L <= 0 ? 0 : (L + tile - 1) / tile;
        int st = LSEFIT_OK;
        if (m < 1 || m > maxM || L < 0) st = LSEFIT_ERR_INVALID_ARG;
        else if (L < m + 1) st = LSEFIT_ERR_SINGULAR;
        w.pstatus[f] = st;
        w.rec[f * rl + 0] = cc;
        w.rec[f * rl + 1] = ss;
    }
    // inclusive scan of the tile counts within the wave, then the wave totals
    // (and the FUSED earlier-fit counts, summed) meet in LDS
    int64_t incl = tiles;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t v = __shfl_up(incl, off, kWave);
        incl += lane_id() >= off ? v : 0;
    }
    if constexpr (FUSED) {
#pragma unroll
        for (int off = kWave / 2; off >= 1; off >>= 1) prev += __shfl_xor(prev, off, kWave);
    }
    __shared__ int64_t wtot[kPlanWaves], wprev[FUSED ? kPlanWaves : 1];
    const int wv = tid / kWave;
    if (lane_id() == kWave - 1) wtot[wv] = incl;
    if constexpr (FUSED) {
        if (lane_id() == 0) wprev[wv] = prev;
    }
    __syncthreads();
    int64_t before = 0, total = 0, base = 0;
#pragma unroll
    for (int i = 0; i < kPlanWaves; ++i) {
        before += i < wv ? wtot[i] : 0;
        total += wtot[i];
        if constexpr (FUSED) base += wprev[i];
    }
    const int64_t start = before + incl - tiles;   // tiles of this block's fits before f
    if constexpr (FUSED) {
        if (f < d.batch) w.tile_start[f] = base + start;
        if (blockIdx.x == gridDim.x - 1 && tid == kPlanThreads - 1) {
            w.tile_start[d.batch] = base + total;
            w.tile_start[d.batch + 1] = tile;   // the table's own tile size, for every later pass over it
        }
    } else {
        if (f < d.batch) w.tile_start[f] = start;
        if (tid == kPlanThreads - 1) block_tot[blockIdx.x] = total;
    }
}

__global__ void __launch_bounds__(kPlanThreads)
    k_plan_offsets(FitDesc d, Work w, const int64_t* __restrict__ block_tot, int64_t nblocks, int64_t tile) {
    const KernelClock kclock_(w.clock);
    const int tid = threadIdx.x;
    const int64_t f = (int64_t)blockIdx.x * kPlanThreads + tid;
    // this thread's entry, loaded with the block totals
    const int64_t local = f < d.batch ? w.tile_start[f] : 0;
    int64_t part = 0;
    for (int64_t b = tid; b < blockIdx.x; b += kPlanThreads) part += block_tot[b];
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) part += __shfl_xor(part, off, kWave);
    __shared__ int64_t wsum[kPlanWaves];
    if (lane_id() == 0) wsum[tid / kWave] = part;
    __syncthreads();
    int64_t base = 0;
#pragma unroll
    for (int i = 0; i < kPlanWaves; ++i) base += wsum[i];
    if (f < d.batch) w.tile_start[f] = base + local;
    if (blockIdx.x == nblocks - 1 && tid == 0) {
        w.tile_start[d.batch] = base + block_tot[blockIdx.x];
        w.tile_start[d.batch + 1] = tile;   // the table's own tile size, for every later pass over it
    }
}

// ---------------------------------------------------------------------------
// read-bandwidth probe (measurement only; no fitting arithmetic): streams x and
// y with 16-byte loads and folds them into one float per block so that the
// loads stay live.  PATTERN 0: each wave reads one contiguous share, as the
// power-sum kernel of a single fit does; PATTERN 1: the grid strides over the
// 16-byte vectors.  NT: non-temporal loads.
// ---------------------------------------------------------------------------
template <bool NT, typename V>
__device__ inline V probe_load(const V* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// first vector, end and stride of one lane under each load pattern (pattern 2:
// each block reads one contiguous share and its waves take turns over the
// 16-byte vectors of that share)
template <int PATTERN>
__device__ inline void probe_range(int64_t nvec, int64_t W, int64_t wave, int lane, int64_t* j, int64_t* end,
                                   int64_t* step) {
    if (PATTERN == 0) {
        *j = wave * nvec / W + lane;
        *end = (wave + 1) * nvec / W;
        *step = kWave;
    } else if (PATTERN == 1) {
        *j = wave * kWave + lane;
        *end = nvec;
        *step = W * kWave;
    } else {
        const int64_t nb = gridDim.x, wpb = blockDim.x / kWave;
        *j = (int64_t)blockIdx.x * nvec / nb + (int64_t)wave_id_in_block() * kWave + lane;
        *end = ((int64_t)blockIdx.x + 1) * nvec / nb;
        *step = wpb * kWave;
    }
}

template <int U, int PATTERN, bool NT>
__global__ void __launch_bounds__(256)
    k_read_probe(const float* __restrict__ x, const float* __restrict__ y, int64_t nvec, int64_t W,
                 float* __restrict__ out, KClock kc) {
    const KernelClock kclock_(kc.slot);
    typedef float V __attribute__((ext_vector_type(4)));
    const V* xv = reinterpret_cast<const V*>(x);
    const V* yv = reinterpret_cast<const V*>(y);
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    float acc = 0.0f;
    int64_t j, end, step;
    probe_range<PATTERN>(nvec, W, wave, lane, &j, &end, &step);
    for (; j + (int64_t)(U - 1) * step < end; j += (int64_t)U * step) {
        V a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = probe_load<NT>(xv + j + u * step);
            b[u] = probe_load<NT>(yv + j + u * step);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (a[u].x + a[u].y) + (a[u].z + a[u].w) + (b[u].x + b[u].y) + (b[u].z + b[u].w);
    }
    for (; j < end; j += step) {
        const V a = probe_load<NT>(xv + j), b = probe_load<NT>(yv + j);
        acc += (a.x + a.y) + (a.z + a.w) + (b.x + b.y) + (b.z + b.w);
    }
    acc = (float)wave_sum((double)acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

hipError_t launch_read_probe(const float* x, const float* y, int64_t nvec, const Launch& L, int pattern, bool nt,
                             float* out, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
#define LSEFIT_PROBE(UU, PP, NN)                                                                                  \
    if (L.unroll == UU && pattern == PP && nt == NN) {                                                            \
        launch_timed((k_read_probe<UU, PP, NN>), grid, block, st, x, y, nvec, L.waves, out, KClock{}); \
        return hipGetLastError();                                                                                 \
    }
    LSEFIT_PROBE(1, 0, false) LSEFIT_PROBE(2, 0, false) LSEFIT_PROBE(4, 0, false)
    LSEFIT_PROBE(1, 0, true) LSEFIT_PROBE(2, 0, true) LSEFIT_PROBE(4, 0, true)
    LSEFIT_PROBE(1, 1, false) LSEFIT_PROBE(2, 1, false) LSEFIT_PROBE(4, 1, false)
    LSEFIT_PROBE(1, 1, true) LSEFIT_PROBE(2, 1, true) LSEFIT_PROBE(4, 1, true)
    LSEFIT_PROBE(1, 2, false) LSEFIT_PROBE(2, 2, false) LSEFIT_PROBE(4, 2, false)
    LSEFIT_PROBE(1, 2, true) LSEFIT_PROBE(2, 2, true) LSEFIT_PROBE(4, 2, true)
#undef LSEFIT_PROBE
    return hipErrorInvalidValue;
}

// copy probe (measurement only): reads x and y and writes them to ox and oy
// with 16-byte loads and stores, the traffic of the adjoint pass (8 bytes read
// and 8 bytes written per float32 point); load patterns as the read probe
template <int U, int PATTERN, bool NT>
__global__ void __launch_bounds__(256)
    k_copy_probe(const float* __restrict__ x, const float* __restrict__ y, float* __restrict__ ox,
                 float* __restrict__ oy, int64_t nvec, int64_t W, KClock kc) {
    const KernelClock kclock_(kc.slot);
    typedef float V __attribute__((ext_vector_type(4)));
    const V* xv = reinterpret_cast<const V*>(x);
    const V* yv = reinterpret_cast<const V*>(y);
    V* oxv = reinterpret_cast<V*>(ox);
    V* oyv = reinterpret_cast<V*>(oy);
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    int64_t j, end, step;
    probe_range<PATTERN>(nvec, W, wave, lane, &j, &end, &step);
    auto store = [](V* p, const V& v) {
        if constexpr (NT) __builtin_nontemporal_store(v, p);
        else *p = v;
    };
    for (; j + (int64_t)(U - 1) * step < end; j += (int64_t)U * step) {
        V a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = probe_load<NT>(xv + j + u * step);
            b[u] = probe_load<NT>(yv + j + u * step);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            store(oxv + j + u * step, a[u]);
            store(oyv + j + u * step, b[u]);
        }
    }
    for (; j < end; j += step) {
        store(oxv + j, probe_load<NT>(xv + j));
        store(oyv + j, probe_load<NT>(yv + j));
    }
}

hipError_t launch_copy_probe(const float* x, const float* y, float* ox, float* oy, int64_t nvec, const Launch& L,
                             int pattern, bool nt, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
#define LSEFIT_PROBE(UU, PP, NN)                                                                 \
    if (L.unroll == UU && pattern == PP && nt == NN) {                                           \
        launch_timed((k_copy_probe<UU, PP, NN>), grid, block, st, x, y, ox, oy, nvec, L.waves, KClock{}); \
        return hipGetLastError();                                                                \
    }
    LSEFIT_PROBE(1, 0, false) LSEFIT_PROBE(2, 0, false) LSEFIT_PROBE(4, 0, false)
    LSEFIT_PROBE(1, 0, true) LSEFIT_PROBE(2, 0, true) LSEFIT_PROBE(4, 0, true)
    LSEFIT_PROBE(1, 1, false) LSEFIT_PROBE(2, 1, false) LSEFIT_PROBE(4, 1, false)
    LSEFIT_PROBE(1, 1, true) LSEFIT_PROBE(2, 1, true) LSEFIT_PROBE(4, 1, true)
    LSEFIT_PROBE(1, 2, false) LSEFIT_PROBE(2, 2, false) LSEFIT_PROBE(4, 2, false)
    LSEFIT_PROBE(1, 2, true) LSEFIT_PROBE(2, 2, true) LSEFIT_PROBE(4, 2, true)
#undef LSEFIT_PROBE
    return hipErrorInvalidValue;
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

int64_t plan_blocks(int64_t batch) { return (batch + kPlanThreads - 1) / kPlanThreads; }

hipError_t launch_plan(const FitDesc& d, const Work& w, int maxM, int64_t tile, bool range_given, double c,
                       double s, int dtype, const void* x, int64_t* block_tot, hipStream_t st) {
    const int64_t nb = plan_blocks(d.batch);
    const int rg = range_given ? 1 : 0;
    int shift = 0;
    while (shift < 62 && (int64_t(1) << shift) < tile) ++shift;
    if (nb <= kPlanFusedBlocks && (int64_t(1) << shift) == tile) {
        auto fused = [&]<int NPREV>() {
            if (dtype == LSEFIT_F32)
                launch_timed(k_plan_count<float, true, NPREV>, dim3(nb), dim3(kPlanThreads), st, d, w, maxM, tile, rg,
                             c, s, (const float*)x, block_tot, shift);
            else
                launch_timed(k_plan_count<double, true, NPREV>, dim3(nb), dim3(kPlanThreads), st, d, w, maxM, tile,
                             rg, c, s, (const double*)x, block_tot, shift);
        };
        static_assert(kPlanFusedBlocks == 32, "one instantiation per power of two of earlier blocks");
        if (nb <= 1) fused.template operator()<0>();
        else if (nb <= 4) fused.template operator()<3>();
        else if (nb <= 8) fused.template operator()<7>();
        else if (nb <= 16) fused.template operator()<15>();
        else fused.template operator()<31>();
        return hipGetLastError();
    }
    if (dtype == LSEFIT_F32)
        launch_timed(k_plan_count<float, false, 0>, dim3(nb), dim3(kPlanThreads), st, d, w, maxM, tile, rg, c, s,
                     (const float*)x, block_tot, 0);
    else
        launch_timed(k_plan_count<double, false, 0>, dim3(nb), dim3(kPlanThreads), st, d, w, maxM, tile, rg, c, s,
                     (const double*)x, block_tot, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_offsets, dim3(nb), dim3(kPlanThreads), 0, st, d, w, block_tot, nb, tile);
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

hipError_t launch_solve_moments(const double* moments, const Work& w, int m, int maxM, int solver, double* coef,
                                int32_t* status, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::solve_moments(moments, w, m, solver, coef, status, st));
}

hipError_t launch_refine(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                         const Launch& L, int mis, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::refine(d, w, dtype, x, y, L, mis, st));
}

hipError_t launch_adjoint(const FitDesc& d, const Work& w, int maxM, int solver, int dtype, const void* x,
                          const void* y, const double* grad_coef, int32_t coef_stride, void* gx, void* gy,
                          const Launch& L, int mis, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::adjoint(d, w, solver, dtype, x, y, grad_coef, coef_stride, gx, gy,
                                                           L, mis, st));
}

hipError_t launch_residual(const FitDesc& d, const Work& w, int maxM, int dtype, const void* x, const void* y,
                           void* resid, const Launch& L, int mis, hipStream_t st) {
    LSEFIT_SWITCH_MAXM(maxM, return Launchers<MM>::residual(d, w, dtype, x, y, resid, L, mis, st));
}

}  // namespace lsefit
