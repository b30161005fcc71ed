// Chebyshev-basis fits (degree up to LSEFIT_MAX_DEGREE_CHEBYSHEV).
//
// The least-squares problem of Sec. II written in the basis T_0..T_m of
// Chebyshev polynomials of t = (x - c)/s instead of powers of x (Sec. V leaves
// higher-order polynomials as further work; the monomial normal matrix loses
// all precision there).  Since T_j T_k = (T_(j+k) + T_|j-k|) / 2, the Gram
// matrix is G_jk = (C_(j+k) + C_|j-k|) / 2 with C_k = sum_i T_k(t_i), C_0 = n,
// and the right side is D_j = sum_i y_i T_j(t_i); G c = D gives the Chebyshev
// coefficients c.  Float64 accumulation only.
//
// Per point the pass forms T_2..T_m by the three-term recurrence
// T_(k+1) = 2 t T_k - T_(k-1) and accumulates C_1..C_m, D_0..D_m and
// E_j = sum_i T_m(t_i) T_j(t_i) (j = 1..m); the upper sums follow from the same
// identity, C_(m+j) = 2 E_j - C_(m-j).  That is 4m+1 float64 operations per
// point instead of the 5m+2 of running the recurrence up to T_2m: the pass
// runs the recurrence on V_k = 2 T_k, V_(k+1) = (2t) V_k - V_(k-1) with
// V_1 = 2t and V_2 = (2t)^2 - 2, which needs 2t alone (one FMA from x) and
// is exactly twice T_k in floating point too (scaling by two commutes with
// rounding), so the sums come out exact multiples 2 or 4 of the T sums and
// are scaled back once per wave.
#include "kernels_impl.hpp"

namespace lsefit {

constexpr int kChebMax = LSEFIT_MAX_DEGREE_CHEBYSHEV;

// partial sums of one lane: [2 C_1..2 C_M, 4 E_1..4 E_M, D_0, 2 D_1..2 D_M]
// (nacc(M) values; cheb_wave_sums scales them back)
template <int M>
struct AccCheb {
    double C[M];       // sum V_1..V_M
    double E[M];       // sum V_M V_1..V_M V_M
    double D[M + 1];   // sum y, sum y V_1..y V_M
    double two_inv_s, two_nc;
    __device__ inline void init(double c, double is) {
#pragma unroll
        for (int k = 0; k < M; ++k) C[k] = E[k] = 0.0;
#pragma unroll
        for (int j = 0; j <= M; ++j) D[j] = 0.0;
        two_inv_s = 2.0 * is;
        two_nc = -2.0 * (c * is);
    }
    __device__ inline void point(double xv, double yv) {
        const double t2 = fma(xv, two_inv_s, two_nc);  // 2t
        double V[M + 1];
        V[1] = t2;
        if constexpr (M >= 2) V[2] = fma(t2, t2, -2.0);
#pragma unroll
        for (int k = 3; k <= M; ++k) V[k] = fma(t2, V[k - 1], -V[k - 2]);
        D[0] += yv;
#pragma unroll
        for (int k = 1; k <= M; ++k) {
            C[k - 1] += V[k];
            D[k] = fma(yv, V[k], D[k]);
            E[k - 1] = fma(V[M], V[k], E[k - 1]);
        }
    }
    template <typename V, int VW>
    __device__ inline void vec(const V& xv, const V& yv) {
#pragma unroll
        for (int e = 0; e < VW; ++e) point((double)xv[e], (double)yv[e]);
    }
    __device__ inline void scalar(double xv, double yv) { point(xv, yv); }
};

// ---------------------------------------------------------------------------
// range of the basis: t = (x - c)/s maps the exact extent [lo, hi] of the
// fit's finite x onto [-1, 1], the interval on which the T_k are orthogonal
// and bounded by 1 (a power-of-two scale could leave t on [-1/2, 1/2], where
// their Gram matrix is nearly singular at high degree)
// ---------------------------------------------------------------------------
__device__ inline void cheb_range(double lo, double hi, double* c, double* s) {
    if (!(lo <= hi)) {  // no finite x
        *c = 0.0;
        *s = 1.0;
        return;
    }
    const double half = 0.5 * hi - 0.5 * lo;
    *c = 0.5 * hi + 0.5 * lo;
    *s = half > 0.0 ? half : 1.0;
}

template <typename In>
struct MinMax {
    In lo, hi;
    __device__ inline MinMax() : lo(INFINITY), hi(-INFINITY) {}
    __device__ inline void add(In v) {
        if (isfinite(v)) {
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    template <typename V, int VW>
    __device__ inline void vec(const V& v) {
#pragma unroll
        for (int e = 0; e < VW; ++e) add(v[e]);
    }
};

// x only, the sweep of the single-fit streaming pass (grid stride over 16-byte vectors)
template <typename In>
__device__ inline void minmax_strided(const In* __restrict__ x, int64_t n, int mis, int64_t gwave, int64_t W,
                                      MinMax<In>& r) {
    constexpr int VW = VecOf<In>::W;
    constexpr int U = 4;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    const int64_t step = W * kWave;
    if (mis >= 0) {
        int64_t a = (VW - mis) % VW;
        if (a > n) a = n;
        const int64_t nv = (n - a) / VW;
        const int64_t b = a + nv * VW;
        if (gwave == 0 && lane < a) r.add(ld_scalar(x + lane));
        const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
        int64_t j = gwave * kWave + lane;
        for (; j + (int64_t)(U - 1) * step < nv; j += (int64_t)U * step) {
            V v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ld_stream(xv + j + u * step);
#pragma unroll
            for (int u = 0; u < U; ++u) r.template vec<V, VW>(v[u]);
        }
        for (; j < nv; j += step) r.template vec<V, VW>(ld_stream(xv + j));
        if (gwave == 0 && lane < n - b) r.add(ld_scalar(x + b + lane));
    } else {
        for (int64_t i = gwave * kWave + lane; i < n; i += step) r.add(ld_scalar(x + i));
    }
}

// x only, one wave over points [lo, hi) of a batch; U vectors per lane are
// loaded before any is used (one array: four give a wave the bytes in flight
// that two of x and y give the power-sum pass)
template <typename In>
__device__ inline void minmax_segment(const In* __restrict__ x, int64_t lo, int64_t hi, int mis, MinMax<In>& r) {
    constexpr int VW = VecOf<In>::W;
    constexpr int U = 4;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    if (mis >= 0) {
        int64_t a = lo + (int64_t)((VW - (int)((lo + mis) % VW)) % VW);
        if (a > hi) a = hi;
        const int64_t nv = (hi - a) / VW;
        const int64_t b = a + nv * VW;
        if (lane < a - lo) r.add(ld_scalar(x + lo + lane));
        const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
        int64_t j = lane;
        for (; j + (int64_t)(U - 1) * kWave < nv; j += (int64_t)U * kWave) {
            V v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ld_stream(xv + j + u * kWave);
#pragma unroll
            for (int u = 0; u < U; ++u) r.template vec<V, VW>(v[u]);
        }
        for (; j < nv; j += kWave) r.template vec<V, VW>(ld_stream(xv + j));
        if (lane < hi - b) r.add(ld_scalar(x + b + lane));
    } else {
        for (int64_t i = lo + lane; i < hi; i += kWave) r.add(ld_scalar(x + i));
    }
}

// single fit: one (min, max) pair per block into part[2 blockIdx.x ..]
template <typename In>
__global__ void __launch_bounds__(256)
    k_range_cheb_single(FitDesc d, Work w, const In* __restrict__ x, int64_t W, int mis) {
    const KernelClock kclock_(w.clock);
    __shared__ double slo[4], shi[4];
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    MinMax<In> r;
    minmax_strided(x, d.n_single, mis, wave, W, r);
    const double lo = wave_min((double)r.lo), hi = wave_max((double)r.hi);
    if (lane_id() == 0) {
        slo[wave_id_in_block()] = lo;
        shi[wave_id_in_block()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = slo[0], b = shi[0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) {
            a = fmin(a, slo[i]);
            b = fmax(b, shi[i]);
        }
        w.part[2 * (int64_t)blockIdx.x] = a;
        w.part[2 * (int64_t)blockIdx.x + 1] = b;
    }
}

// single fit: fold the G block pairs, set (c, s) and the fit's status
__global__ void __launch_bounds__(256) k_range_fold_single(Work w, int64_t G) {
    const KernelClock kclock_(w.clock);
    __shared__ double slo[4], shi[4];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
        lo = fmin(lo, w.part[2 * g]);
        hi = fmax(hi, w.part[2 * g + 1]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane_id() == 0) {
        slo[wave_id_in_block()] = lo;
        shi[wave_id_in_block()] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) {
            lo = fmin(lo, slo[i]);
            hi = fmax(hi, shi[i]);
        }
        cheb_range(lo, hi, &w.rec[0], &w.rec[1]);
        w.pstatus[0] = LSEFIT_OK;
    }
}

// batch: one (min, max) pair per (wave, fit) slot
template <typename In>
__global__ void __launch_bounds__(256)
    k_range_cheb_batch(FitDesc d, Work w, const In* __restrict__ x, int64_t W, int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rec_len(maxm), wave, W,
                        [&](int64_t, int64_t lo, int64_t hi, int64_t slot, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) return;
        MinMax<In> r;
        minmax_segment(x, lo, hi, mis, r);
        const double a = wave_min((double)r.lo), b = wave_max((double)r.hi);
        if (lane_id() == 0) {
            w.part[2 * slot] = a;
            w.part[2 * slot + 1] = b;
        }
    });
}

// batch: one thread per fit folds the slots of the waves that streamed it
__global__ void __launch_bounds__(256) k_range_fold_batch(FitDesc d, Work w, int64_t W, int maxm) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch || w.pstatus[f] != LSEFIT_OK) return;
    const int64_t NT = w.tile_start[d.batch];
    const int64_t w0 = wave_of_tile(w.tile_start[f], NT, W);
    const int64_t w1 = wave_of_tile(w.tile_start[f + 1] - 1, NT, W);
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t wv = w0; wv <= w1; ++wv) {
        if (!wave_owns_tiles(wv, NT, W)) continue;
        lo = fmin(lo, w.part[2 * (wv + f)]);
        hi = fmax(hi, w.part[2 * (wv + f) + 1]);
    }
    double* r = w.rec + f * rec_len(maxm);
    cheb_range(lo, hi, &r[0], &r[1]);
}

// the waves of a block add their sums in order; one partial per block, stored
// sum-major (sum k of block g at part[k G + g], G blocks)
template <int K>
__device__ inline void cheb_block_partial(const Work& w, const double (&v)[K]) {
    __shared__ double sh[4][K];
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[wave_id_in_block()][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int nw = blockDim.x / kWave;
        double acc = sh[0][threadIdx.x];
        for (int i = 1; i < nw; ++i) acc += sh[i][threadIdx.x];
        w.part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = acc;
    }
}

// the wave's [C_1..C_M, E_1..E_M, D_0..D_M] (the V = 2T sums times 1/2 or 1/4: exact)
template <int M>
__device__ inline void cheb_wave_sums(const AccCheb<M>& acc, double (&v)[nacc(M)]) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
        v[k] = 0.5 * wave_sum(acc.C[k]);
        v[M + k] = 0.25 * wave_sum(acc.E[k]);
    }
    v[2 * M] = wave_sum(acc.D[0]);
#pragma unroll
    for (int j = 1; j <= M; ++j) v[2 * M + j] = 0.5 * wave_sum(acc.D[j]);
}

// the single-fit sweep of stream_strided (same points, same order per lane)
// with two register sets of U vectors per array that take turns: while one
// round is accumulated the next is in flight in the other set, so no loaded
// vector is ever copied (at high degree the pass is bound by float64 issue,
// and the copies of a single prefetch buffer cost about 3 VALU instructions
// per point)
template <int U, typename In, class Acc>
__device__ inline void stream_strided_pp(const In* __restrict__ x, const In* __restrict__ y, int64_t n, int mis,
                                         int64_t gwave, int64_t W, Acc& acc) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    const int64_t step = W * kWave;
    if (mis < 0) {
        for (int64_t i = gwave * kWave + lane; i < n; i += step) acc.scalar(ld_scalar(x + i), ld_scalar(y + i));
        return;
    }
    int64_t a = (VW - mis) % VW;
    if (a > n) a = n;
    const int64_t nv = (n - a) / VW;
    const int64_t b = a + nv * VW;
    if (gwave == 0 && lane < a) acc.scalar(ld_scalar(x + lane), ld_scalar(y + lane));
    const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
    const V* __restrict__ yv = reinterpret_cast<const V*>(y + a);
    const int64_t span = (int64_t)(U - 1) * step;
    const int64_t round = (int64_t)U * step;
    // the scheduling barrier keeps the loads where they are issued: without
    // it the scheduler moves them next to their first use (fewer live
    // registers, but every round then waits on its own loads)
    auto load = [&](V (&xs)[U], V (&ys)[U], int64_t j0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xs[u] = ld_stream(xv + j0 + u * step);
            ys[u] = ld_stream(yv + j0 + u * step);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto use = [&](const V (&xs)[U], const V (&ys)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc.template vec<V, VW>(xs[u], ys[u]);
    };
    // R = the rounds this lane takes (U vectors per array, all in bounds); the
    // loop does two per pass, so that both register sets are loaded and used
    // in one straight block, and loads the pass after next's first round
    // unconditionally (re-reading the current one, in bounds, when there is
    // none: behind a branch, the path without them would make the compiler
    // wait for the fresh loads too)
    int64_t j = gwave * kWave + lane;
    const int64_t R = j + span < nv ? (nv - 1 - span - j) / round + 1 : 0;
    if (R > 0) {
        V xa[U], ya[U], xb[U], yb[U];
        load(xa, ya, j);
        for (int64_t r = 2; r <= R; r += 2) {
            load(xb, yb, j + round);
            use(xa, ya);
            load(xa, ya, r < R ? j + 2 * round : j);
            use(xb, yb);
            j += 2 * round;
        }
        if (R & 1) {
            use(xa, ya);
            j += round;
        }
    }
    for (; j < nv; j += step) acc.template vec<V, VW>(ld_stream(xv + j), ld_stream(yv + j));
    if (gwave == 0 && lane < n - b) acc.scalar(ld_scalar(x + b + lane), ld_scalar(y + b + lane));
}

// single fit of degree M: grid-stride sweep, one partial per block
template <typename In, int U, int M>
__global__ void __launch_bounds__(256)
    k_moments_cheb_single(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W, int mis,
                          RangeArg ra) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    double c, inv_s;
    if (ra.mode == kRangeFromRecord) {
        c = w.rec[0];
        inv_s = 1.0 / w.rec[1];
    } else {
        single_range(d, w, x, ra, &c, &inv_s);
    }
    AccCheb<M> acc;
    acc.init(c, inv_s);
    stream_strided_pp<U>(x, y, d.n_single, mis, wave, W, acc);
    double v[nacc(M)];
    cheb_wave_sums(acc, v);
    cheb_block_partial<nacc(M)>(w, v);
}

// batch, degrees up to MAXC <= maxm: each wave walks its tiles, one partial
// slot per (wave, fit) segment
template <typename In, int U, int MAXC>
__global__ void __launch_bounds__(256)
    k_moments_cheb_batch(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y,
                         int64_t W, int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    const int stride = nacc(maxm);
    const int rl = rec_len(maxm);
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rl, wave, W,
                        [&](int64_t, int64_t lo, int64_t hi, int64_t slot, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) return;
        const double c = mt.c;
        const double inv_s = 1.0 / mt.s;
        double* __restrict__ out = w.part + slot * stride;
        auto body = [&]<int M>() {
            AccCheb<M> acc;
            acc.init(c, inv_s);
            stream_segment<U>(x, y, lo, hi, mis, acc);
            double v[nacc(M)];
            cheb_wave_sums(acc, v);
            if (lane_id() == 0)
#pragma unroll
                for (int k = 0; k < nacc(M); ++k) out[k] = v[k];
        };
        dispatch_degree<MAXC>(mt.deg, body);
    });
}

// ---------------------------------------------------------------------------
// finishing a Chebyshev fit: one wave per fit.  The sums go to a per-wave LDS
// row [C_0..C_2m, D_0..D_m]; lane r < m+1 then holds row r of [G | D] in
// registers for the elimination, and the lanes share pivot rows and solved
// unknowns through readlane.
// ---------------------------------------------------------------------------
// S = this wave's LDS row [C_0..C_2m, D_0..D_m] of fit f (written and fenced by
// the caller): assemble, solve, write the Chebyshev coefficients (then, with
// write_b, the x-basis coefficients after them; else c and s after them when
// the stride leaves room), the record's b and the status
template <int M>
__device__ __forceinline__ void cheb_solve_wave(const Work& w, int64_t f, int maxm, double c0, double s0, const double* S,
                                       const Finish& fz) {
    constexpr int N = M + 1;
    const int lane = lane_id();
    const bool mine = lane < N;
    double row[M + 2];
    bool finite = true;
#pragma unroll
    for (int c = 0; c <= N; ++c) row[c] = 0.0;
    if (mine) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
            const int dk = lane > c ? lane - c : c - lane;
            row[c] = 0.5 * (S[lane + c] + S[dk]);
            finite = finite && isfinite(row[c]);
        }
        row[N] = S[2 * M + 1 + lane];
        finite = finite && isfinite(row[N]);
    }
    double x = 0.0;
    int st = __ballot(!finite) ? LSEFIT_ERR_NONFINITE
                               : (fz.solver == LSEFIT_SOLVER_CHOLESKY ? wave_cholesky<M>(row, x)
                                                                      : wave_gepp<M>(row, x));
    if (st == LSEFIT_OK && __ballot(mine && !isfinite(x))) st = LSEFIT_ERR_NONFINITE;
    double* r = w.rec + f * rec_len(maxm);
    double* out = fz.coef + f * (int64_t)fz.coef_stride;
    if (st != LSEFIT_OK) {
        if (mine) {
            out[lane] = NAN;
            r[rec_b(maxm) + lane] = NAN;
            if (fz.write_b) out[N + lane] = NAN;
        }
    } else {
        if (mine) {
            out[lane] = x;
            r[rec_b(maxm) + lane] = x;
        }
        if (fz.write_b) {
            // Chebyshev -> powers of t (lane k holds coefficient k of T_(j-1), T_j)
            double Tp = lane == 0 ? 1.0 : 0.0;
            double Tc = lane == 1 ? 1.0 : 0.0;
            double b = bcast(x, 0) * Tp + (N > 1 ? bcast(x, 1) * Tc : 0.0);
#pragma unroll
            for (int j = 1; j + 1 < N; ++j) {
                const double up = __shfl_up(Tc, 1, kWave);
                const double Tn = (lane > 0 ? 2.0 * up : 0.0) - Tp;
                b += bcast(x, j + 1) * Tn;
                Tp = Tc;
                Tc = Tn;
            }
            // powers of t -> powers of x: a_k = sum_(j>=k) b_j C(j,k) (-c)^(j-k) s^-j
            const double inv_s = 1.0 / s0;
            double acc = 0.0, binom = 1.0, cpow = 1.0, spow = 1.0;
            for (int i = 0; i < lane && i < N; ++i) spow *= inv_s;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const double bj = bcast(b, j);
                if (lane <= j) {
                    acc += bj * binom * cpow * spow;
                    binom = binom * (double)(j + 1) / (double)(j + 1 - lane);
                    cpow *= -c0;
                    spow *= inv_s;
                }
            }
            if (mine) out[N + lane] = acc;
        } else if (fz.coef_stride >= N + 2 && lane == 0) {
            out[N] = c0;
            out[N + 1] = s0;
        }
    }
    if (lane == 0) {
        w.pstatus[f] = st;
        if (fz.status) fz.status[f] = st;
    }
}

__device__ inline void cheb_fail(const FitDesc& d, const Work& w, int64_t f, int maxm, const Finish& fz, int st) {
    const int m = fit_deg(d, f);
    const bool valid = m >= 1 && m <= maxm;
    const int n = valid ? m + 1 : fz.coef_stride;
    double* out = fz.coef + f * (int64_t)fz.coef_stride;
    for (int k = 0; k < n; ++k) out[k] = NAN;
    if (fz.write_b && valid)
        for (int k = 0; k < n; ++k) out[n + k] = NAN;
    fz.status[f] = st;
}

// the summed partials v = [C_1..C_M, E_1..E_M, D_0..D_M] of fit f (uniform)
// -> S = [C_0..C_2M, D_0..D_M] in this wave's LDS row (C_(M+j) = 2 E_j - C_(M-j)),
// the record's sums and, if asked, moments_out; lane 0 writes
template <int M>
__device__ __forceinline__ void cheb_store_sums(const Work& w, int64_t f, int maxm, double n, const double (&v)[nacc(M)],
                                       const Finish& fz, double* S) {
    if (lane_id() == 0) {
        S[0] = n;
#pragma unroll
        for (int k = 1; k <= M; ++k) S[k] = v[k - 1];
#pragma unroll
        for (int j = 1; j <= M; ++j) S[M + j] = 2.0 * v[M + j - 1] - S[M - j];
#pragma unroll
        for (int j = 0; j <= M; ++j) S[2 * M + 1 + j] = v[2 * M + j];
        double* r = w.rec + f * rec_len(maxm);
        for (int k = 0; k <= 2 * M; ++k) r[rec_S(maxm) + k] = S[k];
        for (int j = 0; j <= M; ++j) r[rec_T(maxm) + j] = S[2 * M + 1 + j];
        if (fz.moments_out) {
            fz.moments_out[0] = r[0];
            fz.moments_out[1] = r[1];
            for (int k = 0; k < 3 * M + 2; ++k) fz.moments_out[2 + k] = S[k];
        }
    }
    wave_lds_fence();
}

// Single fit of degree M: the finish block adds up the W block partials
// (block_sum_partials) and wave 0 finishes.  The fit's status and range are
// loaded at the start, with the partials; the partials are summed whatever the
// status and the status only decides what is written.
template <int M>
__global__ void __launch_bounds__(kFinishWaves * kWave)
    k_finish_cheb_single(FitDesc d, Work w, int64_t W, int maxm, Finish fz) {
    const KernelClock kclock_(w.clock);
    constexpr int K = nacc(M);
    __shared__ double sums[K];
    __shared__ double S[3 * M + 2];
    const int pst = w.pstatus[0];
    const double c = w.rec[0], s = w.rec[1];
    block_sum_partials<K>(w.part, W, sums);
    __syncthreads();
    if (wave_id_in_block() != 0) return;
    if (pst != LSEFIT_OK) {
        if (lane_id() == 0 && fz.mode != kMomentsOnly) cheb_fail(d, w, 0, maxm, fz, pst);
        return;
    }
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = sums[k];
    cheb_store_sums<M>(w, 0, maxm, (double)d.n_single, v, fz, S);
    if (fz.mode != kMomentsOnly) cheb_solve_wave<M>(w, 0, maxm, c, s, S, fz);
}

// Batch, degrees up to MAXC: wave v of block b finishes fits 4b + v,
// 4b + v + 4 gridDim.x, ..., summing the partial slots of the waves that
// streamed each.
template <int MAXC>
__global__ void __launch_bounds__(256) k_finish_cheb_batch(FitDesc d, Work w, int64_t W, int maxm, Finish fz) {
    const KernelClock kclock_(w.clock);
    __shared__ double S[4][3 * MAXC + 2];
    const int wid = wave_id_in_block(), lane = lane_id();
    const int stride = nacc(maxm);
    const int64_t NT = w.tile_start[d.batch];
    for (int64_t f = (int64_t)blockIdx.x * 4 + wid; f < d.batch; f += (int64_t)gridDim.x * 4) {
        const int pst = w.pstatus[f];
        if (pst != LSEFIT_OK) {
            if (lane == 0 && fz.mode != kMomentsOnly) cheb_fail(d, w, f, maxm, fz, pst);
            continue;
        }
        const int64_t w0 = wave_of_tile(w.tile_start[f], NT, W);
        const int64_t w1 = wave_of_tile(w.tile_start[f + 1] - 1, NT, W);
        auto body = [&]<int M>() {
            constexpr int K = nacc(M);
            double v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = 0.0;
            for (int64_t wv = w0 + lane; wv <= w1; wv += kWave) {
                if (!wave_owns_tiles(wv, NT, W)) continue;
                const double* p = w.part + (wv + f) * stride;
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] += p[k];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
            const double* r = w.rec + f * rec_len(maxm);
            cheb_store_sums<M>(w, f, maxm, (double)(fit_hi(d, f) - fit_lo(d, f)), v, fz, S[wid]);
            if (fz.mode != kMomentsOnly) cheb_solve_wave<M>(w, f, maxm, r[0], r[1], S[wid], fz);
            wave_lds_fence();
        };
        dispatch_degree<MAXC>(fit_deg(d, f), body);
    }
}

// Batch of degrees <= 4, one fit per thread: the thread sums its fit's partial
// slots in wave order, forms C_0..C_2M (C_(M+j) = 2 E_j - C_(M-j)) and the Gram
// system G_jk = (C_(j+k) + C_|j-k|)/2, G c = D, in its registers and solves it
// (matrix_gepp / matrix_cholesky: the pivot and singular rules of the wave
// solve).  At these degrees a wave per fit leaves most lanes idle and the
// batch's small solves in a long serial chain.  Coefficient output as
// cheb_solve_wave without write_b: c_0..c_M, then (c, s) when the stride holds
// them.
template <int MAXC>
__global__ void __launch_bounds__(256) k_finish_cheb_lane(FitDesc d, Work w, int64_t W, int maxm, Finish fz) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch) return;
    // the loads that depend on no other, issued together: status, degree,
    // tile range, point count and the range from the record
    const int pst = w.pstatus[f];
    const int deg = fit_deg(d, f);
    const int64_t NT = w.tile_start[d.batch];
    const int64_t ts = w.tile_start[f], te = w.tile_start[f + 1];
    const int64_t n = fit_hi(d, f) - fit_lo(d, f);
    double* r = w.rec + f * rec_len(maxm);
    const double rc = r[0], rs = r[1];
    if (pst != LSEFIT_OK) {
        if (fz.mode != kMomentsOnly) cheb_fail(d, w, f, maxm, fz, pst);
        return;
    }
    const int stride = nacc(maxm);
    const int64_t w0 = wave_of_tile(ts, NT, W);
    const int64_t w1 = wave_of_tile(te - 1, NT, W);
    // the sums of the largest degree's count, whatever this fit's degree (a
    // degree-m fit's sums are the first ones of its slots; an index past the
    // slot reads its last sum again), so that the loads sit outside the degree
    // switch and a wave of mixed degrees waits for its partial sums once
    constexpr int KMAX = nacc(MAXC);
    double all[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) all[k] = 0.0;
    for (int64_t wv = w0; wv <= w1; ++wv) {
        if (!wave_owns_tiles(wv, NT, W)) continue;
        const double* p = w.part + (wv + f) * stride;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) all[k] += p[k < stride ? k : stride - 1];
    }
    auto body = [&]<int M>() {
        constexpr int N = M + 1;
        constexpr int K = nacc(M);
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = all[k];
        double S[2 * M + 1], D[N];
        S[0] = (double)n;
#pragma unroll
        for (int k = 1; k <= M; ++k) S[k] = v[k - 1];
#pragma unroll
        for (int j = 1; j <= M; ++j) S[M + j] = 2.0 * v[M + j - 1] - S[M - j];
#pragma unroll
        for (int j = 0; j <= M; ++j) D[j] = v[2 * M + j];
#pragma unroll
        for (int k = 0; k <= 2 * M; ++k) r[rec_S(maxm) + k] = S[k];
#pragma unroll
        for (int j = 0; j <= M; ++j) r[rec_T(maxm) + j] = D[j];
        if (fz.mode == kMomentsOnly) return;
        double A[N][N + 1], X[1][N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
#pragma unroll
            for (int k = 0; k < N; ++k) A[j][k] = 0.5 * (S[j + k] + S[j > k ? j - k : k - j]);
            A[j][N] = D[j];
        }
        const int st = fz.solver == LSEFIT_SOLVER_CHOLESKY ? matrix_cholesky<N, 1>(A, X) : matrix_gepp<N, 1>(A, X);
        double* out = fz.coef + f * (int64_t)fz.coef_stride;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double c = st == LSEFIT_OK ? X[0][k] : NAN;
            out[k] = c;
            r[rec_b(maxm) + k] = c;
        }
        if (st == LSEFIT_OK && fz.coef_stride >= N + 2) {
            out[N] = rc;
            out[N + 1] = rs;
        }
        w.pstatus[f] = st;
        if (fz.status) fz.status[f] = st;
    };
    dispatch_degree<MAXC>(deg, body);
}

// ---------------------------------------------------------------------------
// residuals (Table V's errors at any degree): e = y - f(t) with
// f = sum_j c_j T_j(t) by Clenshaw's recurrence b_j = c_j + 2t b_(j+1) - b_(j+2),
// f = c_0 + t b_1 - b_2, in float64 in the t variable; the point loop is the
// monomial residual pass's.  Partial sums of e^2: one per block (single fit)
// or per (wave, fit) slot, one double each.
// ---------------------------------------------------------------------------
template <int M>
struct ChebResidPoint {
    double cf[M + 1];
    double inv_s, nc;
    __device__ inline void init(const double* r, int maxm) {
        inv_s = 1.0 / r[1];
        nc = -r[0] * inv_s;
#pragma unroll
        for (int j = 0; j <= M; ++j) cf[j] = r[rec_b(maxm) + j];
    }
    __device__ inline double err(double xv, double yv) const {
        const double t = fma(xv, inv_s, nc);
        const double t2 = t + t;
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int j = M; j >= 1; --j) {
            const double b0 = fma(t2, b1, cf[j] - b2);
            b2 = b1;
            b1 = b0;
        }
        return yv - fma(t, b1, cf[0] - b2);
    }
};

template <typename In, int U, int M>
__global__ void __launch_bounds__(256)
    k_residual_cheb_single(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y,
                           In* __restrict__ resid, int64_t W, int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    __shared__ double sh[4];
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    double acc = 0.0;
    if (w.pstatus[0] == LSEFIT_OK) {
        ChebResidPoint<M> P;
        P.init(w.rec, maxm);
        resid_points<ChebResidPoint<M>, In, true, U>(x, y, resid, 0, d.n_single, mis, wave, W, P, acc);
    } else if (resid) {
        for (int64_t i = wave * kWave + lane_id(); i < d.n_single; i += W * kWave) resid[i] = (In)NAN;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) sh[wave_id_in_block()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) t += sh[i];
        w.part[blockIdx.x] = t;
    }
}

template <typename In, int U, int MAXC>
__global__ void __launch_bounds__(256)
    k_residual_cheb_batch(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y,
                          In* __restrict__ resid, int64_t W, int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    const int rl = rec_len(maxm);
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rl, wave, W,
                        [&](int64_t f, int64_t lo, int64_t hi, int64_t slot, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) {
            if (resid)
                for (int64_t i = lo + lane_id(); i < hi; i += kWave) resid[i] = (In)NAN;
            return;
        }
        auto body = [&]<int M>() {
            ChebResidPoint<M> P;
            P.init(w.rec + f * rl, maxm);
            double acc = 0.0;
            resid_points<ChebResidPoint<M>, In, false, U>(x, y, resid, lo, hi, mis, 0, W, P, acc);
            acc = wave_sum(acc);
            if (lane_id() == 0) w.part[slot] = acc;
        };
        dispatch_degree<MAXC>(mt.deg, body);
    });
}

// sse of a single fit: one block sums the G block partials in a fixed order
__global__ void __launch_bounds__(256) k_sse_fold_single(Work w, int64_t G, double* __restrict__ sse) {
    const KernelClock kclock_(w.clock);
    __shared__ double sh[4];
    double t = 0.0;
    for (int64_t g = threadIdx.x; g < G; g += blockDim.x) t += w.part[g];
    t = wave_sum(t);
    if (lane_id() == 0) sh[wave_id_in_block()] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sh[0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) s += sh[i];
        sse[0] = w.pstatus[0] == LSEFIT_OK ? s : NAN;
    }
}

// sse of each fit of a batch: one thread per fit sums its slots in wave order
__global__ void __launch_bounds__(256) k_sse_fold_batch(FitDesc d, Work w, int64_t W, double* __restrict__ sse) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch) return;
    if (w.pstatus[f] != LSEFIT_OK) {
        sse[f] = NAN;
        return;
    }
    const int64_t NT = w.tile_start[d.batch];
    const int64_t w0 = wave_of_tile(w.tile_start[f], NT, W);
    const int64_t w1 = wave_of_tile(w.tile_start[f + 1] - 1, NT, W);
    double s = 0.0;
    for (int64_t wv = w0; wv <= w1; ++wv)
        if (wave_owns_tiles(wv, NT, W)) s += w.part[wv + f];
    sse[f] = s;
}

// one fit of degree M from caller-provided sums [c, s, C_0..C_2m, D_0..D_m], one wave
template <int M>
__global__ void __launch_bounds__(64) k_solve_cheb_moments(const double* __restrict__ mom, Work w, Finish fz) {
    const KernelClock kclock_(w.clock);
    __shared__ double S[3 * M + 2];
    const int lane = lane_id();
    const double c0 = mom[0], s0 = mom[1];
    if (lane == 0) {
        w.rec[0] = c0;
        w.rec[1] = s0;
    }
    const bool ok = s0 > 0.0 && isfinite(c0) && isfinite(s0);
    if (!ok) {
        if (lane == 0) {
            w.pstatus[0] = LSEFIT_ERR_NONFINITE;
            const FitDesc d{nullptr, nullptr, 0, 1, M};
            cheb_fail(d, w, 0, M, fz, LSEFIT_ERR_NONFINITE);
        }
        return;
    }
    for (int k = lane; k < 3 * M + 2; k += kWave) S[k] = mom[2 + k];
    wave_lds_fence();
    cheb_solve_wave<M>(w, 0, M, c0, s0, S, fz);
}

template <typename In>
hipError_t moments_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const In* y, const Launch& L,
                              int mis, const RangeArg& ra, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
    if (is_single(d)) {
        auto body = [&]<int M>() {
            launch_timed((k_moments_cheb_single<In, 2, M>), grid, block, st, d, w, x, y, L.waves, mis, ra);
        };
        dispatch_degree<kChebMax>(d.degree, body);
    } else if (maxm <= 4) {
        launch_timed((k_moments_cheb_batch<In, 2, 4>), grid, block, st, d, w, x, y, L.waves, mis,
                           maxm);
    } else if (maxm <= 8) {
        launch_timed((k_moments_cheb_batch<In, 2, 8>), grid, block, st, d, w, x, y, L.waves, mis,
                           maxm);
    } else {
        launch_timed((k_moments_cheb_batch<In, 2, kChebMax>), grid, block, st, d, w, x, y, L.waves,
                           mis, maxm);
    }
    return hipGetLastError();
}

template <typename In>
hipError_t range_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const Launch& L, int mis,
                            hipStream_t st) {
    const int64_t G = L.waves / L.wpb;
    if (is_single(d)) {
        launch_timed((k_range_cheb_single<In>), dim3(G), dim3(L.wpb * kWave), st, d, w, x, L.waves, mis);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_timed(k_range_fold_single, dim3(1), dim3(256), st, w, G);
        return hipGetLastError();
    }
    launch_timed((k_range_cheb_batch<In>), dim3(G), dim3(L.wpb * kWave), st, d, w, x, L.waves,
                       mis, maxm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_timed(k_range_fold_batch, dim3((d.batch + 255) / 256), dim3(256), st, d, w, L.waves, maxm);
    return hipGetLastError();
}

hipError_t launch_range_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const Launch& L,
                             int mis, hipStream_t st) {
    if (dtype == LSEFIT_F32) return range_cheb_typed(d, w, maxm, (const float*)x, L, mis, st);
    return range_cheb_typed(d, w, maxm, (const double*)x, L, mis, st);
}

hipError_t launch_moments_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                               const Launch& L, int mis, const RangeArg& ra, hipStream_t st) {
    if (dtype == LSEFIT_F32)
        return moments_cheb_typed(d, w, maxm, (const float*)x, (const float*)y, L, mis, ra, st);
    return moments_cheb_typed(d, w, maxm, (const double*)x, (const double*)y, L, mis, ra, st);
}

hipError_t launch_solve_cheb_moments(const double* moments, const Work& w, int m, const Finish& fz,
                                    hipStream_t st) {
    auto body = [&]<int M>() { launch_timed(k_solve_cheb_moments<M>, dim3(1), dim3(kWave), st, moments, w, fz); };
    dispatch_degree<kChebMax>(m, body);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint of a batch in the Chebyshev basis with a given range: per fit
// lambda = G^-1 dL/dc (one wave per fit, the wave solve of the forward's Gram
// system from its stored sums), then per point
//   dL/dy = q(t),  dL/dx = (q'(t) (y - f(t)) - q(t) f'(t)) / s,
// f = sum_j c_j T_j and q = sum_j lambda_j T_j with their derivatives, all by
// Clenshaw's recurrence b_j = a_j + 2t b_(j+1) - b_(j+2) and its derivative
// b_j' = 2 b_(j+1) + 2t b_(j+1)' - b_(j+2)'; value a_0 + t b_1 - b_2,
// derivative b_1 + t b_1' - b_2'.
// ---------------------------------------------------------------------------
template <int MAXC>
__global__ void __launch_bounds__(256)
    k_adjoint_cheb_solve(FitDesc d, Work w, int maxm, int solver, const double* __restrict__ gcoef,
                         int32_t coef_stride) {
    const KernelClock kclock_(w.clock);
    const int wid = wave_id_in_block(), lane = lane_id();
    for (int64_t f = (int64_t)blockIdx.x * 4 + wid; f < d.batch; f += (int64_t)gridDim.x * 4) {
        if (w.pstatus[f] != LSEFIT_OK) continue;
        double* r = w.rec + f * rec_len(maxm);
        const double* S = r + rec_S(maxm);
        auto body = [&]<int M>() {
            constexpr int N = M + 1;
            const bool mine = lane < N;
            double row[M + 2];
            bool finite = true;
#pragma unroll
            for (int c = 0; c <= N; ++c) row[c] = 0.0;
            if (mine) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    const int dk = lane > c ? lane - c : c - lane;
                    row[c] = 0.5 * (S[lane + c] + S[dk]);
                    finite = finite && isfinite(row[c]);
                }
                row[N] = gcoef[f * (int64_t)coef_stride + lane];
                finite = finite && isfinite(row[N]);
            }
            double lam = 0.0;
            int st = __ballot(!finite) ? LSEFIT_ERR_NONFINITE
                                       : (solver == LSEFIT_SOLVER_CHOLESKY ? wave_cholesky<M>(row, lam)
                                                                           : wave_gepp<M>(row, lam));
            if (st == LSEFIT_OK && __ballot(mine && !isfinite(lam))) st = LSEFIT_ERR_NONFINITE;
            if (mine) r[rec_lam(maxm) + lane] = st == LSEFIT_OK ? lam : NAN;
        };
        dispatch_degree<MAXC>(fit_deg(d, f), body);
    }
}

template <int M, typename In>
struct ChebAdjointPoint {
    double cf[M + 1], lam[M + 1];
    double inv_s, nc;
    __device__ inline void init(const double* r, int maxm) {
        inv_s = 1.0 / r[1];
        nc = -r[0] * inv_s;
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            cf[j] = r[rec_b(maxm) + j];
            lam[j] = r[rec_lam(maxm) + j];
        }
    }
    __device__ inline void point(double xv, double yv, In& gx, In& gy) const {
        const double t = fma(xv, inv_s, nc);
        const double t2 = t + t;
        double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0;   // f's recurrence and its derivative
        double p1 = 0.0, p2 = 0.0, e1 = 0.0, e2 = 0.0;   // q's
#pragma unroll
        for (int j = M; j >= 1; --j) {
            const double b0 = fma(t2, b1, cf[j] - b2);
            const double d0 = fma(t2, d1, 2.0 * b1 - d2);
            const double p0 = fma(t2, p1, lam[j] - p2);
            const double e0 = fma(t2, e1, 2.0 * p1 - e2);
            b2 = b1;
            b1 = b0;
            d2 = d1;
            d1 = d0;
            p2 = p1;
            p1 = p0;
            e2 = e1;
            e1 = e0;
        }
        const double f = fma(t, b1, cf[0] - b2), fp = fma(t, d1, b1 - d2);
        const double q = fma(t, p1, lam[0] - p2), qp = fma(t, e1, p1 - e2);
        gx = (In)((qp * (yv - f) - q * fp) * inv_s);
        gy = (In)q;
    }
};

template <typename In, int U, int MAXC>
__global__ void __launch_bounds__(256)
    k_adjoint_cheb_stream(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y,
                          In* __restrict__ gx, In* __restrict__ gy, int64_t W, int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    (void)W;
    const int rl = rec_len(maxm);
    // tiles go to blocks and the waves of a block stream each segment together
    // (no per-wave partial sums here), as in the power-basis adjoint pass
    const int64_t first = (int64_t)wave_id_in_block() * kWave + lane_id();
    const int64_t step = (int64_t)(blockDim.x / kWave) * kWave;
    const bool edge = wave_id_in_block() == 0;
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rl, (int64_t)blockIdx.x, (int64_t)gridDim.x,
                        [&](int64_t f, int64_t lo, int64_t hi, int64_t, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) {
            adjoint_nan(gx, gy, lo, hi, first, step);
            return;
        }
        auto body = [&]<int M>() {
            ChebAdjointPoint<M, In> P;
            P.init(w.rec + f * rl, maxm);
            adjoint_segment<U>(P, x, y, gx, gy, lo, hi, mis, first, step, edge);
        };
        dispatch_degree<MAXC>(mt.deg, body);
    });
}

template <typename In, int MAXC>
hipError_t adjoint_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const In* y, In* gx, In* gy,
                              const Launch& L, int mis, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
    switch (L.unroll) {
        case 1: launch_timed((k_adjoint_cheb_stream<In, 1, MAXC>), grid, block, st, d, w, x, y, gx, gy, L.waves, mis, maxm); break;
        case 2: launch_timed((k_adjoint_cheb_stream<In, 2, MAXC>), grid, block, st, d, w, x, y, gx, gy, L.waves, mis, maxm); break;
        case 4: launch_timed((k_adjoint_cheb_stream<In, 4, MAXC>), grid, block, st, d, w, x, y, gx, gy, L.waves, mis, maxm); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_cheb(const FitDesc& d, const Work& w, int maxm, int solver, int dtype, const void* x,
                               const void* y, const double* grad_coef, int32_t coef_stride, void* gx, void* gy,
                               const Launch& L, int mis, hipStream_t st) {
    int64_t blocks = (d.batch + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (maxm <= 4)
        hipLaunchKernelGGL(k_adjoint_cheb_solve<4>, dim3(blocks), dim3(256), 0, st, d, w, maxm, solver, grad_coef,
                           coef_stride);
    else if (maxm <= 8)
        hipLaunchKernelGGL(k_adjoint_cheb_solve<8>, dim3(blocks), dim3(256), 0, st, d, w, maxm, solver, grad_coef,
                           coef_stride);
    else
        hipLaunchKernelGGL(k_adjoint_cheb_solve<kChebMax>, dim3(blocks), dim3(256), 0, st, d, w, maxm, solver,
                           grad_coef, coef_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define LSEFIT_ADJC(T, MC) \
    return adjoint_cheb_typed<T, MC>(d, w, maxm, (const T*)x, (const T*)y, (T*)gx, (T*)gy, L, mis, st);
    if (dtype == LSEFIT_F32) {
        if (maxm <= 4) LSEFIT_ADJC(float, 4)
        if (maxm <= 8) LSEFIT_ADJC(float, 8)
        LSEFIT_ADJC(float, kChebMax)
    }
    if (maxm <= 4) LSEFIT_ADJC(double, 4)
    if (maxm <= 8) LSEFIT_ADJC(double, 8)
    LSEFIT_ADJC(double, kChebMax)
#undef LSEFIT_ADJC
}

template <typename In, int U>
hipError_t residual_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const In* y, In* resid,
                               double* sse, const Launch& L, int mis, hipStream_t st) {
    const int64_t G = L.waves / L.wpb;
    const dim3 grid(G), block(L.wpb * kWave);
    if (is_single(d)) {
        auto body = [&]<int M>() {
            launch_timed((k_residual_cheb_single<In, U, M>), grid, block, st, d, w, x, y, resid, L.waves,
                               mis, maxm);
        };
        dispatch_degree<kChebMax>(d.degree, body);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_timed(k_sse_fold_single, dim3(1), dim3(256), st, w, G, sse);
        return hipGetLastError();
    }
    if (maxm <= 4)
        launch_timed((k_residual_cheb_batch<In, U, 4>), grid, block, st, d, w, x, y, resid, L.waves,
                           mis, maxm);
    else if (maxm <= 8)
        launch_timed((k_residual_cheb_batch<In, U, 8>), grid, block, st, d, w, x, y, resid, L.waves,
                           mis, maxm);
    else
        launch_timed((k_residual_cheb_batch<In, U, kChebMax>), grid, block, st, d, w, x, y, resid,
                           L.waves, mis, maxm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_timed(k_sse_fold_batch, dim3((d.batch + 255) / 256), dim3(256), st, d, w, L.waves, sse);
    return hipGetLastError();
}

hipError_t launch_residual_cheb(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                                void* resid, double* sse, const Launch& L, int mis, hipStream_t st) {
    if (dtype == LSEFIT_F32)
        return residual_cheb_typed<float, 2>(d, w, maxm, (const float*)x, (const float*)y, (float*)resid, sse, L,
                                             mis, st);
    return residual_cheb_typed<double, 2>(d, w, maxm, (const double*)x, (const double*)y, (double*)resid, sse, L,
                                          mis, st);
}

hipError_t launch_finish_cheb(const FitDesc& d, const Work& w, int maxm, int64_t W, const Finish& fz,
                              hipStream_t st) {
    if (is_single(d)) {
        auto body = [&]<int M>() {
            launch_timed(k_finish_cheb_single<M>, dim3(1), dim3(kFinishWaves * kWave), st, d, w, W, maxm, fz);
        };
        dispatch_degree<kChebMax>(d.degree, body);
        return hipGetLastError();
    }
    if (maxm <= 4 && !fz.write_b && !fz.moments_out) {
        launch_timed(k_finish_cheb_lane<4>, dim3((d.batch + 255) / 256), dim3(256), st, d, w, W, maxm, fz);
        return hipGetLastError();
    }
    int64_t blocks = (d.batch + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    const dim3 grid(blocks), block(256);
    if (maxm <= 4)
        launch_timed(k_finish_cheb_batch<4>, grid, block, st, d, w, W, maxm, fz);
    else if (maxm <= 8)
        launch_timed(k_finish_cheb_batch<8>, grid, block, st, d, w, W, maxm, fz);
    else
        launch_timed(k_finish_cheb_batch<kChebMax>, grid, block, st, d, w, W, maxm, fz);
    return hipGetLastError();
}

}  // namespace lsefit
