// Chebyshev-basis fits (degree up to LSEFIT_MAX_DEGREE_CHEBYSHEV).
//
// The least-squares problem of Sec. II written in the basis T_0..T_m of
// Chebyshev polynomials of t = (x - c)/s instead of powers of x (Sec. V leaves
// higher-order polynomials as further work; the monomial normal matrix loses
// all precision there).  The streaming pass sums C_k = sum_i T_k(t_i)
// (k = 1..2m, by the three-term recurrence T_(k+1) = 2 t T_k - T_(k-1)) and
// D_j = sum_i y_i T_j(t_i); since T_j T_k = (T_(j+k) + T_|j-k|) / 2, the Gram
// matrix is G_jk = (C_(j+k) + C_|j-k|) / 2 with C_0 = n, and G c = D gives the
// Chebyshev coefficients c.  Float64 accumulation only.
#include "kernels_impl.hpp"

namespace lsefit {

constexpr int kChebMax = LSEFIT_MAX_DEGREE_CHEBYSHEV;

template <int M>
struct AccCheb {
    double C[2 * M];   // C_1..C_2M
    double D[M + 1];   // D_0..D_M
    double inv_s, nc;
    __device__ inline void init(double c, double is) {
#pragma unroll
        for (int k = 0; k < 2 * M; ++k) C[k] = 0.0;
#pragma unroll
        for (int j = 0; j <= M; ++j) D[j] = 0.0;
        inv_s = is;
        nc = -c * is;
    }
    __device__ inline void point(double xv, double yv) {
        const double t = fma(xv, inv_s, nc);
        const double t2 = t + t;
        double tp = 1.0, tc = t;
        D[0] += yv;
        C[0] += tc;
        D[1] = fma(yv, tc, D[1]);
#pragma unroll
        for (int k = 2; k <= 2 * M; ++k) {
            const double tn = fma(t2, tc, -tp);
            C[k - 1] += tn;
            if (k <= M) D[k] = fma(yv, tn, D[k]);
            tp = tc;
            tc = tn;
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

// x only, one wave over points [lo, hi) of a batch
template <typename In>
__device__ inline void minmax_segment(const In* __restrict__ x, int64_t lo, int64_t hi, int mis, MinMax<In>& r) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    if (mis >= 0) {
        int64_t a = lo + (int64_t)((VW - (int)((lo + mis) % VW)) % VW);
        if (a > hi) a = hi;
        const int64_t nv = (hi - a) / VW;
        const int64_t b = a + nv * VW;
        if (lane < a - lo) r.add(ld_scalar(x + lo + lane));
        const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
        for (int64_t j = lane; j < nv; j += kWave) r.template vec<V, VW>(ld_stream(xv + j));
        if (lane < hi - b) r.add(ld_scalar(x + b + lane));
    } else {
        for (int64_t i = lo + lane; i < hi; i += kWave) r.add(ld_scalar(x + i));
    }
}

// single fit: one (min, max) pair per block into part[2 blockIdx.x ..]
template <typename In>
__global__ void __launch_bounds__(256)
    k_range_cheb_single(FitDesc d, Work w, const In* __restrict__ x, int64_t W, int mis) {
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
    k_range_cheb_batch(FitDesc d, Work w, const In* __restrict__ x, int64_t tile, int64_t W, int mis) {
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    walk_segments(d, w.tile_start, tile, wave, W, [&](int64_t f, int64_t lo, int64_t hi, int64_t slot) {
        if (w.pstatus[f] != LSEFIT_OK) return;
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

// the waves of a block add their sums in order; one partial per block
template <int K>
__device__ inline void cheb_block_partial(const Work& w, const double (&v)[K], int stride) {
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
        w.part[(int64_t)blockIdx.x * stride + threadIdx.x] = acc;
    }
}

template <int M>
__device__ inline void cheb_wave_sums(const AccCheb<M>& acc, double (&v)[nacc(M)]) {
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) v[k] = wave_sum(acc.C[k]);
#pragma unroll
    for (int j = 0; j <= M; ++j) v[2 * M + j] = wave_sum(acc.D[j]);
}

// single fit of degree M: grid-stride sweep, one partial per block
template <typename In, int U, int M>
__global__ void __launch_bounds__(256)
    k_moments_cheb_single(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W, int mis,
                          RangeArg ra) {
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
    stream_strided<U>(x, y, d.n_single, mis, wave, W, acc);
    double v[nacc(M)];
    cheb_wave_sums(acc, v);
    cheb_block_partial<nacc(M)>(w, v, nacc(M));
}

// batch, degrees up to MAXC <= maxm: each wave walks its tiles, one partial
// slot per (wave, fit) segment
template <typename In, int U, int MAXC>
__global__ void __launch_bounds__(256)
    k_moments_cheb_batch(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t tile,
                         int64_t W, int mis, int maxm) {
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    const int stride = nacc(maxm);
    const int rl = rec_len(maxm);
    walk_segments(d, w.tile_start, tile, wave, W, [&](int64_t f, int64_t lo, int64_t hi, int64_t slot) {
        if (w.pstatus[f] != LSEFIT_OK) return;
        const double c = w.rec[f * rl + 0];
        const double inv_s = 1.0 / w.rec[f * rl + 1];
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
        dispatch_degree<MAXC>(fit_deg(d, f), body);
    });
}

// ---------------------------------------------------------------------------
// finishing a Chebyshev fit: one thread, matrices in LDS (up to 17 x 18)
// ---------------------------------------------------------------------------
constexpr int kChebN = kChebMax + 1;

struct ChebShared {
    double A[kChebN][kChebN + 1];
    double L[kChebN][kChebN];
    double X[kChebN];
    double Tp[kChebN], Tc[kChebN], Tn[kChebN], b[kChebN];
};

// partial pivoting on the augmented N x (N+1) matrix A
__device__ inline int lds_gepp(ChebShared& sm, int N) {
    double amax = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) amax = fmax(amax, fabs(sm.A[i][j]));
    const double tiny = ldexp(amax, -40);
    for (int k = 0; k < N; ++k) {
        int p = k;
        for (int r = k + 1; r < N; ++r)
            if (fabs(sm.A[r][k]) > fabs(sm.A[p][k])) p = r;
        if (!(fabs(sm.A[p][k]) > tiny)) return LSEFIT_ERR_SINGULAR;
        if (p != k)
            for (int c = 0; c <= N; ++c) {
                const double tmp = sm.A[k][c];
                sm.A[k][c] = sm.A[p][c];
                sm.A[p][c] = tmp;
            }
        for (int r = k + 1; r < N; ++r) {
            const double l = sm.A[r][k] / sm.A[k][k];
            for (int c = k; c <= N; ++c) sm.A[r][c] -= l * sm.A[k][c];
        }
    }
    for (int i = N - 1; i >= 0; --i) {
        double acc = sm.A[i][N];
        for (int c = i + 1; c < N; ++c) acc -= sm.A[i][c] * sm.X[c];
        sm.X[i] = acc / sm.A[i][i];
    }
    return LSEFIT_OK;
}

// A = L L^T on the N x N part, then the two triangular solves
__device__ inline int lds_cholesky(ChebShared& sm, int N) {
    double amax = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) amax = fmax(amax, fabs(sm.A[i][j]));
    const double tiny = ldexp(amax, -40);
    for (int j = 0; j < N; ++j) {
        double dg = sm.A[j][j];
        for (int k = 0; k < j; ++k) dg -= sm.L[j][k] * sm.L[j][k];
        if (!(dg > tiny)) return LSEFIT_ERR_SINGULAR;
        sm.L[j][j] = sqrt(dg);
        for (int i = j + 1; i < N; ++i) {
            double acc = sm.A[i][j];
            for (int k = 0; k < j; ++k) acc -= sm.L[i][k] * sm.L[j][k];
            sm.L[i][j] = acc / sm.L[j][j];
        }
    }
    for (int i = 0; i < N; ++i) {
        double acc = sm.A[i][N];
        for (int k = 0; k < i; ++k) acc -= sm.L[i][k] * sm.X[k];
        sm.X[i] = acc / sm.L[i][i];
    }
    for (int i = N - 1; i >= 0; --i) {
        double acc = sm.X[i];
        for (int k = i + 1; k < N; ++k) acc -= sm.L[k][i] * sm.X[k];
        sm.X[i] = acc / sm.L[i][i];
    }
    return LSEFIT_OK;
}

// v = [C_1..C_2m, D_0..D_m] of fit f: assemble G, solve, write the Chebyshev
// coefficients (then, for a single fit, the x-basis coefficients after them;
// for a batch, c and s after them when the stride leaves room)
__device__ inline void cheb_finish(const Work& w, int64_t f, int m, int maxm, double n, const double* v,
                                   const Finish& fz, ChebShared& sm) {
    const int N = m + 1;
    const int rl = rec_len(maxm);
    double* r = w.rec + f * rl;
    const double c0 = r[0], s0 = r[1];
    auto Cs = [&](int k) { return k == 0 ? n : v[k - 1]; };
    for (int k = 0; k <= 2 * m; ++k) r[rec_S(maxm) + k] = Cs(k);
    for (int j = 0; j < N; ++j) r[rec_T(maxm) + j] = v[2 * m + j];
    if (fz.moments_out) {
        fz.moments_out[0] = c0;
        fz.moments_out[1] = s0;
        for (int k = 0; k <= 2 * m; ++k) fz.moments_out[2 + k] = Cs(k);
        for (int j = 0; j < N; ++j) fz.moments_out[3 + 2 * m + j] = v[2 * m + j];
    }
    if (fz.mode == kMomentsOnly) return;
    bool finite = true;
    for (int j = 0; j < N; ++j) {
        for (int k = 0; k < N; ++k) {
            const int dk = j > k ? j - k : k - j;
            sm.A[j][k] = 0.5 * (Cs(j + k) + Cs(dk));
            finite = finite && isfinite(sm.A[j][k]);
        }
        sm.A[j][N] = v[2 * m + j];
        finite = finite && isfinite(sm.A[j][N]);
    }
    int st = !finite ? LSEFIT_ERR_NONFINITE
                     : (fz.solver == LSEFIT_SOLVER_CHOLESKY ? lds_cholesky(sm, N) : lds_gepp(sm, N));
    for (int j = 0; j < N && st == LSEFIT_OK; ++j)
        if (!isfinite(sm.X[j])) st = LSEFIT_ERR_NONFINITE;
    double* out = fz.coef + f * (int64_t)fz.coef_stride;
    if (st != LSEFIT_OK) {
        for (int j = 0; j < N; ++j) {
            out[j] = NAN;
            r[rec_b(maxm) + j] = NAN;
            if (fz.write_b) out[N + j] = NAN;
        }
    } else {
        for (int j = 0; j < N; ++j) {
            out[j] = sm.X[j];
            r[rec_b(maxm) + j] = sm.X[j];
        }
        if (fz.write_b) {
            // Chebyshev -> powers of t (b), then -> powers of x (a)
            for (int k = 0; k < N; ++k) {
                sm.Tp[k] = k == 0 ? 1.0 : 0.0;
                sm.Tc[k] = k == 1 ? 1.0 : 0.0;
                sm.b[k] = sm.X[0] * sm.Tp[k] + (N > 1 ? sm.X[1] * sm.Tc[k] : 0.0);
            }
            for (int j = 1; j + 1 < N; ++j) {
                for (int k = 0; k < N; ++k) sm.Tn[k] = (k > 0 ? 2.0 * sm.Tc[k - 1] : 0.0) - sm.Tp[k];
                for (int k = 0; k < N; ++k) {
                    sm.b[k] += sm.X[j + 1] * sm.Tn[k];
                    sm.Tp[k] = sm.Tc[k];
                    sm.Tc[k] = sm.Tn[k];
                }
            }
            const double inv_s = 1.0 / s0;
            for (int k = 0; k < N; ++k) {
                double acc = 0.0, binom = 1.0, cpow = 1.0, spow = 1.0;
                for (int i = 0; i < k; ++i) spow *= inv_s;
                for (int j = k; j < N; ++j) {
                    acc += sm.b[j] * binom * cpow * spow;
                    binom = binom * (double)(j + 1) / (double)(j + 1 - k);
                    cpow *= -c0;
                    spow *= inv_s;
                }
                out[N + k] = acc;
            }
        } else if (fz.coef_stride >= N + 2) {
            out[N] = c0;
            out[N + 1] = s0;
        }
    }
    w.pstatus[f] = st;
    if (fz.status) fz.status[f] = st;
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

// one block per fit: strided sums over the fit's partial slots, waves in order,
// then thread 0 finishes (single fit: the slots are the W block partials)
__global__ void __launch_bounds__(256) k_finish_cheb(FitDesc d, Work w, int64_t W, int maxm, Finish fz) {
    __shared__ ChebShared sm;
    __shared__ double sh[4][3 * kChebMax + 1];
    __shared__ double vv[3 * kChebMax + 1];
    const int stride = nacc(maxm);
    const bool single = is_single(d);
    for (int64_t f = blockIdx.x; f < d.batch; f += gridDim.x) {
        const int pst = w.pstatus[f];
        if (pst != LSEFIT_OK) {
            if (threadIdx.x == 0 && fz.mode != kMomentsOnly) cheb_fail(d, w, f, maxm, fz, pst);
            continue;
        }
        const int m = fit_deg(d, f);
        int64_t w0 = 0, w1 = W - 1, NT = 0;
        if (!single) {
            NT = w.tile_start[d.batch];
            w0 = wave_of_tile(w.tile_start[f], NT, W);
            w1 = wave_of_tile(w.tile_start[f + 1] - 1, NT, W);
        }
        auto body = [&]<int M>() {
            constexpr int K = nacc(M);
            double v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = 0.0;
            for (int64_t wv = w0 + threadIdx.x; wv <= w1; wv += blockDim.x) {
                if (!single && !wave_owns_tiles(wv, NT, W)) continue;
                const double* p = w.part + (single ? wv : wv + f) * stride;
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] += p[k];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
            if (lane_id() == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) sh[wave_id_in_block()][k] = v[k];
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                const int nw = blockDim.x / kWave;
                for (int k = 0; k < K; ++k) {
                    double acc = sh[0][k];
                    for (int i = 1; i < nw; ++i) acc += sh[i][k];
                    vv[k] = acc;
                }
                cheb_finish(w, f, M, maxm, (double)(fit_hi(d, f) - fit_lo(d, f)), vv, fz, sm);
            }
            __syncthreads();
        };
        dispatch_degree<kChebMax>(m, body);
    }
}

// one fit from caller-provided sums [c, s, C_0..C_2m, D_0..D_m]
__global__ void k_solve_cheb_moments(const double* __restrict__ mom, Work w, int m, Finish fz) {
    __shared__ ChebShared sm;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    w.rec[0] = mom[0];
    w.rec[1] = mom[1];
    const bool ok = mom[1] > 0.0 && isfinite(mom[0]) && isfinite(mom[1]);
    w.pstatus[0] = ok ? LSEFIT_OK : LSEFIT_ERR_NONFINITE;
    if (!ok) {
        const FitDesc d{nullptr, nullptr, 0, 1, m};
        cheb_fail(d, w, 0, m, fz, LSEFIT_ERR_NONFINITE);
        return;
    }
    cheb_finish(w, 0, m, m, mom[2], mom + 3, fz, sm);
}

template <typename In>
hipError_t moments_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const In* y, const Launch& L,
                              int mis, const RangeArg& ra, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
    if (is_single(d)) {
        auto body = [&]<int M>() {
            hipLaunchKernelGGL((k_moments_cheb_single<In, 2, M>), grid, block, 0, st, d, w, x, y, L.waves, mis, ra);
        };
        dispatch_degree<kChebMax>(d.degree, body);
    } else if (maxm <= 4) {
        hipLaunchKernelGGL((k_moments_cheb_batch<In, 2, 4>), grid, block, 0, st, d, w, x, y, L.tile, L.waves, mis,
                           maxm);
    } else if (maxm <= 8) {
        hipLaunchKernelGGL((k_moments_cheb_batch<In, 2, 8>), grid, block, 0, st, d, w, x, y, L.tile, L.waves, mis,
                           maxm);
    } else {
        hipLaunchKernelGGL((k_moments_cheb_batch<In, 2, kChebMax>), grid, block, 0, st, d, w, x, y, L.tile, L.waves,
                           mis, maxm);
    }
    return hipGetLastError();
}

template <typename In>
hipError_t range_cheb_typed(const FitDesc& d, const Work& w, int maxm, const In* x, const Launch& L, int mis,
                            hipStream_t st) {
    const int64_t G = L.waves / L.wpb;
    if (is_single(d)) {
        hipLaunchKernelGGL((k_range_cheb_single<In>), dim3(G), dim3(L.wpb * kWave), 0, st, d, w, x, L.waves, mis);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_range_fold_single, dim3(1), dim3(256), 0, st, w, G);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_range_cheb_batch<In>), dim3(G), dim3(L.wpb * kWave), 0, st, d, w, x, L.tile, L.waves,
                       mis);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_range_fold_batch, dim3((d.batch + 255) / 256), dim3(256), 0, st, d, w, L.waves, maxm);
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
    hipLaunchKernelGGL(k_solve_cheb_moments, dim3(1), dim3(64), 0, st, moments, w, m, fz);
    return hipGetLastError();
}

hipError_t launch_finish_cheb(const FitDesc& d, const Work& w, int maxm, int64_t W, const Finish& fz,
                              hipStream_t st) {
    int64_t blocks = d.batch < 65536 ? d.batch : 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_finish_cheb, dim3(blocks), dim3(256), 0, st, d, w, W, maxm, fz);
    return hipGetLastError();
}

}  // namespace lsefit
