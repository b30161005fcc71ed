// Kernels of the moment-pass least-squares fit for gfx950 (CDNA4, wave64).
//
// The power sums S_p = sum t^p and T_j = sum t^j y of Sec. II are one
// HBM-bound streaming pass: each wave of a persistent grid owns a balanced,
// contiguous share of the points, loads x and y with 16-byte vector loads,
// forms t = (x - c)/s and its powers by repeated multiplication, accumulates
// per lane, reduces across the wave with a fixed butterfly and writes one
// partial per (wave, fit).  A second kernel sums the partials of each fit in
// wave order and solves the Hankel normal system (Gaussian elimination with
// partial pivoting, end of Sec. II) in float64.
#pragma once

#include "kernels.hpp"
#include "launchers.hpp"

#include <type_traits>

namespace lsefit {

template <typename In>
struct VecOf;
template <>
struct VecOf<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <>
struct VecOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};

template <typename V>
__device__ inline V ld_stream(const V* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ inline T ld_scalar(const T* p) {
    return __builtin_nontemporal_load(p);
}

// ---------------------------------------------------------------------------
// per-lane accumulators
// ---------------------------------------------------------------------------

// float64 form: t, powers and sums in float64 (full-rate on CDNA4 vector ALUs).
template <int M>
struct AccF64 {
    double S[2 * M];  // S_1..S_2M
    double T[M + 1];  // T_0..T_M
    double inv_s, nc;
    __device__ inline void init(double c, double is) {
#pragma unroll
        for (int k = 0; k < 2 * M; ++k) S[k] = 0.0;
#pragma unroll
        for (int j = 0; j <= M; ++j) T[j] = 0.0;
        inv_s = is;
        nc = -c * is;
    }
    __device__ inline void point(double xv, double yv) {
        // powers up to t^M by a product tree, p_k = p_(k/2) p_(k - k/2) (depth
        // ceil(log2 M) instead of a chain of dependent multiplies); a power above
        // t^M is only ever added to its sum, so its product p_(k/2) p_(k - k/2)
        // is formed inside the fused multiply-add of that sum, as are the t^j y
        // of the right-hand side: 4M + 1 float64 operations per point
        double p[M + 1];
        p[1] = fma(xv, inv_s, nc);
#pragma unroll
        for (int k = 2; k <= M; ++k) p[k] = p[k / 2] * p[k - k / 2];
        T[0] += yv;
#pragma unroll
        for (int k = 1; k <= M; ++k) {
            S[k - 1] += p[k];
            T[k] = fma(yv, p[k], T[k]);
        }
#pragma unroll
        for (int k = M + 1; k <= 2 * M; ++k) S[k - 1] = fma(p[k / 2], p[k - k / 2], S[k - 1]);
    }
    template <typename V, int VW>
    __device__ inline void vec(const V& xv, const V& yv) {
#pragma unroll
        for (int e = 0; e < VW; ++e) point((double)xv[e], (double)yv[e]);
    }
    __device__ inline void scalar(double xv, double yv) { point(xv, yv); }
    __device__ inline void out(double (&v)[nacc(M)]) const {
#pragma unroll
        for (int k = 0; k < 2 * M; ++k) v[k] = S[k];
#pragma unroll
        for (int j = 0; j <= M; ++j) v[2 * M + j] = T[j];
    }
};

// compensated float32 form: t and powers in float32; the sums of a group of
// points (one 16-byte vector) are plain float32 and are folded into (sum,
// compensation) pairs by Kahan's method once per group.
template <int M>
struct AccF32C {
    float S[2 * M], cS[2 * M];
    float T[M + 1], cT[M + 1];
    float inv_s, nc;
    __device__ static inline void kahan(float& s, float& c, float v) {
        const float yv = v - c;
        const float t = s + yv;
        c = (t - s) - yv;
        s = t;
    }
    __device__ inline void init(double c, double is) {
#pragma unroll
        for (int k = 0; k < 2 * M; ++k) S[k] = cS[k] = 0.0f;
#pragma unroll
        for (int j = 0; j <= M; ++j) T[j] = cT[j] = 0.0f;
        inv_s = (float)is;
        nc = (float)(-c * is);
    }
    template <int G>
    __device__ inline void group(const float (&xs)[G], const float (&ys)[G]) {
        float t[G], p[G];
#pragma unroll
        for (int e = 0; e < G; ++e) {
            t[e] = fmaf(xs[e], inv_s, nc);
            p[e] = t[e];
        }
        float g = ys[0];
#pragma unroll
        for (int e = 1; e < G; ++e) g += ys[e];
        kahan(T[0], cT[0], g);
        // powers by a product tree per point (as in the float64 form)
        float pw[2 * M + 1][G];
#pragma unroll
        for (int e = 0; e < G; ++e) {
            pw[1][e] = t[e];
#pragma unroll
            for (int k = 2; k <= 2 * M; ++k) pw[k][e] = pw[k / 2][e] * pw[k - k / 2][e];
        }
#pragma unroll
        for (int k = 1; k <= 2 * M; ++k) {
#pragma unroll
            for (int e = 0; e < G; ++e) p[e] = pw[k][e];
            float gs = p[0];
#pragma unroll
            for (int e = 1; e < G; ++e) gs += p[e];
            kahan(S[k - 1], cS[k - 1], gs);
            if (k <= M) {
                float gt = ys[0] * p[0];
#pragma unroll
                for (int e = 1; e < G; ++e) gt = fmaf(ys[e], p[e], gt);
                kahan(T[k], cT[k], gt);
            }
        }
    }
    template <typename V, int VW>
    __device__ inline void vec(const V& xv, const V& yv) {
        float xs[VW], ys[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            xs[e] = xv[e];
            ys[e] = yv[e];
        }
        group<VW>(xs, ys);
    }
    __device__ inline void scalar(float xv, float yv) {
        float xs[1] = {xv}, ys[1] = {yv};
        group<1>(xs, ys);
    }
    __device__ inline void out(double (&v)[nacc(M)]) const {
#pragma unroll
        for (int k = 0; k < 2 * M; ++k) v[k] = (double)S[k] - (double)cS[k];
#pragma unroll
        for (int j = 0; j <= M; ++j) v[2 * M + j] = (double)T[j] - (double)cT[j];
    }
};

// refinement: r = y - sum_j b_j t^j and R_j = sum t^j r, all float64.
template <int M>
struct AccRefine {
    double R[M + 1];
    double b[M + 1];
    double inv_s, nc;
    __device__ inline void init(double c, double is, const double* bb) {
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            R[j] = 0.0;
            b[j] = bb[j];
        }
        inv_s = is;
        nc = -c * is;
    }
    __device__ inline void point(double xv, double yv) {
        const double t = fma(xv, inv_s, nc);
        double f = b[M];
#pragma unroll
        for (int j = M - 1; j >= 0; --j) f = fma(f, t, b[j]);
        const double r = yv - f;
        double p = t;
        R[0] += r;
        R[1] = fma(p, r, R[1]);
#pragma unroll
        for (int j = 2; j <= M; ++j) {
            p *= t;
            R[j] = fma(p, r, R[j]);
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
// one wave streams points [lo, hi) of x and y into an accumulator.  `mis` is
// the common misalignment (in elements, modulo the vector width) of the base
// pointers, or -1 when they differ (then every load is scalar).
// ---------------------------------------------------------------------------
template <int U, typename In, class Acc>
__device__ inline void stream_segment(const In* __restrict__ x, const In* __restrict__ y, int64_t lo, int64_t hi,
                                      int mis, Acc& acc) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    if (mis >= 0) {
        int64_t a = lo + (int64_t)((VW - (int)((lo + mis) % VW)) % VW);
        if (a > hi) a = hi;
        const int64_t nv = (hi - a) / VW;
        const int64_t b = a + nv * VW;
        if (lane < a - lo) acc.scalar(ld_scalar(x + lo + lane), ld_scalar(y + lo + lane));
        const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
        const V* __restrict__ yv = reinterpret_cast<const V*>(y + a);
        int64_t j = lane;
        const int64_t rounds = nv / (kWave * U);
        for (int64_t r = 0; r < rounds; ++r) {
            V xs[U], ys[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xs[u] = ld_stream(xv + j + u * kWave);
                ys[u] = ld_stream(yv + j + u * kWave);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc.template vec<V, VW>(xs[u], ys[u]);
            j += (int64_t)kWave * U;
        }
        for (; j < nv; j += kWave) acc.template vec<V, VW>(ld_stream(xv + j), ld_stream(yv + j));
        if (lane < hi - b) acc.scalar(ld_scalar(x + b + lane), ld_scalar(y + b + lane));
    } else {
        for (int64_t i = lo + lane; i < hi; i += kWave) acc.scalar(ld_scalar(x + i), ld_scalar(y + i));
    }
}

// single fit: the whole grid strides over the 16-byte vectors of x and y (wave
// g reads vectors g*64 + lane, then every W*64 further), so consecutive waves
// read consecutive kilobytes and the grid sweeps the arrays front to back.
// Wave 0 also takes the unaligned head and the ragged tail.  The next round's
// U vectors per array are loaded before the current round is accumulated, so
// that a wave covers its own load latency with its arithmetic (few waves fit
// per SIMD at high degree).
//
// `prologue` runs once per lane after the first round's loads are issued and
// before anything is accumulated (it must be called by every wave of the
// block: it may hold a barrier); the power-sum pass derives (c, s) there, so
// that the range sample's latency overlaps the first loads.
template <int U, bool PRO, typename In, class Acc, class Pro>
__device__ inline void stream_strided(const In* __restrict__ x, const In* __restrict__ y, int64_t n, int mis,
                                      int64_t gwave, int64_t W, Acc& acc, Pro&& prologue) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    const int64_t step = W * kWave;
    if (mis < 0) {
        prologue();
        for (int64_t i = gwave * kWave + lane; i < n; i += step) acc.scalar(ld_scalar(x + i), ld_scalar(y + i));
        return;
    }
    int64_t a = (VW - mis) % VW;
    if (a > n) a = n;
    const int64_t nv = (n - a) / VW;
    const int64_t b = a + nv * VW;
    // without a prologue the head goes first, so that no vector is live across
    // it (the register budget of the passes with large accumulators)
    if (!PRO && gwave == 0 && lane < a) acc.scalar(ld_scalar(x + lane), ld_scalar(y + lane));
    const V* __restrict__ xv = reinterpret_cast<const V*>(x + a);
    const V* __restrict__ yv = reinterpret_cast<const V*>(y + a);
    const int64_t span = (int64_t)(U - 1) * step;
    int64_t j = gwave * kWave + lane;
    bool have = j + span < nv;
    V xs[U], ys[U];
    if (have) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xs[u] = ld_stream(xv + j + u * step);
            ys[u] = ld_stream(yv + j + u * step);
        }
    }
    if constexpr (PRO) {
        prologue();
        if (gwave == 0 && lane < a) acc.scalar(ld_scalar(x + lane), ld_scalar(y + lane));
    }
    while (have) {
        const int64_t jn = j + (int64_t)U * step;
        const bool next = jn + span < nv;
        V xn[U], yn[U];
        if (next) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xn[u] = ld_stream(xv + jn + u * step);
                yn[u] = ld_stream(yv + jn + u * step);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc.template vec<V, VW>(xs[u], ys[u]);
        if (next) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xs[u] = xn[u];
                ys[u] = yn[u];
            }
        }
        j = jn;
        have = next;
    }
    for (; j < nv; j += step) acc.template vec<V, VW>(ld_stream(xv + j), ld_stream(yv + j));
    if (gwave == 0 && lane < n - b) acc.scalar(ld_scalar(x + b + lane), ld_scalar(y + b + lane));
}

template <int U, typename In, class Acc>
__device__ inline void stream_strided(const In* __restrict__ x, const In* __restrict__ y, int64_t n, int mis,
                                      int64_t gwave, int64_t W, Acc& acc) {
    stream_strided<U, false>(x, y, n, mis, gwave, W, acc, [] {});
}

// run body.template operator()<m>() for the runtime degree m (1 <= m <= MAXM)
template <int MAXM, class Body>
__host__ __device__ inline void dispatch_degree(int m, Body&& body) {
    switch (m) {
        case 1: if constexpr (MAXM >= 1) body.template operator()<1>(); break;
        case 2: if constexpr (MAXM >= 2) body.template operator()<2>(); break;
        case 3: if constexpr (MAXM >= 3) body.template operator()<3>(); break;
        case 4: if constexpr (MAXM >= 4) body.template operator()<4>(); break;
        case 5: if constexpr (MAXM >= 5) body.template operator()<5>(); break;
        case 6: if constexpr (MAXM >= 6) body.template operator()<6>(); break;
        case 7: if constexpr (MAXM >= 7) body.template operator()<7>(); break;
        case 8: if constexpr (MAXM >= 8) body.template operator()<8>(); break;
        case 9: if constexpr (MAXM >= 9) body.template operator()<9>(); break;
        case 10: if constexpr (MAXM >= 10) body.template operator()<10>(); break;
        case 11: if constexpr (MAXM >= 11) body.template operator()<11>(); break;
        case 12: if constexpr (MAXM >= 12) body.template operator()<12>(); break;
        case 13: if constexpr (MAXM >= 13) body.template operator()<13>(); break;
        case 14: if constexpr (MAXM >= 14) body.template operator()<14>(); break;
        case 15: if constexpr (MAXM >= 15) body.template operator()<15>(); break;
        case 16: if constexpr (MAXM >= 16) body.template operator()<16>(); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// per-fit combine and solve
// ---------------------------------------------------------------------------

// run body.template operator()<NK>() for the number of partial sums a finish
// of this mode reads: the M + 1 refinement sums, the one sum of squares, or all
// nacc(M).  With NK fixed at compile time the loads of a partial slot carry no
// per-sum condition, so they are issued together rather than each behind a
// branch of its own (a wait per load).
template <int M, class Body>
__device__ inline void dispatch_sum_count(int mode, Body&& body) {
    if (mode == kRefine) body.template operator()<M + 1>();
    else if (mode == kSSE) body.template operator()<1>();
    else body.template operator()<nacc(M)>();
}

// n: the fit's number of points; (c, s): its range from the record (loaded by
// the caller with its other loads, so that they share one memory round trip);
// rin: a copy of the fit's record to read the refinement's sums and solution
// from (NULL: the record itself); the results always go to the record
template <int M, int MAXM>
__device__ inline void finish_fit(const FitDesc& d, const Work& w, int64_t f, const double (&v)[nacc(M)],
                                  const Finish& fz, int64_t n, double c, double s, const double* rin = nullptr) {
    constexpr int N = M + 1;
    constexpr int rl = rec_len(MAXM);
    if (fz.mode == kSSE) {
        fz.coef[f] = v[0];
        return;
    }
    double* r = w.rec + f * rl;
    const double* rr = rin ? rin : r;
    double* a_out = fz.coef + f * (int64_t)fz.coef_stride;
    double S[2 * M + 1];
    double b[1][N], a[N];
    int st;
    if (fz.mode == kRefine) {
#pragma unroll
        for (int k = 0; k <= 2 * M; ++k) S[k] = rr[rec_S(MAXM) + k];
        double R[1][N], delta[1][N];
#pragma unroll
        for (int j = 0; j < N; ++j) R[0][j] = v[j];
        st = normal_solve<N, 1>(fz.solver, S, R, delta);
#pragma unroll
        for (int j = 0; j < N; ++j) b[0][j] = rr[rec_b(MAXM) + j] + delta[0][j];
    } else {
        S[0] = (double)n;
#pragma unroll
        for (int k = 1; k <= 2 * M; ++k) S[k] = v[k - 1];
        double T[1][N];
#pragma unroll
        for (int j = 0; j < N; ++j) T[0][j] = v[2 * M + j];
#pragma unroll
        for (int k = 0; k <= 2 * M; ++k) r[rec_S(MAXM) + k] = S[k];
#pragma unroll
        for (int j = 0; j < N; ++j) r[rec_T(MAXM) + j] = T[0][j];
        if (fz.moments_out) {
            fz.moments_out[0] = c;
            fz.moments_out[1] = s;
#pragma unroll
            for (int k = 0; k <= 2 * M; ++k) fz.moments_out[2 + k] = S[k];
#pragma unroll
            for (int j = 0; j < N; ++j) fz.moments_out[3 + 2 * M + j] = T[0][j];
        }
        if (fz.mode == kMomentsOnly) return;
        st = normal_solve<N, 1>(fz.solver, S, T, b);
    }
    if (st == LSEFIT_OK) {
        to_x_basis<N>(b[0], c, s, a);
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (!isfinite(a[k])) st = LSEFIT_ERR_NONFINITE;
    }
    if (st != LSEFIT_OK) {
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = b[0][k] = NAN;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        r[rec_b(MAXM) + k] = b[0][k];
        a_out[k] = a[k];
        if (fz.write_b) a_out[N + k] = b[0][k];
        if (fz.b_at >= 0) a_out[fz.b_at + k] = b[0][k];
    }
    if (fz.cs_at >= 0) {
        a_out[fz.cs_at] = c;
        a_out[fz.cs_at + 1] = s;
    }
    w.pstatus[f] = st;
    fz.status[f] = st;
}

// a fit that never reached elimination: NaN coefficients (all coef_stride of
// them when the degree itself is out of range) and its status
template <int MAXM>
__device__ inline void fail_fit(const FitDesc& d, const Work& w, int64_t f, const Finish& fz, int st) {
    if (fz.mode == kSSE) {
        fz.coef[f] = NAN;
        return;
    }
    const int m = fit_deg(d, f);
    const bool valid = m >= 1 && m <= MAXM;
    const int n = valid ? m + 1 : fz.coef_stride;
    double* a_out = fz.coef + f * (int64_t)fz.coef_stride;
    for (int k = 0; k < n; ++k) a_out[k] = NAN;
    if (fz.write_b && valid)
        for (int k = 0; k < n; ++k) a_out[n + k] = NAN;
    if (fz.b_at >= 0 && valid)
        for (int k = 0; k < n; ++k) a_out[fz.b_at + k] = NAN;
    if (fz.cs_at >= 0) {   // the range the plan recorded for the fit
        a_out[fz.cs_at] = w.rec[f * rec_len(MAXM)];
        a_out[fz.cs_at + 1] = w.rec[f * rec_len(MAXM) + 1];
    }
    fz.status[f] = st;
}

// finish_fit by one wave (every lane holds the same v): the normal system is
// solved with a row per lane (wave_gepp / wave_cholesky, the same operations
// per entry as hankel_solve / hankel_cholesky) and the change back to the
// x-basis runs with a coefficient per lane.  sm: 3M+2 doubles of this wave's LDS.
//
// rin: a copy of the fit's record to read from (NULL: the record itself); the
// results are always written to the record in the workspace.
template <int M, int MAXM>
__device__ inline void finish_fit_wave(const FitDesc& d, const Work& w, int64_t f, const double (&v)[nacc(M)],
                                       const Finish& fz, double* sm, const double* rin = nullptr) {
    constexpr int N = M + 1;
    constexpr int rl = rec_len(MAXM);
    const int lane = lane_id();
    const bool mine = lane < N;
    if (fz.mode == kSSE) {
        if (lane == 0) fz.coef[f] = v[0];
        return;
    }
    double* r = w.rec + f * rl;
    const double* rr = rin ? rin : r;
    const double c = rr[0], s = rr[1];
    // S_0..S_2M and the right side (T, or the refinement sums) into LDS
    if (lane == 0) {
        if (fz.mode == kRefine) {
#pragma unroll
            for (int k = 0; k <= 2 * M; ++k) sm[k] = rr[rec_S(MAXM) + k];
#pragma unroll
            for (int j = 0; j < N; ++j) sm[2 * M + 1 + j] = v[j];
        } else {
            sm[0] = (double)(fit_hi(d, f) - fit_lo(d, f));
#pragma unroll
            for (int k = 1; k <= 2 * M; ++k) sm[k] = v[k - 1];
#pragma unroll
            for (int j = 0; j < N; ++j) sm[2 * M + 1 + j] = v[2 * M + j];
#pragma unroll
            for (int k = 0; k <= 2 * M; ++k) r[rec_S(MAXM) + k] = sm[k];
#pragma unroll
            for (int j = 0; j < N; ++j) r[rec_T(MAXM) + j] = sm[2 * M + 1 + j];
            if (fz.moments_out) {
                fz.moments_out[0] = c;
                fz.moments_out[1] = s;
#pragma unroll
                for (int k = 0; k < 3 * M + 2; ++k) fz.moments_out[2 + k] = sm[k];
            }
        }
    }
    wave_lds_fence();
    if (fz.mode == kMomentsOnly) return;
    double row[M + 2];
    bool finite = true;
#pragma unroll
    for (int cc = 0; cc <= N; ++cc) row[cc] = 0.0;
    if (mine) {
#pragma unroll
        for (int cc = 0; cc < N; ++cc) {
            row[cc] = sm[lane + cc];
            finite = finite && isfinite(row[cc]);
        }
        row[N] = sm[2 * M + 1 + lane];
        finite = finite && isfinite(row[N]);
    }
    wave_lds_fence();
    double x = 0.0;
    int st = __ballot(!finite) ? LSEFIT_ERR_NONFINITE
                               : (fz.solver == LSEFIT_SOLVER_CHOLESKY ? wave_cholesky<M>(row, x)
                                                                      : wave_gepp<M>(row, x));
    if (st == LSEFIT_OK && __ballot(mine && !isfinite(x))) st = LSEFIT_ERR_NONFINITE;
    double b = x;
    if (fz.mode == kRefine && mine) b = rr[rec_b(MAXM) + lane] + x;
    // a_k = sum_(j>=k) b_j C(j,k) (-c)^(j-k) s^-j, lane k (the order of to_x_basis)
    double a = 0.0;
    if (st == LSEFIT_OK) {
        const double inv_s = 1.0 / s;
        double binom = 1.0, cpow = 1.0, spow = 1.0;
        for (int i = 0; i < lane && i < N; ++i) spow *= inv_s;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const double bj = bcast(b, j);
            if (lane <= j) {
                a += bj * binom * cpow * spow;
                binom = binom * (double)(j + 1) / (double)(j + 1 - lane);
                cpow *= -c;
                spow *= inv_s;
            }
        }
        if (__ballot(mine && !isfinite(a))) st = LSEFIT_ERR_NONFINITE;
    }
    if (st != LSEFIT_OK) a = b = NAN;
    double* a_out = fz.coef + f * (int64_t)fz.coef_stride;
    if (mine) {
        r[rec_b(MAXM) + lane] = b;
        a_out[lane] = a;
        if (fz.write_b) a_out[N + lane] = b;
        if (fz.b_at >= 0) a_out[fz.b_at + lane] = b;
    }
    if (fz.cs_at >= 0 && lane < 2) a_out[fz.cs_at + lane] = lane == 0 ? c : s;
    if (lane == 0) {
        w.pstatus[f] = st;
        fz.status[f] = st;
    }
}

// the threads of one block sum the partial slots of fit f in a fixed order
// (strided per thread, butterfly per wave, waves in order), then wave 0
// finishes the fit
template <int MAXM>
__device__ inline void block_combine_fit(const FitDesc& d, const Work& w, int64_t f, int64_t W, const Finish& fz) {
    constexpr int stride = nacc(MAXM);
    __shared__ double sh[4][stride];
    __shared__ double sm[3 * MAXM + 2];
    const int pst = w.pstatus[f];
    if (pst != LSEFIT_OK) {
        if (threadIdx.x == 0 && fz.mode != kMomentsOnly) fail_fit<MAXM>(d, w, f, fz, pst);
        return;
    }
    const int nw = blockDim.x / kWave;
    const int64_t NT = w.tile_start[d.batch];
    const int64_t ts = w.tile_start[f], te = w.tile_start[f + 1];
    const int64_t w0 = wave_of_tile(ts, NT, W), w1 = wave_of_tile(te - 1, NT, W);
    auto body = [&]<int M>() {
        constexpr int K = nacc(M);
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = 0.0;
        dispatch_sum_count<M>(fz.mode, [&]<int NK>() {
            for (int64_t wv = w0 + threadIdx.x; wv <= w1; wv += blockDim.x) {
                if (!wave_owns_tiles(wv, NT, W)) continue;
                const double* p = w.part + (wv + f) * stride;
#pragma unroll
                for (int k = 0; k < NK; ++k) v[k] += p[k];
            }
#pragma unroll
            for (int k = 0; k < NK; ++k) v[k] = wave_sum(v[k]);
        });
        const int wv = wave_id_in_block();
        if (lane_id() == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) sh[wv][k] = v[k];
        }
        __syncthreads();
        if (wv == 0) {
            wave_column_sums<K, stride>(sh, nw, v);
            finish_fit_wave<M, MAXM>(d, w, f, v, fz, sm);
        }
        __syncthreads();
    };
    dispatch_degree<MAXM>(fit_deg(d, f), body);
}

// The G block partials of a single fit, stored sum-major (part[k * G + g]), are
// added up by a finish block of kFinishWaves waves: wave v takes sums v,
// v + kFinishWaves, ...; lane l adds blocks l, l + 64, l + 128, ... in that
// order, then the wave's butterfly (wave_sum) adds the lanes, and lane 0 writes
// the total of sum k to out[k] (LDS).  All of a wave's loads are issued
// together, kFinishChunk per lane and sum at a time, so that one memory round
// trip covers up to 512 blocks: a lane past the last block reads the last block
// again and drops it, rather than branching around its load.
constexpr int kFinishWaves = 8;
constexpr int kFinishChunk = 8;
// up to this degree one lane solves and changes the basis in registers
// (finish_fit: the same operations as the wave form, so the same bits, and
// 0.1-0.25 µs sooner without the lane exchanges); above it the wave does, a
// row per lane (finish_fit_wave), which is sooner from degree 5 on
constexpr int kFinishLaneMax = 4;

template <int NK>
__device__ inline void block_sum_partials(const double* __restrict__ part, int64_t G, double* out) {
    constexpr int C = (NK + kFinishWaves - 1) / kFinishWaves;   // sums per wave, at most
    const int wv = wave_id_in_block(), lane = lane_id();
    if (wv >= NK) return;
    const double* p[C];
    double t[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        p[c] = part + (int64_t)min(wv + c * kFinishWaves, NK - 1) * G;
        t[c] = 0.0;
    }
    for (int64_t g0 = 0; g0 < G; g0 += kFinishChunk * kWave) {
        double x[kFinishChunk][C];
#pragma unroll
        for (int i = 0; i < kFinishChunk; ++i) {
            const int64_t g = min(g0 + i * kWave + lane, G - 1);
#pragma unroll
            for (int c = 0; c < C; ++c) x[i][c] = p[c][g];
        }
#pragma unroll
        for (int i = 0; i < kFinishChunk; ++i) {
            const bool in = g0 + i * kWave + lane < G;
#pragma unroll
            for (int c = 0; c < C; ++c) t[c] = in ? t[c] + x[i][c] : t[c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double tot = wave_sum(t[c]);
        const int k = wv + c * kFinishWaves;
        if (lane == 0 && k < NK) out[k] = tot;
    }
}

// single fit: the finish block adds up the partials (block_sum_partials) and
// wave 0 finishes the fit.  Every load the finish needs is issued at its start
// -- the fit's status and range record with the partials -- so that they cost
// one memory round trip, not three in a row; the partials are summed whatever
// the status (the pass before always writes them) and the status only decides
// what is written.
template <int MAXM>
__device__ inline void finish_single_block(const FitDesc& d, const Work& w, int64_t G, const Finish& fz) {
    constexpr int rl = rec_len(MAXM);
    __shared__ double sums[nacc(MAXM)];
    __shared__ double sm[3 * MAXM + 2];
    __shared__ double rs[rl];
    const int pst = w.pstatus[0];
    const double rv = threadIdx.x < rl ? w.rec[threadIdx.x] : 0.0;
    auto body = [&]<int M>() {
        constexpr int K = nacc(M);
        dispatch_sum_count<M>(fz.mode, [&]<int NK>() { block_sum_partials<NK>(w.part, G, sums); });
        if (threadIdx.x < rl) rs[threadIdx.x] = rv;
        __syncthreads();
        if (wave_id_in_block() == 0) {
            if (pst != LSEFIT_OK) {
                if (lane_id() == 0 && fz.mode != kMomentsOnly) fail_fit<MAXM>(d, w, 0, fz, pst);
            } else {
                const int nk = fz.mode == kRefine ? M + 1 : (fz.mode == kSSE ? 1 : K);
                double v[K];
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] = k < nk ? sums[k] : 0.0;
                if constexpr (M <= kFinishLaneMax) {
                    if (lane_id() == 0)
                        finish_fit<M, MAXM>(d, w, 0, v, fz, fit_hi(d, 0) - fit_lo(d, 0), rs[0], rs[1], rs);
                } else {
                    finish_fit_wave<M, MAXM>(d, w, 0, v, fz, sm, rs);
                }
            }
        }
    };
    dispatch_degree<MAXM>(d.degree, body);
}

template <int MAXM>
__global__ void __launch_bounds__(kFinishWaves * kWave) k_finish_single(FitDesc d, Work w, int64_t G, Finish fz) {
    const KernelClock kclock_(w.clock);
    finish_single_block<MAXM>(d, w, G, fz);
}

// ---------------------------------------------------------------------------
// single fit: every block of the streaming grid derives (c, s) itself, from the
// same sample (kSingleRangeSamples evenly strided points, first and last
// included; exact min/max, so the result does not depend on the block shape)
// ---------------------------------------------------------------------------
constexpr int kSingleRangeSamples = 256;

template <typename In>
__device__ inline void single_range(const FitDesc& d, const Work& w, const In* __restrict__ x, const RangeArg& ra,
                                    double* c_out, double* inv_s_out) {
    __shared__ double smin[4], smax[4];
    double c = ra.c, s = ra.s;
    if (ra.mode == LSEFIT_RANGE_AUTO) {
        const int64_t n = d.n_single;
        const int64_t K = n < kSingleRangeSamples ? n : kSingleRangeSamples;
        double lo = INFINITY, hi = -INFINITY;
        double v[kSingleRangeSamples / kWave];
#pragma unroll
        for (int j = 0; j < kSingleRangeSamples / kWave; ++j) {
            const int64_t i = threadIdx.x + (int64_t)j * blockDim.x;
            v[j] = NAN;
            if (i < K) v[j] = (double)x[K == 1 ? 0 : i * (n - 1) / (K - 1)];
        }
#pragma unroll
        for (int j = 0; j < kSingleRangeSamples / kWave; ++j) {
            if (isfinite(v[j])) {
                lo = fmin(lo, v[j]);
                hi = fmax(hi, v[j]);
            }
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane_id() == 0) {
            smin[wave_id_in_block()] = lo;
            smax[wave_id_in_block()] = hi;
        }
        __syncthreads();
        const int nw = blockDim.x / kWave;
        lo = smin[0];
        hi = smax[0];
        for (int i = 1; i < nw; ++i) {
            lo = fmin(lo, smin[i]);
            hi = fmax(hi, smax[i]);
        }
        snap_range(lo, hi, &c, &s);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.rec[0] = c;
        w.rec[1] = s;
        w.pstatus[0] = LSEFIT_OK;
    }
    *c_out = c;
    *inv_s_out = 1.0 / s;
}

// single fit: the waves of a block add their wave sums in order into one
// partial per block, stored sum-major (sum k of block g at part[k G + g], G
// blocks), so that the finish reads the partials of each sum contiguously
template <int K, int STRIDE>
__device__ inline void single_block_partial(const Work& w, const double (&v)[K]) {
    __shared__ double sh[4][STRIDE];
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

// ---------------------------------------------------------------------------
// power-sum pass
// ---------------------------------------------------------------------------
template <int MAXM, int PREC, typename In, int U>
__global__ void __launch_bounds__(256)
    k_moments(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W,
              int mis, RangeArg ra) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    constexpr int stride = nacc(MAXM);
    constexpr int rl = rec_len(MAXM);
    if (is_single(d)) {
        auto body = [&]<int M>() {
            using Acc = std::conditional_t<PREC == LSEFIT_PREC_F64, AccF64<M>, AccF32C<M>>;
            double v[nacc(M)];
            Acc acc;
            // (c, s) from the range sample while the first loads are in flight
            stream_strided<U, true>(x, y, d.n_single, mis, wave, W, acc, [&] {
                double c, inv_s;
                single_range(d, w, x, ra, &c, &inv_s);
                acc.init(c, inv_s);
            });
            acc.out(v);
#pragma unroll
            for (int k = 0; k < nacc(M); ++k) v[k] = wave_sum(v[k]);
            single_block_partial<nacc(M), stride>(w, v);
        };
        dispatch_degree<MAXM>(d.degree, body);
        return;
    }
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rl, wave, W,
                        [&](int64_t f, int64_t lo, int64_t hi, int64_t slot, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) return;
        const double inv_s = 1.0 / mt.s;
        double* __restrict__ out = w.part + slot * stride;
        auto body = [&]<int M>() {
            using Acc = std::conditional_t<PREC == LSEFIT_PREC_F64, AccF64<M>, AccF32C<M>>;
            Acc acc;
            acc.init(mt.c, inv_s);
            stream_segment<U>(x, y, lo, hi, mis, acc);
            double v[nacc(M)];
            acc.out(v);
#pragma unroll
            for (int k = 0; k < nacc(M); ++k) v[k] = wave_sum(v[k]);
            if (lane_id() == 0) {
#pragma unroll
                for (int k = 0; k < nacc(M); ++k) out[k] = v[k];
            }
        };
        dispatch_degree<MAXM>(mt.deg, body);
    });
}

template <int MAXM, typename In, int U>
__global__ void __launch_bounds__(256)
    k_refine(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W,
             int mis) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    constexpr int stride = nacc(MAXM);
    constexpr int rl = rec_len(MAXM);
    if (is_single(d)) {
        const double* r = w.rec;
        const bool ok = w.pstatus[0] == LSEFIT_OK;
        const double c = r[0];
        const double inv_s = 1.0 / r[1];
        auto body = [&]<int M>() {
            double v[M + 1];
#pragma unroll
            for (int k = 0; k <= M; ++k) v[k] = 0.0;
            if (ok) {
                AccRefine<M> acc;
                acc.init(c, inv_s, r + rec_b(MAXM));
                stream_strided<U>(x, y, d.n_single, mis, wave, W, acc);
#pragma unroll
                for (int k = 0; k <= M; ++k) v[k] = wave_sum(acc.R[k]);
            }
            single_block_partial<M + 1, stride>(w, v);
        };
        dispatch_degree<MAXM>(d.degree, body);
        return;
    }
    walk_segments_ahead(d, w.tile_start, w.pstatus, w.rec, rl, wave, W,
                        [&](int64_t f, int64_t lo, int64_t hi, int64_t slot, const SegMeta& mt) {
        if (mt.st != LSEFIT_OK) return;
        const double* r = w.rec + f * rl;
        const double c = mt.c;
        const double inv_s = 1.0 / mt.s;
        double* __restrict__ out = w.part + slot * stride;
        auto body = [&]<int M>() {
            AccRefine<M> acc;
            acc.init(c, inv_s, r + rec_b(MAXM));
            stream_segment<U>(x, y, lo, hi, mis, acc);
            double v[M + 1];
#pragma unroll
            for (int k = 0; k <= M; ++k) v[k] = wave_sum(acc.R[k]);
            if (lane_id() == 0) {
#pragma unroll
                for (int k = 0; k <= M; ++k) out[k] = v[k];
            }
        };
        dispatch_degree<MAXM>(mt.deg, body);
    });
}

template <int MAXM>
__global__ void __launch_bounds__(256) k_combine_lane(FitDesc d, Work w, int64_t W, Finish fz) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch) return;
    constexpr int stride = nacc(MAXM);
    constexpr int rl = rec_len(MAXM);
    // the loads that depend on no other, issued together: status, degree, tile
    // range, point count and the range from the record
    const int pst = w.pstatus[f];
    const int deg = fit_deg(d, f);
    const int64_t NT = w.tile_start[d.batch];
    const int64_t ts = w.tile_start[f], te = w.tile_start[f + 1];
    const int64_t n = fit_hi(d, f) - fit_lo(d, f);
    const double c = w.rec[f * rl], s = w.rec[f * rl + 1];
    if (pst != LSEFIT_OK) {
        if (fz.mode != kMomentsOnly) fail_fit<MAXM>(d, w, f, fz, pst);
        return;
    }
    const int64_t w0 = wave_of_tile(ts, NT, W), w1 = wave_of_tile(te - 1, NT, W);
    // the sums of the largest degree's count, whatever this fit's degree: a
    // degree-m fit's sums are the first ones of its slots, and the loads then
    // sit outside the degree switch, so that a wave of mixed degrees waits for
    // its partial sums once
    double all[stride];
#pragma unroll
    for (int k = 0; k < stride; ++k) all[k] = 0.0;
    dispatch_sum_count<MAXM>(fz.mode, [&]<int NK>() {
        for (int64_t wv = w0; wv <= w1; ++wv) {
            if (!wave_owns_tiles(wv, NT, W)) continue;
            const double* p = w.part + (wv + f) * stride;
#pragma unroll
            for (int k = 0; k < NK; ++k) all[k] += p[k];
        }
    });
    auto body = [&]<int M>() {
        constexpr int K = nacc(M);
        const int nk = fz.mode == kRefine ? M + 1 : (fz.mode == kSSE ? 1 : K);
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = k < nk ? all[k] : 0.0;
        finish_fit<M, MAXM>(d, w, f, v, fz, n, c, s);
    };
    dispatch_degree<MAXM>(deg, body);
}

constexpr int kCombineThreads = 256;

template <int MAXM>
__global__ void __launch_bounds__(kCombineThreads) k_combine_block(FitDesc d, Work w, int64_t W, Finish fz) {
    const KernelClock kclock_(w.clock);
    for (int64_t f = blockIdx.x; f < d.batch; f += gridDim.x) block_combine_fit<MAXM>(d, w, f, W, fz);
}

template <int M, int MAXM>
__global__ void k_solve_moments(const double* __restrict__ mom, Work w, int solver, double* coef, int32_t* status) {
    const KernelClock kclock_(w.clock);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int N = M + 1;
    constexpr int rl = rec_len(MAXM);
    double* r = w.rec;
    const double c = mom[0], s = mom[1];
    double S[2 * M + 1], T[1][N], b[1][N], a[N];
#pragma unroll
    for (int k = 0; k <= 2 * M; ++k) S[k] = mom[2 + k];
#pragma unroll
    for (int j = 0; j < N; ++j) T[0][j] = mom[3 + 2 * M + j];
    r[0] = c;
    r[1] = s;
#pragma unroll
    for (int k = 0; k <= 2 * M; ++k) r[rec_S(MAXM) + k] = S[k];
#pragma unroll
    for (int j = 0; j < N; ++j) r[rec_T(MAXM) + j] = T[0][j];
    int st = (s > 0.0 && isfinite(c) && isfinite(s)) ? normal_solve<N, 1>(solver, S, T, b) : LSEFIT_ERR_NONFINITE;
    if (st == LSEFIT_OK) {
        to_x_basis<N>(b[0], c, s, a);
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (!isfinite(a[k])) st = LSEFIT_ERR_NONFINITE;
    }
    if (st != LSEFIT_OK) {
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = b[0][k] = NAN;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        r[rec_b(MAXM) + k] = b[0][k];
        coef[k] = a[k];
        coef[N + k] = b[0][k];
    }
    (void)rl;
    w.pstatus[0] = st;
    status[0] = st;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// largest degree for which the adjoint walk solves for lambda itself (above it,
// the solve's registers would cost the walk occupancy)
constexpr int kAdjointSolveInStream = 3;

template <int MAXM>
__global__ void __launch_bounds__(256)
    k_adjoint_solve(FitDesc d, Work w, int solver, const double* __restrict__ gcoef, int32_t coef_stride) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch) return;
    constexpr int rl = rec_len(MAXM);
    double* r = w.rec + f * rl;
    // every load at once, one memory round trip: status, degree, range, and the
    // power sums and dL/da at the largest degree's size (the record holds
    // 2 MAXM + 1 sums and coef_stride >= MAXM + 1; a lower degree uses the first)
    const int pst = w.pstatus[f];
    const int deg = fit_deg(d, f);
    const double c = r[0], s = r[1];
    double gall[MAXM + 1], Sall[2 * MAXM + 1];
#pragma unroll
    for (int k = 0; k <= MAXM; ++k) gall[k] = gcoef[f * (int64_t)coef_stride + k];
#pragma unroll
    for (int k = 0; k <= 2 * MAXM; ++k) Sall[k] = r[rec_S(MAXM) + k];
    if (pst != LSEFIT_OK) return;
    auto body = [&]<int M>() {
        constexpr int N = M + 1;
        double g[N], gt[1][N], lam[1][N], S[2 * M + 1];
#pragma unroll
        for (int k = 0; k < N; ++k) g[k] = gall[k];
        to_t_basis_adjoint<N>(g, c, s, gt[0]);
#pragma unroll
        for (int k = 0; k <= 2 * M; ++k) S[k] = Sall[k];
        const int st = normal_solve<N, 1>(solver, S, gt, lam);
#pragma unroll
        for (int k = 0; k < N; ++k) r[rec_lam(MAXM) + k] = st == LSEFIT_OK ? lam[0][k] : NAN;
    };
    dispatch_degree<MAXM>(deg, body);
}

template <int M, typename In>
struct AdjointPoint {
    double b[M + 1], lam[M + 1];
    double inv_s, nc;
    template <int MAXM_>
    __device__ inline void init(double c, double s, const double (&bb)[MAXM_ + 1], const double (&ll)[MAXM_ + 1]) {
        inv_s = 1.0 / s;
        nc = -c * inv_s;
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            b[j] = bb[j];
            lam[j] = ll[j];
        }
    }
    __device__ inline void point(double xv, double yv, In& gx, In& gy) const {
        const double t = fma(xv, inv_s, nc);
        double f = b[M], df = 0.0, q = lam[M], dq = 0.0;
#pragma unroll
        for (int j = M - 1; j >= 0; --j) {
            df = fma(df, t, f);
            f = fma(f, t, b[j]);
            dq = fma(dq, t, q);
            q = fma(q, t, lam[j]);
        }
        const double rr = yv - f;
        gx = (In)((dq * rr - q * df) * inv_s);
        gy = (In)q;
    }
};

// dL/dx and dL/dy of the points [lo, hi) of one fit through the point rule P
// (P.point(x, y, gx, gy)), streamed by the waves of one block together: lane
// `first` (in 16-byte vectors: wave-in-block * 64 + lane) takes every
// `step`-th vector (waves per block * 64), so that the block walks one
// contiguous stream; U vectors of x and y per lane are loaded before any is
// used.  The unaligned head and the ragged tail go to the block's first wave
// (edge).
template <int U, typename In, class PT>
__device__ inline void adjoint_segment(const PT& P, const In* __restrict__ x, const In* __restrict__ y,
                                       In* __restrict__ gx, In* __restrict__ gy, int64_t lo, int64_t hi, int mis,
                                       int64_t first, int64_t step, bool edge) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    if (mis >= 0) {
        int64_t a = lo + (int64_t)((VW - (int)((lo + mis) % VW)) % VW);
        if (a > hi) a = hi;
        const int64_t nv = (hi - a) / VW;
        const int64_t b = a + nv * VW;
        if (edge && lane < a - lo) P.point((double)x[lo + lane], (double)y[lo + lane], gx[lo + lane], gy[lo + lane]);
        const V* xv = reinterpret_cast<const V*>(x + a);
        const V* yv = reinterpret_cast<const V*>(y + a);
        V* gxv = reinterpret_cast<V*>(gx + a);
        V* gyv = reinterpret_cast<V*>(gy + a);
        auto vec = [&](const V& xs, const V& ys, int64_t j) {
            V ox, oy;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                In gxe, gye;
                P.point((double)xs[e], (double)ys[e], gxe, gye);
                ox[e] = gxe;
                oy[e] = gye;
            }
            __builtin_nontemporal_store(ox, gxv + j);
            __builtin_nontemporal_store(oy, gyv + j);
        };
        int64_t j = first;
        for (; j + (int64_t)(U - 1) * step < nv; j += (int64_t)U * step) {
            V xs[U], ys[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xs[u] = ld_stream(xv + j + u * step);
                ys[u] = ld_stream(yv + j + u * step);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) vec(xs[u], ys[u], j + u * step);
        }
        for (; j < nv; j += step) vec(ld_stream(xv + j), ld_stream(yv + j), j);
        if (edge && lane < hi - b) P.point((double)x[b + lane], (double)y[b + lane], gx[b + lane], gy[b + lane]);
    } else {
        for (int64_t i = lo + first; i < hi; i += step) P.point((double)x[i], (double)y[i], gx[i], gy[i]);
    }
}

// fits whose status is not OK get NaN gradients (the block's lanes take turns)
template <typename In>
__device__ inline void adjoint_nan(In* __restrict__ gx, In* __restrict__ gy, int64_t lo, int64_t hi, int64_t first,
                                   int64_t step) {
    for (int64_t i = lo + first; i < hi; i += step) {
        gx[i] = (In)NAN;
        gy[i] = (In)NAN;
    }
}

// What the adjoint walk reads of one fit: its tiles, points, status, degree,
// range, b and lambda -- or, when the walk solves for lambda itself (SOLVE),
// dL/da and the power sums instead of lambda.
template <int MAXM, bool SOLVE>
struct AdjMeta {
    int64_t fs, fe, lo, hi;
    double c, s;
    double b[MAXM + 1], lam[MAXM + 1];
    double g[SOLVE ? MAXM + 1 : 1], S[SOLVE ? 2 * MAXM + 1 : 1];
    int st, deg;
};

template <int MAXM, bool SOLVE>
__device__ inline AdjMeta<MAXM, SOLVE> load_adj_meta(const FitDesc& d, const Work& w, int64_t f,
                                                     const double* __restrict__ gcoef, int32_t coef_stride) {
    constexpr int rl = rec_len(MAXM);
    AdjMeta<MAXM, SOLVE> m;
    m.fs = w.tile_start[f];
    m.fe = w.tile_start[f + 1];
    m.lo = fit_lo(d, f);
    m.hi = fit_hi(d, f);
    m.st = w.pstatus[f];
    m.deg = fit_deg(d, f);
    const double* r = w.rec + f * rl;
    m.c = r[0];
    m.s = r[1];
    // entries past the fit's degree are read but not used (the record holds the
    // largest degree's sizes, and coef_stride >= MAXM + 1)
#pragma unroll
    for (int j = 0; j <= MAXM; ++j) m.b[j] = r[rec_b(MAXM) + j];
    if constexpr (SOLVE) {
#pragma unroll
        for (int j = 0; j <= MAXM; ++j) m.g[j] = gcoef[f * (int64_t)coef_stride + j];
#pragma unroll
        for (int k = 0; k <= 2 * MAXM; ++k) m.S[k] = r[rec_S(MAXM) + k];
    } else {
#pragma unroll
        for (int j = 0; j <= MAXM; ++j) m.lam[j] = r[rec_lam(MAXM) + j];
    }
    return m;
}

// lambda = A_t^-1 M^T dL/da of a fit of degree M from its loaded dL/da and power
// sums: the operations of k_adjoint_solve, so the same bits.  NaN when the solve
// fails.
template <int M, int MAXM>
__device__ inline void adjoint_lambda(int solver, const AdjMeta<MAXM, true>& m, double (&lam)[MAXM + 1]) {
    constexpr int N = M + 1;
    double g[N], gt[1][N], l[1][N], S[2 * M + 1];
#pragma unroll
    for (int k = 0; k < N; ++k) g[k] = m.g[k];
    to_t_basis_adjoint<N>(g, m.c, m.s, gt[0]);
#pragma unroll
    for (int k = 0; k <= 2 * M; ++k) S[k] = m.S[k];
    const int st = normal_solve<N, 1>(solver, S, gt, l);
#pragma unroll
    for (int k = 0; k <= MAXM; ++k) lam[k] = k < N ? (st == LSEFIT_OK ? l[0][k] : NAN) : 0.0;
}

// The adjoint pass has no per-wave partial sums, so its tiles go to blocks, not
// waves: block k takes tiles floor(k NT / K) .. floor((k+1) NT / K) - 1 of the
// forward's tile table (K blocks) and streams each fit inside that range as
// one segment, its waves together (adjoint_segment).  The next fit's record is
// loaded before the current segment is streamed.
//
// SOLVE: no separate solve launch before this one -- the walk loads dL/da and
// the power sums with the record and solves for lambda itself when the fit's
// turn comes (every block that streams part of the fit, with the same
// operations, so the same bits); the block that holds the fit's first tile
// writes lambda to the record.
template <int MAXM, typename In, int U, bool SOLVE>
__global__ void __launch_bounds__(256)
    k_adjoint_stream(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, In* __restrict__ gx,
                     In* __restrict__ gy, int64_t W, int mis, int solver, const double* __restrict__ gcoef,
                     int32_t coef_stride) {
    const KernelClock kclock_(w.clock);
    (void)W;
    const int64_t K = gridDim.x;
    const int64_t NT = w.tile_start[d.batch];
    const int64_t tile = w.tile_start[d.batch + 1];
    const int64_t t0 = (int64_t)blockIdx.x * NT / K;
    const int64_t t1 = ((int64_t)blockIdx.x + 1) * NT / K;
    if (t0 >= t1) return;
    const int64_t first = (int64_t)wave_id_in_block() * kWave + lane_id();
    const int64_t step = (int64_t)(blockDim.x / kWave) * kWave;
    const bool edge = wave_id_in_block() == 0;
    int64_t lo = 0, hi = d.batch;   // largest f with tile_start[f] <= t0
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (w.tile_start[mid] <= t0) lo = mid;
        else hi = mid;
    }
    int64_t f = lo;
    AdjMeta<MAXM, SOLVE> cur = load_adj_meta<MAXM, SOLVE>(d, w, f, gcoef, coef_stride);
    int64_t t = t0;
    while (t < t1) {
        if (cur.fe <= t) {   // a fit without tiles
            ++f;
            cur = load_adj_meta<MAXM, SOLVE>(d, w, f, gcoef, coef_stride);
            continue;
        }
        const int64_t te = cur.fe < t1 ? cur.fe : t1;
        const bool more = te < t1;   // then fit f + 1 < B holds the next tile
        AdjMeta<MAXM, SOLVE> nxt = cur;
        if (more) nxt = load_adj_meta<MAXM, SOLVE>(d, w, f + 1, gcoef, coef_stride);
        const int64_t plo = cur.lo + (t - cur.fs) * tile;
        int64_t phi = cur.lo + (te - cur.fs) * tile;
        if (phi > cur.hi) phi = cur.hi;
        if (cur.st != LSEFIT_OK) {
            adjoint_nan(gx, gy, plo, phi, first, step);
        } else {
            auto body = [&]<int M>() {
                if constexpr (SOLVE) {
                    adjoint_lambda<M, MAXM>(solver, cur, cur.lam);
                    if (t == cur.fs && threadIdx.x == 0) {
                        double* r = w.rec + f * rec_len(MAXM);
#pragma unroll
                        for (int k = 0; k <= M; ++k) r[rec_lam(MAXM) + k] = cur.lam[k];
                    }
                }
                AdjointPoint<M, In> P;
                P.template init<MAXM>(cur.c, cur.s, cur.b, cur.lam);
                adjoint_segment<U>(P, x, y, gx, gy, plo, phi, mis, first, step, edge);
            };
            dispatch_degree<MAXM>(cur.deg, body);
        }
        t = te;
        ++f;
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// residual pass (Table V of Sec. III): e = y - f(t), f = sum_j b_j t^j in
// float64, optionally stored; partial sums of e^2 as in the power-sum pass
// ---------------------------------------------------------------------------
template <int M>
struct ResidPoint {
    double b[M + 1];
    double inv_s, nc;
    __device__ inline void init(const double* r, int MAXM_) {
        inv_s = 1.0 / r[1];
        nc = -r[0] * inv_s;
#pragma unroll
        for (int j = 0; j <= M; ++j) b[j] = r[rec_b(MAXM_) + j];
    }
    __device__ inline double err(double xv, double yv) const {
        const double t = fma(xv, inv_s, nc);
        double f = b[M];
#pragma unroll
        for (int j = M - 1; j >= 0; --j) f = fma(f, t, b[j]);
        return yv - f;
    }
};

// one wave: points [lo, hi) of one fit (or the whole grid-stride share of a
// single fit when `strided`), e^2 summed per lane into acc, e stored if resid
template <class PT, typename In, bool STRIDED, int U>
__device__ inline void resid_points(const In* __restrict__ x, const In* __restrict__ y, In* __restrict__ resid,
                                    int64_t lo, int64_t hi, int mis, int64_t gwave, int64_t W,
                                    const PT& P, double& acc) {
    constexpr int VW = VecOf<In>::W;
    using V = typename VecOf<In>::type;
    const int lane = lane_id();
    const int64_t step = STRIDED ? W * kWave : kWave;
    const int64_t first = STRIDED ? gwave * kWave + lane : lane;
    const bool edge_wave = STRIDED ? gwave == 0 : true;
    auto one = [&](int64_t i) {
        const double e = P.err((double)x[i], (double)y[i]);
        acc = fma(e, e, acc);
        if (resid) resid[i] = (In)e;
    };
    if (mis >= 0) {
        int64_t a = lo + (int64_t)((VW - (int)((lo + mis) % VW)) % VW);
        if (a > hi) a = hi;
        const int64_t nv = (hi - a) / VW;
        const int64_t b = a + nv * VW;
        if (edge_wave && lane < a - lo) one(lo + lane);
        const V* xv = reinterpret_cast<const V*>(x + a);
        const V* yv = reinterpret_cast<const V*>(y + a);
        V* rv = resid ? reinterpret_cast<V*>(resid + a) : nullptr;
        auto vec = [&](const V& xs, const V& ys, int64_t j) {
            V os;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const double er = P.err((double)xs[e], (double)ys[e]);
                acc = fma(er, er, acc);
                os[e] = (In)er;
            }
            if (rv) __builtin_nontemporal_store(os, rv + j);
        };
        // U vectors per lane are loaded before any is used (U rounds of loads in flight)
        int64_t j = first;
        for (; j + (int64_t)(U - 1) * step < nv; j += (int64_t)U * step) {
            V xs[U], ys[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xs[u] = ld_stream(xv + j + u * step);
                ys[u] = ld_stream(yv + j + u * step);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) vec(xs[u], ys[u], j + u * step);
        }
        for (; j < nv; j += step) vec(ld_stream(xv + j), ld_stream(yv + j), j);
        if (edge_wave && lane < hi - b) one(b + lane);
    } else {
        for (int64_t i = lo + first; i < hi; i += step) one(i);
    }
}

template <int MAXM, typename In, int U>
__global__ void __launch_bounds__(256)
    k_residual(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, In* __restrict__ resid,
               int64_t W, int mis) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    constexpr int stride = nacc(MAXM);
    constexpr int rl = rec_len(MAXM);
    if (is_single(d)) {
        const bool ok = w.pstatus[0] == LSEFIT_OK;
        auto body = [&]<int M>() {
            double acc = 0.0;
            if (ok) {
                ResidPoint<M> P;
                P.init(w.rec, MAXM);
                resid_points<ResidPoint<M>, In, true, U>(x, y, resid, 0, d.n_single, mis, wave, W, P, acc);
            } else if (resid) {
                for (int64_t i = wave * kWave + lane_id(); i < d.n_single; i += W * kWave) resid[i] = (In)NAN;
            }
            double v[1] = {wave_sum(acc)};
            single_block_partial<1, stride>(w, v);
        };
        dispatch_degree<MAXM>(d.degree, body);
        return;
    }
    walk_segments(d, w.tile_start, wave, W, [&](int64_t f, int64_t lo, int64_t hi, int64_t slot) {
        if (w.pstatus[f] != LSEFIT_OK) {
            if (resid)
                for (int64_t i = lo + lane_id(); i < hi; i += kWave) resid[i] = (In)NAN;
            return;
        }
        auto body = [&]<int M>() {
            ResidPoint<M> P;
            P.init(w.rec + f * rl, MAXM);
            double acc = 0.0;
            resid_points<ResidPoint<M>, In, false, U>(x, y, resid, lo, hi, mis, 0, W, P, acc);
            acc = wave_sum(acc);
            if (lane_id() == 0) w.part[slot * stride] = acc;
        };
        dispatch_degree<MAXM>(fit_deg(d, f), body);
    });
}

// ---------------------------------------------------------------------------
// per-degree launchers (explicitly instantiated once per largest degree)
// ---------------------------------------------------------------------------
inline int64_t blocks_for(const Launch& L) { return (L.waves + L.wpb - 1) / L.wpb; }

template <int MAXM>
template <int PREC, typename In>
hipError_t Launchers<MAXM>::moments_t(const FitDesc& d, const Work& w, const void* x, const void* y,
                                      const Launch& L, int mis, const RangeArg& ra, hipStream_t st) {
    const dim3 grid(blocks_for(L)), block(L.wpb * kWave);
    const In* xx = (const In*)x;
    const In* yy = (const In*)y;
    switch (L.unroll) {
        case 1: launch_timed((k_moments<MAXM, PREC, In, 1>), grid, block, st, d, w, xx, yy, L.waves, mis, ra); break;
        case 2: launch_timed((k_moments<MAXM, PREC, In, 2>), grid, block, st, d, w, xx, yy, L.waves, mis, ra); break;
        case 4: launch_timed((k_moments<MAXM, PREC, In, 4>), grid, block, st, d, w, xx, yy, L.waves, mis, ra); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MAXM>
hipError_t Launchers<MAXM>::moments(const FitDesc& d, const Work& w, int prec, int dtype, const void* x,
                                    const void* y, const Launch& L, int mis, const RangeArg& ra, hipStream_t st) {
    if (prec == LSEFIT_PREC_F64 && dtype == LSEFIT_F64)
        return moments_t<LSEFIT_PREC_F64, double>(d, w, x, y, L, mis, ra, st);
    if (prec == LSEFIT_PREC_F64 && dtype == LSEFIT_F32)
        return moments_t<LSEFIT_PREC_F64, float>(d, w, x, y, L, mis, ra, st);
    if (prec == LSEFIT_PREC_F32C && dtype == LSEFIT_F32)
        return moments_t<LSEFIT_PREC_F32C, float>(d, w, x, y, L, mis, ra, st);
    return hipErrorInvalidValue;
}

template <int MAXM>
hipError_t Launchers<MAXM>::combine(const FitDesc& d, const Work& w, const Launch& L, bool by_block, const Finish& fz,
                                    hipStream_t st) {
    if (by_block) {
        int64_t blocks = d.batch < 65536 ? d.batch : 65536;
        if (blocks < 1) blocks = 1;
        launch_timed(k_combine_block<MAXM>, dim3(blocks), dim3(kCombineThreads), st, d, w, L.waves, fz);
    } else {
        const int64_t blocks = (d.batch + 255) / 256;
        launch_timed(k_combine_lane<MAXM>, dim3(blocks > 0 ? blocks : 1), dim3(256), st, d, w, L.waves, fz);
    }
    return hipGetLastError();
}

template <int MAXM>
hipError_t Launchers<MAXM>::finish_single(const FitDesc& d, const Work& w, int64_t G, const Finish& fz, hipStream_t st) {
    launch_timed(k_finish_single<MAXM>, dim3(1), dim3(kFinishWaves * kWave), st, d, w, G, fz);
    return hipGetLastError();
}

template <int MAXM>
hipError_t Launchers<MAXM>::solve_moments(const double* moments, const Work& w, int m, int solver, double* coef,
                                          int32_t* status, hipStream_t st) {
    switch (m) {
#define LSEFIT_SOLVE_CASE(MV)                                                                                   \
    case MV:                                                                                                    \
        if constexpr (MV <= MAXM) {                                                                             \
            launch_timed((k_solve_moments<MV, MAXM>), dim3(1), dim3(64), st, moments, w, solver, coef, status); \
            return hipGetLastError();                                                                           \
        }                                                                                                       \
        break;
        LSEFIT_SOLVE_CASE(1)
        LSEFIT_SOLVE_CASE(2)
        LSEFIT_SOLVE_CASE(3)
        LSEFIT_SOLVE_CASE(4)
        LSEFIT_SOLVE_CASE(5)
        LSEFIT_SOLVE_CASE(6)
        LSEFIT_SOLVE_CASE(7)
        LSEFIT_SOLVE_CASE(8)
#undef LSEFIT_SOLVE_CASE
        default: break;
    }
    return hipErrorInvalidValue;
}

template <int MAXM>
template <typename In>
hipError_t Launchers<MAXM>::refine_t(const FitDesc& d, const Work& w, const void* x, const void* y, const Launch& L,
                                     int mis, hipStream_t st) {
    const dim3 grid(blocks_for(L)), block(L.wpb * kWave);
    const In* xx = (const In*)x;
    const In* yy = (const In*)y;
    switch (L.unroll) {
        case 1: launch_timed((k_refine<MAXM, In, 1>), grid, block, st, d, w, xx, yy, L.waves, mis); break;
        case 2: launch_timed((k_refine<MAXM, In, 2>), grid, block, st, d, w, xx, yy, L.waves, mis); break;
        case 4: launch_timed((k_refine<MAXM, In, 4>), grid, block, st, d, w, xx, yy, L.waves, mis); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MAXM>
hipError_t Launchers<MAXM>::refine(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y,
                                   const Launch& L, int mis, hipStream_t st) {
    return dtype == LSEFIT_F32 ? refine_t<float>(d, w, x, y, L, mis, st) : refine_t<double>(d, w, x, y, L, mis, st);
}

template <int MAXM>
hipError_t Launchers<MAXM>::adjoint(const FitDesc& d, const Work& w, int solver, int dtype, const void* x,
                                    const void* y, const double* grad_coef, int32_t coef_stride, void* gx, void* gy,
                                    const Launch& L, int mis, hipStream_t st) {
    // up to kAdjointSolveInStream the walk solves for lambda itself (one launch);
    // above it a thread per fit solves first, and the walk reads lambda
    constexpr bool solve_in_stream = MAXM <= kAdjointSolveInStream;
    if constexpr (!solve_in_stream) {
        const int64_t sblocks = (d.batch + 255) / 256;
        hipLaunchKernelGGL(k_adjoint_solve<MAXM>, dim3(sblocks > 0 ? sblocks : 1), dim3(256), 0, st, d, w, solver,
                           grad_coef, coef_stride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 grid(blocks_for(L)), block(L.wpb * kWave);
#define LSEFIT_ADJ(UU)                                                                                           \
    if (dtype == LSEFIT_F32)                                                                                     \
        launch_timed((k_adjoint_stream<MAXM, float, UU, solve_in_stream>), grid, block, st, d, w, (const float*)x, \
                     (const float*)y, (float*)gx, (float*)gy, L.waves, mis, solver, grad_coef, coef_stride);    \
    else                                                                                                         \
        launch_timed((k_adjoint_stream<MAXM, double, UU, solve_in_stream>), grid, block, st, d, w,              \
                     (const double*)x, (const double*)y, (double*)gx, (double*)gy, L.waves, mis, solver,       \
                     grad_coef, coef_stride);
    switch (L.unroll) {
        case 1: LSEFIT_ADJ(1) break;
        case 2: LSEFIT_ADJ(2) break;
        case 4: LSEFIT_ADJ(4) break;
        default: return hipErrorInvalidValue;
    }
#undef LSEFIT_ADJ
    return hipGetLastError();
}

template <int MAXM>
hipError_t Launchers<MAXM>::residual(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y,
                                     void* resid, const Launch& L, int mis, hipStream_t st) {
    const dim3 grid(blocks_for(L)), block(L.wpb * kWave);
#define LSEFIT_RES(UU)                                                                                           \
    if (dtype == LSEFIT_F32)                                                                                     \
        launch_timed((k_residual<MAXM, float, UU>), grid, block, st, d, w, (const float*)x,            \
                           (const float*)y, (float*)resid, L.waves, mis);                                \
    else                                                                                                         \
        launch_timed((k_residual<MAXM, double, UU>), grid, block, st, d, w, (const double*)x,          \
                           (const double*)y, (double*)resid, L.waves, mis);
    switch (L.unroll) {
        case 1: LSEFIT_RES(1) break;
        case 2: LSEFIT_RES(2) break;
        case 4: LSEFIT_RES(4) break;
        default: return hipErrorInvalidValue;
    }
#undef LSEFIT_RES
    return hipGetLastError();
}

}  // namespace lsefit
