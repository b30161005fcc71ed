// Device-side building blocks of the moment-pass least-squares fit (gfx950).
//
// Everything here runs inside the kernels (kernels_impl.hpp, dispatch.hip): the per-fit table
// of CSR segments, the balanced tile walk of the persistent streaming grid,
// the wave-level float64 reduction, the range map (c, s), elimination with
// partial pivoting on the Hankel normal matrix and the change of basis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lsefit.h"

namespace lsefit {

constexpr int kWave = 64;
constexpr int kMaxDeg = LSEFIT_MAX_DEGREE;

// Per-wave partial sums of one degree-m segment: S_1..S_2m then T_0..T_m.
__host__ __device__ constexpr int nacc(int m) { return 3 * m + 1; }
// flat length of a streaming QR factor of degree m: d, th (m+1 each), the strict
// upper triangle of the unit factor, the residual sum of squares
__host__ __device__ constexpr int qr_len(int m) { return 2 * (m + 1) + m * (m + 1) / 2 + 1; }

// Per-fit record kept in the workspace (float64 slots), for a call whose
// largest degree is M:
//   [0] c   [1] s   [2 .. 2+2M] S_0..S_2M   [3+2M .. 3+3M] T_0..T_M
//   [4+3M .. 4+4M] b_0..b_M (t-basis solution)   [5+4M .. 5+5M] lambda_0..lambda_M
__host__ __device__ constexpr int rec_len(int M) { return 6 + 5 * M; }
__host__ __device__ constexpr int rec_S(int) { return 2; }
__host__ __device__ constexpr int rec_T(int M) { return 3 + 2 * M; }
__host__ __device__ constexpr int rec_b(int M) { return 4 + 3 * M; }
__host__ __device__ constexpr int rec_lam(int M) { return 5 + 4 * M; }

// The fits of one call: CSR offsets (NULL for a single fit of n_single
// points) and per-fit degrees (NULL for one degree for all).
struct FitDesc {
    const int64_t* offsets;
    const int32_t* degrees;
    int64_t n_single;
    int64_t batch;
    int32_t degree;   // uniform degree, or the largest degree allowed
};

__host__ __device__ inline bool is_single(const FitDesc& d) { return d.offsets == nullptr; }

__device__ inline int64_t fit_lo(const FitDesc& d, int64_t f) { return d.offsets ? d.offsets[f] : 0; }
__device__ inline int64_t fit_hi(const FitDesc& d, int64_t f) { return d.offsets ? d.offsets[f + 1] : d.n_single; }
__device__ inline int fit_deg(const FitDesc& d, int64_t f) { return d.degrees ? d.degrees[f] : d.degree; }

// Workspace regions (device pointers carved out of the caller's buffer).
struct Work {
    int64_t* tile_start = nullptr;  // [B+2] first tile of each fit; tile_start[B] = number of tiles,
                                    // tile_start[B+1] = points per tile
    int32_t* pstatus = nullptr;     // [B] status found while building the tile table
    double* rec = nullptr;          // [B * rec_len(M)]
    double* part = nullptr;         // [(W + B) * nacc(M)] per-(wave, fit) partial sums (batched) or
                                    // per-block partial sums (single fit; [W * max(nacc, qr_len)])
    int64_t* block_tot = nullptr;   // [ceil(B / kPlanThreads)] tile totals of the tile-table blocks
    uint64_t* clock = nullptr;      // [2] start and end of this launch (KernelClock); null unless
                                    // launch_timed arms the launch
};

// threads per block of the tile-table kernels (one thread per fit); the
// workspace holds one tile total per such block
constexpr int kPlanThreads = 256;

// ---------------------------------------------------------------------------
// wave-level reductions.  The float64 sum runs on DPP lane moves (CDNA keeps the
// GFX9 row broadcasts): pairs, quads, half rows and rows combine by mirrored
// moves, so every lane of a row holds the same row sum; two masked row
// broadcasts then fold rows 0..3 into lane 63, which is read back for all lanes.
// The pattern is fixed, so the result is the same bits on every run.  Every
// lane of the wave must be active.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_sum(double v) {
    v += dpp_f64<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xf>(v);   // row_half_mirror
    v += dpp_f64<0x140, 0xf>(v);   // row_mirror
    v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// the same DPP pattern for min and max; lanes of rows outside a row mask
// receive their own value (min and max have no zero to fall back on)
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64_keep(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false));
}

template <bool MAX>
__device__ inline double wave_extreme(double v) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
    v = op(v, dpp_f64_keep<0xb1, 0xf>(v));
    v = op(v, dpp_f64_keep<0x4e, 0xf>(v));
    v = op(v, dpp_f64_keep<0x141, 0xf>(v));
    v = op(v, dpp_f64_keep<0x140, 0xf>(v));
    v = op(v, dpp_f64_keep<0x142, 0xa>(v));
    v = op(v, dpp_f64_keep<0x143, 0xc>(v));
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
__device__ inline double wave_min(double v) { return wave_extreme<false>(v); }
__device__ inline double wave_max(double v) { return wave_extreme<true>(v); }

__device__ inline int wave_id_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }
__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

// ---------------------------------------------------------------------------
// kernel clock (lsefit_timing_*): when a launch carries a clock slot, the first
// thread of block 0 (the first block the dispatcher starts) stores the
// device's constant-rate wall clock into slot[0] when it starts, and the first
// active lane of every wave folds the clock into one of kClockLines separate
// 64-byte lines with an atomic maximum when it leaves the kernel (wave w uses
// line w mod kClockLines, word 1, so that no line takes more than
// 1/kClockLines of the atomics); the launch's duration is then the largest
// end over the lines minus the start.  Without a slot (the normal case) it
// costs one uniform branch at each end.
// ---------------------------------------------------------------------------
constexpr int kClockLines = 32;
constexpr int kClockWords = 8 * kClockLines;   // uint64 words per slot

struct KernelClock {
    uint64_t* slot;
    __device__ explicit KernelClock(uint64_t* s) : slot(s) {
        if (slot && blockIdx.x == 0 && threadIdx.x == 0) slot[0] = wall_clock64();
    }
    __device__ ~KernelClock() {
        if (slot) {
            const uint64_t active = __ballot(1);
            if (lane_id() == __ffsll((unsigned long long)active) - 1) {
                const unsigned w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
                atomicMax((unsigned long long*)(slot + 8 * (w % kClockLines) + 1),
                          (unsigned long long)wall_clock64());
            }
        }
    }
};
// the clock slot of kernels that take no workspace (the bandwidth probes)
struct KClock {
    uint64_t* slot;
};

// ---------------------------------------------------------------------------
// range map: (c, s) from the sampled extremes of x.  s is the power of two at
// or above the half-range; c is the mid-range on a grid of s/8 (0 when small
// against the half-range), rounded to float32 so that x - c is formed the same
// way by float32 and float64 passes.  Any (c, s) gives the same minimiser.
// ---------------------------------------------------------------------------
__device__ inline void snap_range(double lo, double hi, double* c_out, double* s_out) {
    if (!(lo <= hi)) {  // no finite sample
        *c_out = 0.0;
        *s_out = 1.0;
        return;
    }
    double half = 0.5 * hi - 0.5 * lo;
    double mid = 0.5 * hi + 0.5 * lo;
    double s = 1.0, c = mid;
    if (half > 0.0) {
        int e;
        double f = frexp(half, &e);      // half = f 2^e, f in [0.5, 1)
        s = ldexp(1.0, f == 0.5 ? e - 1 : e);
        double q = ldexp(s, -3);
        c = fabs(mid) < ldexp(half, -6) ? 0.0 : rint(mid / q) * q;
    }
    *c_out = (double)(float)c;
    *s_out = s;
}

// ---------------------------------------------------------------------------
// the balanced tile walk of the persistent grid.  Fit f owns tiles
// tile_start[f] .. tile_start[f+1]-1 (tile points each, the last one ragged);
// wave w owns tiles floor(w NT / W) .. floor((w+1) NT / W) - 1 and streams the
// part of each fit inside that range as one segment.  (w, f) pairs that share
// a tile map one-to-one onto partial slots w + f.  NT = tile_start[B] and the
// tile size the table was built with, tile_start[B+1], are read from the table
// itself, so a later pass over the same workspace (the adjoint, the residuals)
// cuts every fit where the forward pass did, whatever its own launch shape.
// ---------------------------------------------------------------------------
template <class Fn>
__device__ inline void walk_segments(const FitDesc& d, const int64_t* __restrict__ tile_start, int64_t wave,
                                     int64_t W, Fn&& fn) {
    const int64_t NT = tile_start[d.batch];
    const int64_t tile = tile_start[d.batch + 1];
    const int64_t t0 = wave * NT / W;
    const int64_t t1 = (wave + 1) * NT / W;
    if (t0 >= t1) return;
    int64_t lo = 0, hi = d.batch;   // largest f with tile_start[f] <= t0
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (tile_start[mid] <= t0) lo = mid;
        else hi = mid;
    }
    int64_t f = lo;
    int64_t t = t0;
    while (t < t1) {
        const int64_t fs = tile_start[f], fe = tile_start[f + 1];
        if (fe <= t) {
            ++f;
            continue;
        }
        const int64_t te = fe < t1 ? fe : t1;
        const int64_t base = fit_lo(d, f);
        const int64_t end = fit_hi(d, f);
        const int64_t plo = base + (t - fs) * tile;
        int64_t phi = base + (te - fs) * tile;
        if (phi > end) phi = end;
        fn(f, plo, phi, wave + f);
        t = te;
        ++f;
    }
}

// walk_segments for the passes that need only a fit's range record, status
// and degree: the next fit's metadata is loaded before the current segment is
// streamed, so that its latency overlaps the segment's loads instead of
// following them.  fn(f, lo, hi, slot, meta).
struct SegMeta {
    int64_t fs, fe, lo, hi;   // tiles and points of the fit
    double c, s;              // its range record
    int st, deg;              // its plan status and degree
};

__device__ inline SegMeta load_meta(const FitDesc& d, const int64_t* __restrict__ tile_start,
                                    const int32_t* __restrict__ pstatus, const double* __restrict__ rec, int rl,
                                    int64_t f) {
    SegMeta m;
    m.fs = tile_start[f];
    m.fe = tile_start[f + 1];
    m.lo = fit_lo(d, f);
    m.hi = fit_hi(d, f);
    m.st = pstatus[f];
    m.deg = fit_deg(d, f);
    m.c = rec[f * rl];
    m.s = rec[f * rl + 1];
    return m;
}

template <class Fn>
__device__ inline void walk_segments_ahead(const FitDesc& d, const int64_t* __restrict__ tile_start,
                                           const int32_t* __restrict__ pstatus, const double* __restrict__ rec,
                                           int rl, int64_t wave, int64_t W, Fn&& fn) {
    const int64_t NT = tile_start[d.batch];
    const int64_t tile = tile_start[d.batch + 1];
    const int64_t t0 = wave * NT / W;
    const int64_t t1 = (wave + 1) * NT / W;
    if (t0 >= t1) return;
    int64_t lo = 0, hi = d.batch;   // largest f with tile_start[f] <= t0
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (tile_start[mid] <= t0) lo = mid;
        else hi = mid;
    }
    int64_t f = lo;
    SegMeta cur = load_meta(d, tile_start, pstatus, rec, rl, f);
    int64_t t = t0;
    while (t < t1) {
        if (cur.fe <= t) {   // a fit without tiles (or before t0)
            ++f;
            cur = load_meta(d, tile_start, pstatus, rec, rl, f);
            continue;
        }
        const int64_t te = cur.fe < t1 ? cur.fe : t1;
        const bool more = te < t1;   // then fit f + 1 < B holds the next tile
        SegMeta nxt = cur;
        if (more) nxt = load_meta(d, tile_start, pstatus, rec, rl, f + 1);
        const int64_t plo = cur.lo + (t - cur.fs) * tile;
        int64_t phi = cur.lo + (te - cur.fs) * tile;
        if (phi > cur.hi) phi = cur.hi;
        fn(f, plo, phi, wave + f, cur);
        t = te;
        ++f;
        cur = nxt;
    }
}

// the wave that owns tile t (inverse of the split above)
__device__ inline int64_t wave_of_tile(int64_t t, int64_t NT, int64_t W) { return ((t + 1) * W - 1) / NT; }

// whether wave w owns at least one tile (with more waves than tiles some own none
// and write no partial)
__device__ inline bool wave_owns_tiles(int64_t w, int64_t NT, int64_t W) { return w * NT / W < (w + 1) * NT / W; }

// ---------------------------------------------------------------------------
// Gaussian elimination with partial pivoting on an augmented normal matrix
// [A | B] (Sec. II: A_jk = S_(j+k) in the power basis; the Gram matrix of the
// Chebyshev basis otherwise).  Pivot: first row of largest magnitude.
// Singular when a pivot is at most 2^-40 max|A|.  N = m + 1; several
// right-hand sides are eliminated together.
// ---------------------------------------------------------------------------
template <int N, int R>
__device__ inline int matrix_gepp(double (&A)[N][N + R], double (&X)[R][N]) {
    double amax = 0.0;
    bool finite = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            finite = finite && isfinite(A[j][k]);
            amax = fmax(amax, fabs(A[j][k]));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) finite = finite && isfinite(A[j][N + r]);
    }
    if (!finite) return LSEFIT_ERR_NONFINITE;
    const double tiny = ldexp(amax, -40);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int p = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            double v = fabs(A[r][k]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best > tiny)) return LSEFIT_ERR_SINGULAR;
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            if (r == p) {
#pragma unroll
                for (int c = 0; c < N + R; ++c) {
                    double tmp = A[k][c];
                    A[k][c] = A[r][c];
                    A[r][c] = tmp;
                }
            }
        }
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double l = A[r][k] / A[k][k];
#pragma unroll
            for (int c = k; c < N + R; ++c) A[r][c] -= l * A[k][c];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            double acc = A[i][N + r];
#pragma unroll
            for (int c = i + 1; c < N; ++c) acc -= A[i][c] * X[r][c];
            X[r][i] = acc / A[i][i];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (!isfinite(X[r][i])) return LSEFIT_ERR_NONFINITE;
    return LSEFIT_OK;
}

// Cholesky (L L^T) solve of a normal system A X = B held as an augmented
// matrix (the columns past N are the right-hand sides): A is symmetric
// positive definite when the fit is determined, so no pivoting is needed.
// Singular when a diagonal of the Schur complement is at most 2^-40 max|A|.
template <int N, int R>
__device__ inline int matrix_cholesky(const double (&A)[N][N + R], double (&X)[R][N]) {
    double Lm[N][N];
    double amax = 0.0;
    bool finite = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            finite = finite && isfinite(A[j][k]);
            amax = fmax(amax, fabs(A[j][k]));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) finite = finite && isfinite(A[j][N + r]);
    }
    if (!finite) return LSEFIT_ERR_NONFINITE;
    const double tiny = ldexp(amax, -40);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double dgl = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dgl -= Lm[j][k] * Lm[j][k];
        if (!(dgl > tiny)) return LSEFIT_ERR_SINGULAR;
        const double ljj = sqrt(dgl);
        Lm[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            double acc = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) acc -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = acc / ljj;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double z[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double acc = A[i][N + r];
#pragma unroll
            for (int k = 0; k < i; ++k) acc -= Lm[i][k] * z[k];
            z[i] = acc / Lm[i][i];
        }
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            double acc = z[i];
#pragma unroll
            for (int k = i + 1; k < N; ++k) acc -= Lm[k][i] * X[r][k];
            X[r][i] = acc / Lm[i][i];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (!isfinite(X[r][i])) return LSEFIT_ERR_NONFINITE;
    return LSEFIT_OK;
}

// the Hankel normal system of Sec. II, A_jk = S_(j+k), with R right-hand sides
template <int N, int R>
__device__ inline void hankel_assemble(const double* S, const double (&rhs)[R][N], double (&A)[N][N + R]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int k = 0; k < N; ++k) A[j][k] = S[j + k];
#pragma unroll
        for (int r = 0; r < R; ++r) A[j][N + r] = rhs[r][j];
    }
}

template <int N, int R>
__device__ inline int hankel_solve(const double* S, const double (&rhs)[R][N], double (&X)[R][N]) {
    double A[N][N + R];
    hankel_assemble<N, R>(S, rhs, A);
    return matrix_gepp<N, R>(A, X);
}

template <int N, int R>
__device__ inline int hankel_cholesky(const double* S, const double (&rhs)[R][N], double (&X)[R][N]) {
    double A[N][N + R];
    hankel_assemble<N, R>(S, rhs, A);
    return matrix_cholesky<N, R>(A, X);
}

// the normal-system solve the options ask for
template <int N, int R>
__device__ inline int normal_solve(int solver, const double* S, const double (&rhs)[R][N], double (&X)[R][N]) {
    return solver == LSEFIT_SOLVER_CHOLESKY ? hankel_cholesky<N, R>(S, rhs, X) : hankel_solve<N, R>(S, rhs, X);
}

// t-basis b (t = (x - c)/s) to x-basis a: a_k = sum_{j>=k} b_j C(j,k) (-c)^(j-k) s^-j
template <int N>
__device__ inline void to_x_basis(const double (&b)[N], double c, double s, double (&a)[N]) {
    const double inv_s = 1.0 / s;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double acc = 0.0;
        double binom = 1.0;      // C(j, k), starting at j = k
        double cpow = 1.0;       // (-c)^(j-k)
        double spow = 1.0;       // s^-j
#pragma unroll
        for (int i = 0; i < k; ++i) spow *= inv_s;
#pragma unroll
        for (int j = k; j < N; ++j) {
            acc += b[j] * binom * cpow * spow;
            binom = binom * (double)(j + 1) / (double)(j + 1 - k);
            cpow *= -c;
            spow *= inv_s;
        }
        a[k] = acc;
    }
}

// ---------------------------------------------------------------------------
// solving a normal system with one wave: lane r < N holds row r of [A | rhs]
// in registers; pivot rows and solved unknowns are shared with readlane.
// The same operations, in the same order per entry, as the one-thread
// solvers above.
// ---------------------------------------------------------------------------
__device__ inline double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// v[k] = sh[0][k] + sh[1][k] + ... + sh[nw-1][k] (in that order) in every
// lane of the calling wave: lane k adds column k, readlane shares the sums
// (K <= 64)
template <int K, int S>
__device__ inline void wave_column_sums(const double (*sh)[S], int nw, double (&v)[K]) {
    static_assert(K <= 64 && K <= S, "one lane per sum");
    const int lane = lane_id();
    double t = 0.0;
    if (lane < K) {
        t = sh[0][lane];
        for (int i = 1; i < nw; ++i) t += sh[i][lane];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = bcast(t, k);
}

// orders this wave's LDS writes before its later LDS reads
__device__ inline void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// max |G| over the N x N part held by lanes 0..N-1
template <int M>
__device__ inline double wave_amax(const double (&row)[M + 2]) {
    constexpr int N = M + 1;
    double la = 0.0;
    if (lane_id() < N) {
#pragma unroll
        for (int c = 0; c < N; ++c) la = fmax(la, fabs(row[c]));
    }
    double amax = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) amax = fmax(amax, bcast(la, r));
    return amax;
}

// Partial pivoting (first row of largest magnitude), singular when a pivot is
// at most 2^-40 max|G|; the same operations, in the same order per entry, as an
// elimination by one thread.  On success lane i < N holds x_i in xl.
template <int M>
__device__ __forceinline__ int wave_gepp(double (&row)[M + 2], double& xl) {
    constexpr int N = M + 1;
    const int lane = lane_id();
    const double tiny = ldexp(wave_amax<M>(row), -40);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int p = k;
        double pv = fabs(bcast(row[k], k));
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double v = fabs(bcast(row[k], r));
            if (v > pv) {
                pv = v;
                p = r;
            }
        }
        if (!(pv > tiny)) return LSEFIT_ERR_SINGULAR;
        p = __builtin_amdgcn_readfirstlane(p);
        if (p != k) {
#pragma unroll
            for (int c = k; c <= N; ++c) {
                const double a = bcast(row[c], p), b = bcast(row[c], k);
                if (lane == k) row[c] = a;
                else if (lane == p) row[c] = b;
            }
        }
        const double pk = bcast(row[k], k);
        if (lane > k && lane < N) {
            const double l = row[k] / pk;
#pragma unroll
            for (int c = k; c <= N; ++c) row[c] -= l * bcast(row[c], k);
        }
    }
    xl = 0.0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double acc = row[N];
#pragma unroll
        for (int c = i + 1; c < N; ++c) acc -= row[c] * bcast(xl, c);
        const double xi = bcast(acc / row[i], i);
        if (lane == i) xl = xi;
    }
    return LSEFIT_OK;
}

// G = L L^T (lane r holds row r of L), then L z = D and L^T x = z; lane i < N
// holds x_i in xl
template <int M>
__device__ __forceinline__ int wave_cholesky(const double (&row)[M + 2], double& xl) {
    constexpr int N = M + 1;
    const int lane = lane_id();
    const double tiny = ldexp(wave_amax<M>(row), -40);
    double L[M + 1];
#pragma unroll
    for (int c = 0; c < N; ++c) L[c] = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double dg = bcast(row[j], j);
#pragma unroll
        for (int k = 0; k < j; ++k) {
            const double ljk = bcast(L[k], j);
            dg -= ljk * ljk;
        }
        if (!(dg > tiny)) return LSEFIT_ERR_SINGULAR;
        const double ljj = sqrt(dg);
        if (lane == j) {
            L[j] = ljj;
        } else if (lane > j && lane < N) {
            double acc = row[j];
#pragma unroll
            for (int k = 0; k < j; ++k) acc -= L[k] * bcast(L[k], j);
            L[j] = acc / ljj;
        }
    }
    double zl = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double acc = row[N];
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= L[k] * bcast(zl, k);
        const double zi = bcast(acc / L[i], i);
        if (lane == i) zl = zi;
    }
    xl = 0.0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double acc = bcast(zl, i);
#pragma unroll
        for (int k = i + 1; k < N; ++k) acc -= bcast(L[i], k) * bcast(xl, k);
        const double xi = acc / bcast(L[i], i);
        if (lane == i) xl = xi;
    }
    return LSEFIT_OK;
}

// (M^T g)_j = sum_{k<=j} C(j,k) (-c)^(j-k) s^-j g_k : the adjoint of to_x_basis
template <int N>
__device__ inline void to_t_basis_adjoint(const double (&g)[N], double c, double s, double (&gt)[N]) {
    const double inv_s = 1.0 / s;
    double spow = 1.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double acc = 0.0;
        double binom = 1.0;   // C(j, k), k from 0
        double cpow_jk[N];
        // (-c)^(j-k) for k = j down to 0
        double cp = 1.0;
#pragma unroll
        for (int k = j; k >= 0; --k) {
            cpow_jk[k] = cp;
            cp *= -c;
        }
#pragma unroll
        for (int k = 0; k <= j; ++k) {
            acc += binom * cpow_jk[k] * g[k];
            binom = binom * (double)(j - k) / (double)(k + 1);
        }
        gt[j] = acc * spow;
        spow *= inv_s;
    }
}

}  // namespace lsefit
