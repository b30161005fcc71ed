// Streaming QR fit: the least-squares problem of Sec. II solved through an
// orthogonal factorisation of V = [t_i^k] (the comparator of Sec. III, QR
// instead of the normal equations), in the tall-skinny tree form: every lane
// factors the rows it streams, and the factors are merged lane -> wave ->
// block -> fit.  The error is governed by cond(V) rather than cond(V)^2.
//
// A factor of the rows seen so far is kept without square roots (Gentleman's
// square-root-free Givens rotations): R = D^(1/2) Rb with Rb unit upper
// triangular, D = diag(d), the rotated right side th (Rb b = th solves the
// fit) and the residual sum of squares e.  Including a row (x; y) of weight w
// rotates it into the factor column by column:
//   d' = d_i + w x_i^2,  cb = d_i / d',  sb = w x_i / d',  w <- cb w,
//   x_k <- x_k - x_i Rb_ik,  Rb_ik <- cb Rb_ik + sb x_k     (k > i, and y/th),
// and adds w y^2 to e at the end.  Since cb + sb x_i = 1, the second update
// is Rb_ik + sb x_k' with the already reduced x_k' (one multiply-add).  Two
// factors merge by including the rows of one, (weight d_i, row Rb_i, right
// side th_i), into the other.
#include "kernels_impl.hpp"

namespace lsefit {

// 1/v for v > 0: the hardware reciprocal refined by two Newton steps
// (r <- r + r (1 - v r)), to within a unit or so in the last place; a rotation
// with such c, s stays orthogonal to the same order as its rounding
__device__ inline double recip(double v) {
    double r = __builtin_amdgcn_rcp(v);
    r = fma(r, fma(-v, r, 1.0), r);
    r = fma(r, fma(-v, r, 1.0), r);
    return r;
}

template <int N>
struct GivensQR {
    static constexpr int NR = N * (N - 1) / 2;   // strict upper part of Rb, packed by rows
    static constexpr int LEN = 2 * N + NR + 1;   // flat: d, th, Rb, e
    double d[N], th[N], r[NR > 0 ? NR : 1], e;

    __device__ inline void zero() {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = th[i] = 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) r[k] = 0.0;
        e = 0.0;
    }
    // offset of Rb_(i, i+1) in r
    static constexpr int row_at(int i) { return i * N - i * (i + 1) / 2; }

    // include the row (x; y) of weight w whose entries before column S are zero.
    // GUARD = false when every d_i (i >= S) is already positive: then
    // d_i' >= d_i > 0 (w x_i^2 >= 0), the zero-weight case cannot occur, and
    // the result is the same bit for bit without its selects
    template <int S, bool GUARD = true>
    __device__ inline void include(double w, double (&x)[N], double y) {
#pragma unroll
        for (int i = S; i < N; ++i) {
            const double xi = x[i];
            const double di = d[i];
            const double wxi = w * xi;
            const double dpi = fma(wxi, xi, di);
            const bool nz = !GUARD || dpi != 0.0;
            const double inv = nz ? recip(dpi) : 0.0;
            const double cb = nz ? di * inv : 1.0;
            const double sb = wxi * inv;
            w *= cb;
            d[i] = dpi;
#pragma unroll
            for (int k = i + 1; k < N; ++k) {
                double& rik = r[row_at(i) + k - i - 1];
                x[k] = fma(-xi, rik, x[k]);
                rik = fma(sb, x[k], rik);
            }
            y = fma(-xi, th[i], y);
            th[i] = fma(sb, y, th[i]);
        }
        e = fma(w * y, y, e);
    }

    // every d_i of columns 1.. positive (d_0 counts the rows, so it is too
    // once one row is in): from then on data rows need no zero-weight guard
    __device__ inline bool settled() const {
        bool ok = true;
#pragma unroll
        for (int i = 1; i < N; ++i) ok = ok && d[i] > 0.0;
        return ok;
    }

    // a data row: x_0 = 1 and weight 1, so the first column needs no products.
    // With TABLE, 1/(d_0 + 1) is read from tab (tab[j] = recip(j + 1), the same
    // value): d_0 counts the data rows exactly, and the caller has checked that
    // it is below the table's length
    template <bool GUARD = true, bool TABLE = false>
    __device__ inline void include_data(double (&x)[N], double y, const double* tab = nullptr) {
        const double dp = d[0] + 1.0;
        double inv;
        if constexpr (TABLE) inv = tab[(int)d[0]];
        else inv = recip(dp);
        const double w = d[0] * inv;
        d[0] = dp;
#pragma unroll
        for (int k = 1; k < N; ++k) {
            double& r0k = r[k - 1];
            x[k] -= r0k;
            r0k = fma(inv, x[k], r0k);
        }
        y -= th[0];
        th[0] = fma(inv, y, th[0]);
        include_from1<GUARD>(w, x, y);
    }
    template <bool GUARD = true>
    __device__ inline void include_from1(double w, double (&x)[N], double y) {
        if constexpr (N > 1) include<1, GUARD>(w, x, y);
        else e = fma(w * y, y, e);
    }

    // merge another factor, given by a reader of its flat entries: get(j) = flat[j]
    template <class Get>
    __device__ inline void merge(Get&& get) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double x[N];
#pragma unroll
            for (int k = 0; k < N; ++k) x[k] = k == i ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < N; ++k) x[k] = get(2 * N + row_at(i) + k - i - 1);
            include_row(i, get(i), x, get(N + i));
        }
        e += get(LEN - 1);
    }
    template <int I = 0>
    __device__ inline void include_row(int i, double w, double (&x)[N], double y) {
        if constexpr (I < N) {
            if (i == I) include<I>(w, x, y);
            else include_row<I + 1>(i, w, x, y);
        }
    }

    __device__ inline double flat(int j) const {
        double v = e;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if (j == i) v = d[i];
            if (j == N + i) v = th[i];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (j == 2 * N + k) v = r[k];
        return v;
    }
};

// 1/(j+1) for j < kRecipRows, by recip() once per block into LDS: a factor of
// k data rows has d_0 = k exactly, so the first-column reciprocal of its next
// row is entry k, read instead of recomputed (the float64 reciprocal issues at
// a quarter of the rate and needs two Newton steps)
constexpr int kRecipRows = 1024;

__device__ inline void fill_recip_rows(double* tab) {
    for (int j = threadIdx.x; j < kRecipRows; j += blockDim.x) tab[j] = recip((double)(j + 1));
    __syncthreads();
}

// one point of the streaming pass: the row (1, t, .., t^m; y), weight 1
template <int M>
struct AccQR {
    static constexpr int N = M + 1;
    GivensQR<N> q;
    double inv_s, nc;
    const double* tab;   // kRecipRows reciprocals 1/(j+1) in LDS (fill_recip_rows)
    __device__ inline void init(double c, double is, const double* t) {
        q.zero();
        inv_s = is;
        nc = -c * is;
        tab = t;
    }
    template <bool GUARD = true, bool TABLE = false>
    __device__ inline void point(double xv, double yv) {
        const double t = fma(xv, inv_s, nc);
        double row[N];
        row[0] = 1.0;
#pragma unroll
        for (int k = 1; k < N; ++k) row[k] = row[k - 1] * t;
        q.template include_data<GUARD, TABLE>(row, yv, tab);
    }
    template <bool GUARD, bool TABLE, typename V, int VW>
    __device__ inline void rows(const V& xv, const V& yv) {
#pragma unroll
        for (int e = 0; e < VW; ++e) point<GUARD, TABLE>((double)xv[e], (double)yv[e]);
    }
    // a lane whose factor has settled (after its first N rows or so, unless
    // its t stay at 0) takes the rows without the zero-weight selects, and
    // while its row count stays inside the table, the first column's
    // reciprocals from it
    template <typename V, int VW>
    __device__ inline void vec(const V& xv, const V& yv) {
        if (q.settled()) {
            if (q.d[0] <= (double)(kRecipRows - VW)) rows<false, true, V, VW>(xv, yv);
            else rows<false, false, V, VW>(xv, yv);
        } else {
            rows<true, false, V, VW>(xv, yv);
        }
    }
    __device__ inline void scalar(double xv, double yv) { point(xv, yv); }
};

// lanes 0 .. 63 -> lane 0: at each level lane l < off merges the factor of lane
// l + off, row by row; the senders (lanes >= off) do not change during the
// level, and every lane takes part in the shuffles.  Fixed order, so the
// result is reproducible.
template <int N>
__device__ inline void wave_merge(GivensQR<N>& q) {
    using Q = GivensQR<N>;
    const int lane = lane_id();
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        const bool recv = lane < off;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double wi = __shfl_down(q.d[i], off, kWave);
            const double yi = __shfl_down(q.th[i], off, kWave);
            double x[N];
#pragma unroll
            for (int k = 0; k < N; ++k) x[k] = k == i ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < N; ++k) x[k] = __shfl_down(q.r[Q::row_at(i) + k - i - 1], off, kWave);
            if (recv) q.include_row(i, wi, x, yi);
        }
        const double eo = __shfl_down(q.e, off, kWave);
        if (recv) q.e += eo;
    }
}

// the block's waves -> one factor, written sum-major (entry j of block g at
// part[j G + g], G blocks)
template <int N>
__device__ inline void block_merge_store(const Work& w, GivensQR<N>& q) {
    constexpr int LEN = GivensQR<N>::LEN;
    __shared__ double sh[4][LEN];
    wave_merge(q);
    const int wid = wave_id_in_block();
    if (lane_id() == 0 && wid > 0) {
#pragma unroll
        for (int j = 0; j < LEN; ++j) sh[wid][j] = q.flat(j);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int v = 1; v < nw; ++v) q.merge([&](int j) { return sh[v][j]; });
#pragma unroll
        for (int j = 0; j < LEN; ++j) w.part[(int64_t)j * gridDim.x + blockIdx.x] = q.flat(j);
    }
}

// Every point updates the same factor, so the rounds carry no parallel work
// worth registers: one vector per round and a register budget (96 VGPRs,
// 5 waves per SIMD, up to m = 3; 128 and 4 at m = 4; 256 above) keep the
// compiler from hoisting across points, and the extra waves cover the
// dependence chain through each column's reciprocal.  (The batched kernel
// takes the budget of its largest degree, 4 or 8: at 5 waves per SIMD its
// degree-3 form was slower.)
constexpr int qr_waves_per_eu(int M) { return M <= 3 ? 5 : (M <= 4 ? 4 : 2); }

template <typename In, int U, int M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(qr_waves_per_eu(M))))
    k_qr_single(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W, int mis,
                RangeArg ra) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    double c, inv_s;
    single_range(d, w, x, ra, &c, &inv_s);
    __shared__ double tab[kRecipRows];
    fill_recip_rows(tab);
    AccQR<M> acc;
    acc.init(c, inv_s, tab);
    stream_strided<U>(x, y, d.n_single, mis, wave, W, acc);
    block_merge_store<M + 1>(w, acc.q);
}

// Solve Rb b = th for a merged factor of npts rows and write a_0..a_m to out
// (then b_0..b_m after them with write_b) and b to the record; returns the
// status.  Singular when fewer than m+1 points or some d_i <= 2^-80 max_k d_k
// (|R_ii| <= 2^-40 max_k |R_kk|); non-finite when any entry is.
template <int N>
__device__ inline int qr_solve_store(const GivensQR<N>& q, int64_t npts, double c, double s, double* rec_b,
                                     double* out, bool write_b) {
    int st = npts < N ? LSEFIT_ERR_SINGULAR : LSEFIT_OK;
    bool finite = isfinite(q.e);
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        finite = finite && isfinite(q.d[i]) && isfinite(q.th[i]);
        dmax = fmax(dmax, q.d[i]);
    }
#pragma unroll
    for (int k = 0; k < GivensQR<N>::NR; ++k) finite = finite && isfinite(q.r[k]);
    if (!finite) st = LSEFIT_ERR_NONFINITE;
    const double tiny = ldexp(dmax, -80);
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (st == LSEFIT_OK && !(q.d[i] > tiny)) st = LSEFIT_ERR_SINGULAR;
    double b[N], a[N];
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double acc = q.th[i];
#pragma unroll
        for (int k = i + 1; k < N; ++k) acc -= q.r[GivensQR<N>::row_at(i) + k - i - 1] * b[k];
        b[i] = acc;
    }
    if (st == LSEFIT_OK) {
        to_x_basis<N>(b, c, s, a);
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (!isfinite(a[k]) || !isfinite(b[k])) st = LSEFIT_ERR_NONFINITE;
    }
    if (st != LSEFIT_OK) {
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = b[k] = NAN;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        out[k] = a[k];
        if (write_b) out[N + k] = b[k];
        rec_b[k] = b[k];
    }
    return st;
}

// Merge the G block factors (thread t takes blocks t, t + 256, ..., in order;
// then lanes, then waves, in order), solve, and write [a | b], the status and,
// if asked, info = [c, s, e].
template <int M>
__global__ void __launch_bounds__(256)
    k_qr_finish(FitDesc d, Work w, int64_t G, int maxm, double* __restrict__ coef, int32_t* __restrict__ status,
                double* __restrict__ info) {
    const KernelClock kclock_(w.clock);
    constexpr int N = M + 1;
    constexpr int LEN = GivensQR<N>::LEN;
    __shared__ double sh[4][LEN];
    GivensQR<N> q;
    q.zero();
    for (int64_t g = threadIdx.x; g < G; g += blockDim.x) q.merge([&](int j) { return w.part[(int64_t)j * G + g]; });
    wave_merge(q);
    const int wid = wave_id_in_block();
    if (lane_id() == 0 && wid > 0) {
#pragma unroll
        for (int j = 0; j < LEN; ++j) sh[wid][j] = q.flat(j);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int nw = blockDim.x / kWave;
    for (int v = 1; v < nw; ++v) q.merge([&](int j) { return sh[v][j]; });
    double* r = w.rec;
    const int st = qr_solve_store<N>(q, d.n_single, r[0], r[1], r + rec_b(maxm), coef, true);
    w.pstatus[0] = st;
    status[0] = st;
    if (info) {
        info[0] = r[0];
        info[1] = r[1];
        info[2] = st == LSEFIT_OK ? q.e : NAN;
    }
}

// ---------------------------------------------------------------------------
// batches: each wave factors its segment of every fit it streams, merges the
// factor to lane 0 and writes it to the fit's slot w + f (qr_len(maxm)
// doubles); one thread per fit then merges the fit's slots in wave order
// ---------------------------------------------------------------------------
template <typename In, int MAXC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(qr_waves_per_eu(MAXC))))
    k_qr_batch(FitDesc d, Work w, const In* __restrict__ x, const In* __restrict__ y, int64_t W,
               int mis, int maxm) {
    const KernelClock kclock_(w.clock);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id_in_block();
    const int stride = qr_len(maxm);
    const int rl = rec_len(maxm);
    __shared__ double tab[kRecipRows];
    fill_recip_rows(tab);
    walk_segments(d, w.tile_start, wave, W, [&](int64_t f, int64_t lo, int64_t hi, int64_t slot) {
        if (w.pstatus[f] != LSEFIT_OK) return;
        const double c = w.rec[f * rl + 0];
        const double inv_s = 1.0 / w.rec[f * rl + 1];
        double* __restrict__ out = w.part + slot * stride;
        auto body = [&]<int M>() {
            AccQR<M> acc;
            acc.init(c, inv_s, tab);
            stream_segment<1>(x, y, lo, hi, mis, acc);
            wave_merge(acc.q);
            if (lane_id() == 0) {
#pragma unroll
                for (int j = 0; j < GivensQR<M + 1>::LEN; ++j) out[j] = acc.q.flat(j);
            }
        };
        dispatch_degree<MAXC>(fit_deg(d, f), body);
    });
}

template <int MAXC>
__global__ void __launch_bounds__(256)
    k_qr_combine(FitDesc d, Work w, int64_t W, int maxm, double* __restrict__ coef, int32_t coef_stride,
                 int32_t* __restrict__ status, double* __restrict__ sse) {
    const KernelClock kclock_(w.clock);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.batch) return;
    double* out = coef + f * (int64_t)coef_stride;
    const int m = fit_deg(d, f);
    const int pst = w.pstatus[f];
    if (pst != LSEFIT_OK) {
        const int n = (m >= 1 && m <= maxm) ? m + 1 : coef_stride;
        for (int k = 0; k < n; ++k) out[k] = NAN;
        status[f] = pst;
        if (sse) sse[f] = NAN;
        return;
    }
    const int stride = qr_len(maxm);
    const int64_t NT = w.tile_start[d.batch];
    const int64_t w0 = wave_of_tile(w.tile_start[f], NT, W), w1 = wave_of_tile(w.tile_start[f + 1] - 1, NT, W);
    double* r = w.rec + f * rec_len(maxm);
    auto body = [&]<int M>() {
        GivensQR<M + 1> q;
        q.zero();
        for (int64_t wv = w0; wv <= w1; ++wv) {
            if (!wave_owns_tiles(wv, NT, W)) continue;
            const double* p = w.part + (wv + f) * stride;
            q.merge([&](int j) { return p[j]; });
        }
        const int st = qr_solve_store<M + 1>(q, fit_hi(d, f) - fit_lo(d, f), r[0], r[1], r + rec_b(maxm), out, false);
        w.pstatus[f] = st;
        status[f] = st;
        if (sse) sse[f] = st == LSEFIT_OK ? q.e : NAN;
    };
    dispatch_degree<MAXC>(m, body);
}

hipError_t launch_qr_single(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y,
                            const Launch& L, int mis, const RangeArg& ra, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
    auto body = [&]<int M>() {
        if (dtype == LSEFIT_F32)
            launch_timed((k_qr_single<float, 1, M>), grid, block, st, d, w, (const float*)x,
                               (const float*)y, L.waves, mis, ra);
        else
            launch_timed((k_qr_single<double, 1, M>), grid, block, st, d, w, (const double*)x,
                               (const double*)y, L.waves, mis, ra);
    };
    dispatch_degree<LSEFIT_MAX_DEGREE>(d.degree, body);
    return hipGetLastError();
}

hipError_t launch_qr_batch(const FitDesc& d, const Work& w, int maxm, int dtype, const void* x, const void* y,
                           const Launch& L, int mis, hipStream_t st) {
    const dim3 grid(L.waves / L.wpb), block(L.wpb * kWave);
    auto go = [&]<int MAXC>() {
        if (dtype == LSEFIT_F32)
            launch_timed((k_qr_batch<float, MAXC>), grid, block, st, d, w, (const float*)x, (const float*)y,
                               L.waves, mis, maxm);
        else
            launch_timed((k_qr_batch<double, MAXC>), grid, block, st, d, w, (const double*)x,
                               (const double*)y, L.waves, mis, maxm);
    };
    if (maxm <= 4) go.template operator()<4>();
    else go.template operator()<LSEFIT_MAX_DEGREE>();
    return hipGetLastError();
}

hipError_t launch_qr_combine(const FitDesc& d, const Work& w, int maxm, int64_t W, double* coef, int32_t coef_stride,
                             int32_t* status, double* sse, hipStream_t st) {
    const int64_t blocks = (d.batch + 255) / 256;
    if (maxm <= 4)
        launch_timed(k_qr_combine<4>, dim3(blocks), dim3(256), st, d, w, W, maxm, coef, coef_stride, status,
                           sse);
    else
        launch_timed(k_qr_combine<LSEFIT_MAX_DEGREE>, dim3(blocks), dim3(256), st, d, w, W, maxm, coef,
                           coef_stride, status, sse);
    return hipGetLastError();
}

hipError_t launch_qr_finish(const FitDesc& d, const Work& w, int64_t G, double* coef, int32_t* status, double* info,
                            hipStream_t st) {
    auto body = [&]<int M>() {
        launch_timed(k_qr_finish<M>, dim3(1), dim3(256), st, d, w, G, d.degree, coef, status, info);
    };
    dispatch_degree<LSEFIT_MAX_DEGREE>(d.degree, body);
    return hipGetLastError();
}

}  // namespace lsefit
