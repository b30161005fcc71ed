// Per-degree launchers: Launchers<MAXM> is instantiated in kernels_m<MAXM>.hip,
// one translation unit per largest degree so that they compile in parallel.
#pragma once

#include "kernels.hpp"

namespace lsefit {

template <int MAXM>
struct Launchers {
    static hipError_t moments(const FitDesc& d, const Work& w, int prec, int dtype, const void* x, const void* y,
                              const Launch& L, int mis, const RangeArg& ra, hipStream_t st);
    static hipError_t finish_single(const FitDesc& d, const Work& w, int64_t G, const Finish& fz, hipStream_t st);
    static hipError_t combine(const FitDesc& d, const Work& w, const Launch& L, bool by_block, const Finish& fz,
                              hipStream_t st);
    static hipError_t solve_moments(const double* moments, const Work& w, int m, int solver, double* coef,
                                    int32_t* status, hipStream_t st);
    static hipError_t refine(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y,
                             const Launch& L, int mis, hipStream_t st);
    static hipError_t adjoint(const FitDesc& d, const Work& w, int solver, int dtype, const void* x, const void* y,
                              const double* grad_coef, int32_t coef_stride, void* gx, void* gy, const Launch& L,
                              int mis, hipStream_t st);
    static hipError_t residual(const FitDesc& d, const Work& w, int dtype, const void* x, const void* y, void* resid,
                               const Launch& L, int mis, hipStream_t st);

   private:
    template <int PREC, typename In>
    static hipError_t moments_t(const FitDesc& d, const Work& w, const void* x, const void* y, const Launch& L,
                                int mis, const RangeArg& ra, hipStream_t st);
    template <typename In>
    static hipError_t refine_t(const FitDesc& d, const Work& w, const void* x, const void* y, const Launch& L,
                               int mis, hipStream_t st);
};

}  // namespace lsefit
