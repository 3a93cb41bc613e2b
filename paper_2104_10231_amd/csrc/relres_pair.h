// relres_pair.h -- the per-pair terms of Eq. 20 on the device, shared by the
// force, adjoint and molecular-dynamics kernels.  Not part of the public ABI.
#pragma once

#include "relres_internal.h"

namespace relres {

// Reciprocal and square root of the pair terms.  FP32: hardware estimates.
// FP64: the FP32 estimate refined by NR Newton steps in FP64, each of which
// squares the relative error (2^-22 -> ~2^-44 -> rounding level); one step is
// ample for FP64 energy/virial sums of FP32-force runs, two give full FP64.
struct MathF32 {
    using T = float;
    static __device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
    // r = sqrt(x) and ir = 1/r from one reciprocal-square-root estimate
    static __device__ __forceinline__ void root(float x, float& r, float& ir)
    {
        ir = __builtin_amdgcn_rsqf(x);
        r = x * ir;
    }
};

template <int NR>
struct MathF64 {
    using T = double;
    static __device__ __forceinline__ double recip(double x)
    {
        double y = (double)__builtin_amdgcn_rcpf((float)x);
#pragma unroll
        for (int k = 0; k < NR; ++k) y = fma(y, fma(-x, y, 1.0), y);
        return y;
    }
    static __device__ __forceinline__ void root(double x, double& r, double& ir)
    {
        double y = (double)__builtin_amdgcn_rsqf((float)x);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double e = fma(-(x * y), y, 1.0);   // 1 - x y^2
            y = fma(0.5 * y, e, y);
        }
        ir = y;
        r = x * y;
        r = fma(0.5 * y, fma(-r, r, x), r);          // one more step on r itself
    }
};

// Pair terms of the FG part of Eq. 20 (r < r_s+): fpair = -u~'(r)/r and the
// energy.  Called only for r2 < r_s+^2.
template <typename M, typename T = typename M::T>
__device__ __forceinline__ void fg_term(const PairCoef<T>& c, const Cutoffs<T>& cut, T r2,
                                        T& fpair, T& en)
{
    if (r2 < cut.rsi2) {
        const T r2i = M::recip(r2);
        const T r6i = r2i * r2i * r2i;
        fpair = r6i * (c.fg_c12 * r6i - c.fg_c6) * r2i;
        en = r6i * (c.fg_e12 * r6i - c.fg_e6) - c.fg_shift;
    } else {
        T r, ir;
        M::root(r2, r, ir);
        const T d = r - cut.rsi;
        const T dp = c.fg_g[1] + d * (T(2) * c.fg_g[2] + d * (T(3) * c.fg_g[3] + d * (T(4) * c.fg_g[4])));
        fpair = -dp * ir;
        en = c.fg_g[0] + d * (c.fg_g[1] + d * (c.fg_g[2] + d * (c.fg_g[3] + d * c.fg_g[4]))) - c.fg_shift;
    }
}

// Pair terms of the CG part of Eq. 20 (hybrid pairs, r < r_c+).
template <typename M, typename T = typename M::T>
__device__ __forceinline__ void cg_term(const PairCoef<T>& c, const Cutoffs<T>& cut, T r2,
                                        T& fpair, T& en)
{
    if (r2 < cut.rsi2) {
        fpair = T(0);
        en = c.sp_g0 - c.sp_shift;
    } else if (r2 < cut.rso2) {
        T r, ir;
        M::root(r2, r, ir);
        const T d = r - cut.rsi;
        const T dp = d * d * (T(3) * c.sp_g3 + T(4) * c.sp_g4 * d);
        fpair = -dp * ir;
        en = c.sp_g0 + d * d * d * (c.sp_g3 + d * c.sp_g4) - c.sp_shift;
    } else if (r2 < cut.rci2) {
        const T r2i = M::recip(r2);
        const T r6i = r2i * r2i * r2i;
        fpair = r6i * (c.cg_c12 * r6i - c.cg_c6) * r2i;
        en = r6i * (c.cg_e12 * r6i - c.cg_e6) - c.cm_shift;
    } else {
        T r, ir;
        M::root(r2, r, ir);
        const T d = r - cut.rci;
        const T dp = c.cm_g[1] + d * (T(2) * c.cm_g[2] + d * (T(3) * c.cm_g[3] + d * (T(4) * c.cm_g[4])));
        fpair = -dp * ir;
        en = c.cm_g[0] + d * (c.cm_g[1] + d * (c.cm_g[2] + d * (c.cm_g[3] + d * c.cm_g[4]))) - c.cm_shift;
    }
}

}  // namespace relres
