// relres_lanes.h -- cross-lane sums within a wave (DPP lane moves), shared
// by the force, adjoint and molecular-dynamics kernels.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace relres {

// Cross-lane moves through DPP (a VALU operand modifier), much cheaper than
// LDS-routed shuffles.  Lanes a DPP move does not write (masked rows, sources
// outside the row) read 0.
constexpr int kDppXor1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;   // lane i <- lane 7-i within 8
constexpr int kDppMirror = 0x140;       // lane i <- lane 15-i within 16
constexpr int kDppBcast15 = 0x142;      // lane 15 of each row -> next row
constexpr int kDppBcast31 = 0x143;      // lane 31 -> rows 2 and 3

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                  CTRL, ROWS, 0xf, false));
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave, complete in lane 63 (fixed order).
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppMirror>(v);
    v += dpp<kDppBcast15, 0xA>(v);
    v += dpp<kDppBcast31, 0xC>(v);
    return v;
}

// wave_sum of K values at once, step by step across the values, so the K
// dependent chains of lane moves and adds overlap (the same sums, in the same
// order, as K separate wave_sum calls); complete in lane 63.
template <int K>
__device__ __forceinline__ void wave_sums(double (&v)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppXor1>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppXor2>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppHalfMirror>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppMirror>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppBcast15, 0xA>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<kDppBcast31, 0xC>(v[k]);
}

// Sum over each aligned group of G lanes (G a power of two <= 64, uniform in
// the wave); every lane of a group holds its group's sum.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G)
{
    if (G >= 2) v += dpp<kDppXor1>(v);
    if (G >= 4) v += dpp<kDppXor2>(v);
    if (G >= 8) v += dpp<kDppHalfMirror>(v);
    if (G >= 16) v += dpp<kDppMirror>(v);
    if (G >= 32) v += __shfl_xor(v, 16);
    if (G >= 64) v += __shfl_xor(v, 32);
    return v;
}

}  // namespace relres
