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
constexpr int kDppRor8 = 0x128;         // lane i <- lane i ^ 8 within 16 (rotate by 8)
constexpr int kDppShr1 = 0x111;         // lane i <- lane i - 1 within 16 (0 past the row)
constexpr int kDppShr2 = 0x112;
constexpr int kDppShr4 = 0x114;
constexpr int kDppShr8 = 0x118;

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

// Inclusive prefix sum over the 64 lanes of a wave by DPP lane moves: shifts
// by 1, 2, 4, 8 within each row of 16, then the rows' totals carried across
// (lane 15 to the next row, lane 31 to the upper two).
__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, kDppShr1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppShr2, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppShr4, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppShr8, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppBcast31, 0xc, 0xf, false);
    return v;
}

constexpr int kIntMin = -2147483647 - 1;

// Inclusive running maximum over the 64 lanes of a wave (the lane moves of
// wave_inclusive_scan; lanes without a source lane take INT_MIN, the
// identity of the maximum, which lets each move fold into the max).
__device__ __forceinline__ int wave_inclusive_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppShr1, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppShr2, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppShr4, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppShr8, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppBcast15, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(kIntMin, v, kDppBcast31, 0xc, 0xf, false));
    return v;
}

// Lane exchange i <-> i ^ X for X in 4, 8, 16 through ds_swizzle (bit mode:
// and-mask 31, xor-mask X; within each half of the wave).
template <int X>
__device__ __forceinline__ double swizzle_xor(double v)
{
    constexpr int kPattern = 0x1F | (X << 10);
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffff), kPattern);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), kPattern);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// The wave sums of 8 values at once by halving: each exchange sends the half
// of a lane's values that its partner keeps (lane ^ 1: four values, ^ 2: two,
// ^ 4: one), then the one value left is summed over lanes ^ 8, ^ 16, ^ 32.
// 8 + 4 + 2 + 2 + 2 + 2 lane moves of 32 bits instead of 6 x 8 x 2.  Every
// lane gets the wave total of component 4 (lane & 1) + 2 (lane >> 1 & 1) +
// (lane >> 2 & 1); lanes 0..7 hold all eight (wave_sum8_lane gives the lane
// of a component).  The order of the additions is fixed.
__device__ __forceinline__ double wave_sum8(const double v[8])
{
    const int lane = (int)__lane_id();
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    double k4[4], s4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        k4[j] = b0 ? v[4 + j] : v[j];
        s4[j] = b0 ? v[j] : v[4 + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) k4[j] += dpp<kDppXor1>(s4[j]);
    double k2[2], s2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        k2[j] = b1 ? k4[2 + j] : k4[j];
        s2[j] = b1 ? k4[j] : k4[2 + j];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) k2[j] += dpp<kDppXor2>(s2[j]);
    double k1 = b2 ? k2[1] : k2[0];
    k1 += swizzle_xor<4>(b2 ? k2[0] : k2[1]);
    k1 += dpp<kDppRor8>(k1);
    k1 += swizzle_xor<16>(k1);
    k1 += __shfl_xor(k1, 32);
    return k1;
}

// The lane (0..7) whose wave_sum8 result is component k; the map reverses
// three bits, so it also gives the component of lane k.
__device__ __forceinline__ constexpr int wave_sum8_lane(int k)
{
    return (k >> 2) | (((k >> 1) & 1) << 1) | ((k & 1) << 2);
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
