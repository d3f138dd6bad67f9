// Device-side helpers shared by the PEOs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace peos {

constexpr int kWave = 64;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;   // empty visited-hash slot
constexpr uint32_t kExpanded = 0x80000000u; // "expanded" flag on a list id
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// lanes below this one
__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int popc(uint64_t x) { return __popcll(x); }

template <typename T>
__device__ __forceinline__ T wave_uniform(T v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// sum within aligned groups of G lanes (G a power of two <= 64)
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// total order on (distance, id): map a float to an unsigned key that sorts
// like the float (negative values reversed), then append the id.
__device__ __forceinline__ uint32_t order_bits(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t sort_key(float d, uint32_t id)
{
    return (static_cast<uint64_t>(order_bits(d)) << 32) | (id & kIdMask);
}

}  // namespace peos
