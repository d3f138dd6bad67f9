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

// Ordering point for LDS traffic between the lanes of a one-wave workgroup.
// A wave's LDS operations execute in order, so a compiler-level barrier
// (a wavefront-scope fence) is enough; unlike __syncthreads it does not wait
// for outstanding global loads, which lets prefetches stay in flight.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Ordering point for one wave's own global-memory accesses (the visited
// bitmap and its cleanup list, which only the wave that searches the query
// touches).  A wave's accesses to one address reach memory in issue order,
// so no cache write-back or invalidation is needed (an agent-scope fence
// would write back the whole L2 of the XCD, at every spill); this keeps the
// compiler from moving accesses across it and orders the wave's lanes.
__device__ __forceinline__ void wave_mem_order()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// lanes below this one
__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int popc(uint64_t x) { return __popcll(x); }

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// value of v in lane t (t uniform across the wave), as a scalar
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int t)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, t);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), t);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// value of v in lane (this lane xor O), all lanes active: lane swaps within
// quads are DPP moves (no LDS round trip), xor 4 / 8 / 16 a swizzle, wider
// ones a permute through the LDS crossbar
template <int O>
__device__ __forceinline__ float xor_lane(float v)
{
    static_assert(O >= 1 && O < 64 && (O & (O - 1)) == 0, "power of two below 64");
    const int b = __float_as_int(v);
    if (O == 1) return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, false));
    if (O == 2) return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, false));
    if (O < 32) return __int_as_float(__builtin_amdgcn_ds_swizzle(b, 0x1F | (O << 10)));
    return __shfl_xor(v, O, kWave);
}

__device__ __forceinline__ float wave_sum(float v)
{
    v += xor_lane<32>(v);
    v += xor_lane<16>(v);
    v += xor_lane<8>(v);
    v += xor_lane<4>(v);
    v += xor_lane<2>(v);
    v += xor_lane<1>(v);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// sum within aligned groups of G lanes (G a power of two <= 64)
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if (G >= 64) v += xor_lane<32>(v);
    if (G >= 32) v += xor_lane<16>(v);
    if (G >= 16) v += xor_lane<8>(v);
    if (G >= 8) v += xor_lane<4>(v);
    if (G >= 4) v += xor_lane<2>(v);
    if (G >= 2) v += xor_lane<1>(v);
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
