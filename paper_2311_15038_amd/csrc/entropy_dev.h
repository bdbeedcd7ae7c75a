// Grey value of a rendered pixel for the best-view snapshot (Section III-C,
// Eq. 2), shared by the frame-histogram kernel and the ray caster's epilogue:
// 8-bit channel codes q = floor(255 clamp(c, 0, 1) + 1/2) in FP32 (product,
// then sum) and the integer BT.601 luminance (77 q_r + 150 q_g + 29 q_b + 128) >> 8.
#pragma once

#include "common.h"

namespace vr {
namespace ent {

__device__ __forceinline__ uint32_t channel_code(float c)
{
    const float x = fminf(fmaxf(c, 0.0f), 1.0f);
    return (uint32_t)floorf(x * 255.0f + 0.5f);
}

__device__ __forceinline__ uint32_t grey_code(float4 p)
{
    return (77u * channel_code(p.x) + 150u * channel_code(p.y) + 29u * channel_code(p.z) + 128u) >> 8;
}

// Adds grey value g of this lane (when `in`) to the LDS histogram h; a wave
// whose active pixels all share one value adds them with one atomic.  Every
// lane of the wave must call it.
__device__ __forceinline__ void count_grey(uint32_t* h, bool in, uint32_t g)
{
    const uint32_t g0 = __builtin_amdgcn_readfirstlane(in ? g : 0u);
    const uint64_t act = __ballot(in);
    if (__ballot(in && g == g0) == act) {
        if (act != 0 && __lane_id() == (uint32_t)__builtin_ctzll(act)) atomicAdd(&h[g0], (uint32_t)__popcll(act));
    } else if (in) {
        atomicAdd(&h[g], 1u);
    }
}

}  // namespace ent
}  // namespace vr
