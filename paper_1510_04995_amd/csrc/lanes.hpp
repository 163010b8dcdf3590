// Lane exchange within a 64-lane wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace girih {

// Value of a neighbouring lane of the wave (DPP move; CTRL 0x130 = wave_shl:1,
// lane i takes lane i+1; 0x138 = wave_shr:1, lane i takes lane i-1); a lane
// with no source lane gets zero (bound_ctrl).
template <int CTRL, typename Real>
__device__ __forceinline__ Real lane_shift(Real v) {
    if constexpr (sizeof(Real) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, true);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, true);
        return __builtin_bit_cast(Real, ((uint64_t)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(Real, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
    }
}

}  // namespace girih
