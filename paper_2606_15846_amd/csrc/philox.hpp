// Counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// device side, shared by the library's kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace navsim {

// Ten rounds on counter c with key (k0, k1); c receives the four output words.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product in one instruction (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Item (w n) >> 32 of n: a uniform pick from one 32-bit word.
__device__ __forceinline__ int32_t pick_of(uint32_t w, int64_t n) {
    return (int32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

}  // namespace navsim
