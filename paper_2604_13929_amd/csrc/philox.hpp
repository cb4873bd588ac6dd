// Counter-based Philox4x32-10 generator (Salmon, Moraes, Dror & Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), device side.
//
// Ten rounds; in each round counter words 0 and 2 are multiplied by two fixed
// odd 32-bit constants, the 64-bit products are split into high and low halves,
// the high halves are xored with the remaining counter words and the round key,
// and the four words are permuted.  The two key words advance by two Weyl
// increments between rounds.  Each 32x32->64 product is one v_mad_u64_u32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmc {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c.x;
        const uint64_t pb = (uint64_t)kMulB * c.z;
        U4 n;
        n.x = (uint32_t)(pb >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)pb;
        n.z = (uint32_t)(pa >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)pa;
        c = n;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c;
}

// Uniforms from the top 24 bits: [0,1) and (0,1], exact in FP32.
__device__ __forceinline__ float u01_co(uint32_t r) { return (float)(r >> 8) * 0x1.0p-24f; }
__device__ __forceinline__ float u01_oc(uint32_t r) { return (float)((r >> 8) + 1u) * 0x1.0p-24f; }

}  // namespace pmc
