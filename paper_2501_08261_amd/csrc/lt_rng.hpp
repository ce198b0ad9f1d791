// Counter-based random numbers shared by the sampler, the flow proposal and
// the Fisher draws: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw,
// SC'11), uniforms (u + 1/2) 2^-32 in (0, 1).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lt_rng {

__host__ __device__ inline void philox4x32_10(uint32_t* c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

__host__ __device__ inline double u01(uint32_t u) { return ((double)u + 0.5) * 2.3283064365386963e-10; }

// purposes (second counter word)
constexpr uint32_t kTagMove = 0x100, kTagShift = 0x200, kTagSwap = 0x300, kTagFlowZ = 0x400, kTagFlowU = 0x500,
                   kTagFlowC = 0x600, kTagFlowW = 0x700, kTagFlowG = 0x800, kTagFlowM = 0x900;

}  // namespace lt_rng
