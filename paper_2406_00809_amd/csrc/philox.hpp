// Counter-based normal numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11) followed by the Box-Muller transform (Box & Muller 1958).
//
// Element e of stream `stream`, step `step`, seed `seed`:
// counter = (e_lo, e_hi, step, stream), key = (seed_lo, seed_hi); two 53-bit
// uniforms in (0, 1) from the four output words; z = sqrt(-2 ln u1) cos(2 pi u2).
// Streams: 0 = the x ~ N(0, I) training batches, 1 = the coefficients eps
// of the Arnoldi sampler (Eq. (3)), 2 = the Arnoldi start vector, 3 = the
// default initial weights (uniform_at, on the host).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gnp {

__host__ __device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double normal_at(uint64_t seed, uint32_t step, uint32_t stream,
                                            uint64_t e) {
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), step, stream};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double two53 = 9007199254740992.0;
    const double u1 = ((double)((((uint64_t)(c[0] >> 5)) << 26) | (c[1] >> 6)) + 0.5) / two53;
    const double u2 = ((double)((((uint64_t)(c[2] >> 5)) << 26) | (c[3] >> 6)) + 0.5) / two53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

// The 53-bit uniform in (0, 1) of element e, from the first two output
// words (the u1 of normal_at).
__host__ __device__ inline double uniform_at(uint64_t seed, uint32_t step, uint32_t stream,
                                             uint64_t e) {
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), step, stream};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ((double)((((uint64_t)(c[0] >> 5)) << 26) | (c[1] >> 6)) + 0.5) / 9007199254740992.0;
}

}  // namespace gnp
