// Counter-based random numbers shared by the samplers (Husimi and flow proposal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scivr {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128
// multiplications with key bumps by the golden-ratio and sqrt(3)-1 Weyl constants.
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                     uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__device__ inline double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// Box-Muller: two uniforms (from the 64-bit words a, b) to two standard normals.
__device__ inline void box_muller(uint64_t a, uint64_t b, double &z0, double &z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double rad = sqrt(-2.0 * log(u01(a)));
    double s, co;
    sincos(two_pi * u01(b), &s, &co);
    z0 = rad * co;
    z1 = rad * s;
}

}  // namespace scivr
