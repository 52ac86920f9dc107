// Philox4x64-10 of Salmon et al. (SC'11): the counter-based generator whose
// output the low-stretch tree's shifts are read from.
#pragma once

namespace grass {

__device__ __forceinline__ void philox4x64_10(unsigned long long (&c)[4], unsigned long long k0,
                                              unsigned long long k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const unsigned long long lo0 = 0xD2E7470EE14C6C93ull * c[0], hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c[0]);
        const unsigned long long lo1 = 0xCA5A826395121157ull * c[2], hi1 = __umul64hi(0xCA5A826395121157ull, c[2]);
        const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

}  // namespace grass
