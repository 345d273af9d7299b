// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), written from its published
// definition: ten rounds of two 64x64 -> 128-bit multiplies with the round
// multipliers below, the key bumped by the two Weyl constants between rounds.
// Used for the per-frame random offset d_o of the automorphism block
// (Section III-B), so that a frame's draw depends only on (key, frame uid).
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define BCH_HD __host__ __device__ __forceinline__
#else
#define BCH_HD inline
#endif

namespace bch {

BCH_HD void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    const unsigned __int128 p = (unsigned __int128)a * b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
}

// x: counter (four words, updated in place to the output); k: key (two words)
BCH_HD void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1)
{
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ull, x[0], hi0, lo0);
        mulhilo64(0xCA5A826395121157ull, x[2], hi1, lo1);
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
    }
}

// d_o of frame uid: word 0 of Philox4x64-10 at counter (uid, 0, 0, 0) under
// key (seed, key_hi), its upper 32 bits mapped to [0, d_p) by a multiply and
// shift (bias below d_p / 2^32)
BCH_HD uint8_t draw_offset(uint64_t seed, uint64_t key_hi, uint64_t uid, int dp)
{
    uint64_t x[4] = {uid, 0, 0, 0};
    philox4x64_10(x, seed, key_hi);
    return (uint8_t)(((x[0] >> 32) * (uint64_t)dp) >> 32);
}

}  // namespace bch
