/*
 * Oracle: the automorphism block B(y) of the enhanced NMS decoder
 * (Section III-B, the three permutation types and the 9-row block).
 * Test infrastructure only.
 *
 * Each branch is a gather map: Y_b[j] = y[maps[b*N + j]].
 *   - interleave pi_I (even-index bits, then odd-index bits): Y[j] = y[2j mod N]
 *     (0-based; for odd N this is exactly the concatenation);
 *   - Frobenius pi_F (bit i moves to position 2i mod N): Y[j] = y[h*j mod N],
 *     h = (N+1)/2 the inverse of 2, so pi_F is the inverse of pi_I;
 *   - cyclic shift pi_Cs by sh_s = s*d_p + d_o, applied after the type:
 *     Y[j] = Z[(j - sh_s) mod N];
 *   d_p = 21 (N = 63) or 42 (N = 127); S_n = {0,1,2}; S_p = {y, pi_I y, pi_F y}.
 * Branch order: b = 3*s + p with p = 0 (identity), 1 (pi_I), 2 (pi_F).
 * n_branches = 1 gives the identity map (plain NMS); 3 gives the three shifts
 * of y alone; 9 gives the full block.
 *
 * The random offset d_o of a frame is drawn from the counter-based generator
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written out here from
 * its published definition with 128-bit products: ten rounds, each
 * multiplying counter words 0 and 2 by the two round multipliers, the high
 * halves XORed with the other counter words and the key, the key advanced by
 * the two Weyl constants between rounds.  d_o = floor(u * d_p / 2^32) with u
 * the upper 32 bits of output word 0 at counter (uid, 0, 0, 0).
 */
#include "oracle.h"

int orc_branch_maps(int N, int n_branches, int d_o, int16_t *maps)
{
    int dp;
    if (N == 63)
        dp = 21;
    else if (N == 127)
        dp = 42;
    else
        dp = N / 3; /* small test codes: spread three shifts evenly */
    if (n_branches != 1 && n_branches != 3 && n_branches != 9)
        return -1;
    if (d_o < 0 || (n_branches > 1 && d_o >= dp))
        return -1;
    int a_of_p[3] = {1, 2, (N + 1) / 2};
    int np = (n_branches == 9) ? 3 : 1;
    int ns = (n_branches == 1) ? 1 : 3;
    for (int s = 0; s < ns; s++) {
        int sh = (n_branches == 1) ? 0 : s * dp + d_o;
        for (int p = 0; p < np; p++) {
            int b = s * np + p;
            for (int j = 0; j < N; j++) {
                int shifted = ((j - sh) % N + N) % N;
                maps[b * N + j] = (int16_t)((a_of_p[p] * shifted) % N);
            }
        }
    }
    return 0;
}

/* One Philox4x64-10 block: ctr[4] (in), key[2] (in), out[4]. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* d_o of frames uid = frame_base .. frame_base + F - 1 under key (seed, key_hi). */
int orc_draw_offsets(int N, uint64_t seed, uint64_t key_hi, int64_t frame_base, int64_t F, uint8_t *d_o)
{
    if (N < 7 || N > ORC_MAXN || F < 0 || frame_base < 0)
        return -1;
    int dp = (N == 63) ? 21 : (N == 127) ? 42 : N / 3;
    uint64_t key[2] = {seed, key_hi};
    for (int64_t f = 0; f < F; f++) {
        uint64_t ctr[4] = {(uint64_t)(frame_base + f), 0, 0, 0}, out[4];
        orc_philox4x64_10(ctr, key, out);
        uint64_t u = out[0] >> 32;
        d_o[f] = (uint8_t)((u * (uint64_t)dp) >> 32);
    }
    return 0;
}
