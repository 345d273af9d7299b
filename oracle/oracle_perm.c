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
