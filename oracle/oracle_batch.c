/*
 * Oracle: frame-by-frame loops over the single-frame decoders, so that a
 * caller can hand over a whole array of frames in one call (test
 * infrastructure only).  Each frame gets its own branch maps from its own
 * random offset d_o (one offset per frame, fixed over the iterations).
 * trace (optional): [F][max_iter][N] posteriors, double (int32 for the
 * fixed-point kind); rows past a frame's last iteration are left untouched.
 */
#include <stdlib.h>
#include "oracle.h"

int orc_decode_batch(int kind, const uint8_t *H, int M, int N, int B,
                     const uint8_t *d_o, const void *llr, int ld, int F,
                     double alpha, int max_iter, int mode, const uint8_t *Hsyn,
                     int Msyn, uint8_t *c_hat, int32_t *iters, uint8_t *conv,
                     void *trace)
{
    int16_t maps[9 * ORC_MAXN];
    double L[ORC_MAXN];
    for (int f = 0; f < F; f++) {
        int r = orc_branch_maps(N, B, B > 1 ? d_o[f] : 0, maps);
        if (r)
            return r;
        int it = 0, cv = 0;
        if (kind == 2) {
            const int8_t *q = (const int8_t *)llr + (size_t)f * ld;
            r = orc_nms_fixed(H, M, N, maps, B, q, max_iter, mode, Hsyn, Msyn,
                              c_hat + (size_t)f * N, &it, &cv,
                              trace ? (int32_t *)trace + (size_t)f * max_iter * N
                                    : NULL);
        } else {
            const float *x = (const float *)llr + (size_t)f * ld;
            for (int i = 0; i < N; i++)
                L[i] = (double)x[i];
            if (kind == 0)
                r = orc_nms_literal(H, M, N, maps, B, L, alpha, max_iter, mode,
                                    Hsyn, Msyn, c_hat + (size_t)f * N, &it,
                                    &cv,
                                    trace ? (double *)trace + (size_t)f * max_iter * N
                                          : NULL);
            else
                r = orc_nms_fast(H, M, N, maps, B, L, alpha, max_iter, mode,
                                 Hsyn, Msyn, c_hat + (size_t)f * N, &it, &cv,
                                 trace ? (double *)trace + (size_t)f * max_iter * N
                                       : NULL);
        }
        if (r)
            return r;
        iters[f] = it;
        conv[f] = (uint8_t)cv;
    }
    return 0;
}

/* Hybrid back-end: OSD-p on the channel LLRs of every frame whose flag is 0;
 * frames with flag 1 keep the word already in c_hat. */
int orc_osd_batch(const uint8_t *G, int K, int N, const float *llr, int ld,
                  int F, int order, const uint8_t *flags, uint8_t *c_hat)
{
    double L[ORC_MAXN];
    for (int f = 0; f < F; f++) {
        if (flags && flags[f])
            continue;
        for (int i = 0; i < N; i++)
            L[i] = (double)llr[(size_t)f * ld + i];
        int r = orc_osd(G, K, N, L, order, c_hat + (size_t)f * N);
        if (r)
            return r;
    }
    return 0;
}
