/*
 * Oracle: order-p ordered statistics decoding and brute-force ML
 * (Section II-B; the hybrid of Section IV-B runs OSD only on NMS failures).
 * Test infrastructure only.
 *
 *   1. z = hard decision [L < 0], r = |L|;
 *   2. positions ordered by r descending, ties by lower index;
 *   3. the most reliable basis (MRB): the first K positions, in that order,
 *      whose columns of G are linearly independent (greedy elimination);
 *   4. G reduced to systematic form on the MRB;
 *   5. candidates: flip patterns e on the MRB with weight <= p, by weight and
 *      then lexicographically in MRB order; candidate c = (z_MRB xor e) G~;
 *   6. the winner minimises the discrepancy D(c) = sum_{i: c_i != z_i} r_i;
 *      the first minimum is kept.
 * ML decoding is the minimum of D over all 2^K codewords.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static double discrepancy(const uint8_t *c, const uint8_t *z, const double *r,
                          int N)
{
    double d = 0.0;
    for (int i = 0; i < N; i++)
        if (c[i] != z[i])
            d += r[i];
    return d;
}

static void encode(const uint8_t *Gs, int K, int N, const uint8_t *u,
                   uint8_t *c)
{
    for (int i = 0; i < N; i++)
        c[i] = 0;
    for (int k = 0; k < K; k++)
        if (u[k])
            for (int i = 0; i < N; i++)
                c[i] ^= Gs[(size_t)k * N + i];
}

int orc_osd(const uint8_t *G, int K, int N, const double *L, int order,
            uint8_t *c_hat)
{
    if (K < 1 || N > ORC_MAXN || K > N || order < 0 || order > K)
        return -1;
    uint8_t z[ORC_MAXN], u[ORC_MAXN], c[ORC_MAXN];
    double r[ORC_MAXN];
    int perm[ORC_MAXN], mrb[ORC_MAXN];
    for (int i = 0; i < N; i++) {
        z[i] = L[i] < 0.0;
        r[i] = fabs(L[i]);
        perm[i] = i;
    }
    /* stable insertion sort by reliability, descending */
    for (int a = 1; a < N; a++) {
        int p = perm[a], b = a - 1;
        while (b >= 0 && r[perm[b]] < r[p]) {
            perm[b + 1] = perm[b];
            b--;
        }
        perm[b + 1] = p;
    }
    uint8_t *Gs = malloc((size_t)K * N);
    if (!Gs)
        return -2;
    memcpy(Gs, G, (size_t)K * N);
    int piv = 0;
    for (int a = 0; a < N && piv < K; a++) {
        int col = perm[a], row = -1;
        for (int k = piv; k < K; k++)
            if (Gs[(size_t)k * N + col]) {
                row = k;
                break;
            }
        if (row < 0)
            continue;
        if (row != piv)
            for (int i = 0; i < N; i++) {
                uint8_t t = Gs[(size_t)row * N + i];
                Gs[(size_t)row * N + i] = Gs[(size_t)piv * N + i];
                Gs[(size_t)piv * N + i] = t;
            }
        for (int k = 0; k < K; k++)
            if (k != piv && Gs[(size_t)k * N + col])
                for (int i = 0; i < N; i++)
                    Gs[(size_t)k * N + i] ^= Gs[(size_t)piv * N + i];
        mrb[piv++] = col;
    }
    if (piv != K) {
        free(Gs);
        return -3; /* G is rank deficient */
    }
    double best = INFINITY;
    /* weight 0 */
    for (int k = 0; k < K; k++)
        u[k] = z[mrb[k]];
    encode(Gs, K, N, u, c);
    best = discrepancy(c, z, r, N);
    memcpy(c_hat, c, (size_t)N);
    /* weight 1..order, lexicographic index tuples */
    for (int w = 1; w <= order && w <= K; w++) {
        int idx[ORC_MAXN];
        for (int q = 0; q < w; q++)
            idx[q] = q;
        for (;;) {
            for (int k = 0; k < K; k++)
                u[k] = z[mrb[k]];
            for (int q = 0; q < w; q++)
                u[idx[q]] ^= 1;
            encode(Gs, K, N, u, c);
            double d = discrepancy(c, z, r, N);
            if (d < best) {
                best = d;
                memcpy(c_hat, c, (size_t)N);
            }
            /* next combination */
            int q = w - 1;
            while (q >= 0 && idx[q] == K - w + q)
                q--;
            if (q < 0)
                break;
            idx[q]++;
            for (int s = q + 1; s < w; s++)
                idx[s] = idx[s - 1] + 1;
        }
    }
    free(Gs);
    return 0;
}

int orc_ml_bruteforce(const uint8_t *G, int K, int N, const double *L,
                      uint8_t *c_hat)
{
    if (K < 1 || K > 24 || N > ORC_MAXN)
        return -1;
    uint8_t z[ORC_MAXN], u[ORC_MAXN], c[ORC_MAXN];
    double r[ORC_MAXN];
    for (int i = 0; i < N; i++) {
        z[i] = L[i] < 0.0;
        r[i] = fabs(L[i]);
    }
    double best = INFINITY;
    for (uint32_t msg = 0; msg < (1u << K); msg++) {
        for (int k = 0; k < K; k++)
            u[k] = (msg >> k) & 1u;
        encode(G, K, N, u, c);
        double d = discrepancy(c, z, r, N);
        if (d < best) {
            best = d;
            memcpy(c_hat, c, (size_t)N);
        }
    }
    return 0;
}
