/*
 * Oracle: binary primitive narrow-sense BCH codes (test infrastructure only).
 *
 * The paper evaluates BCH codes of length 63 and 127 (Section IV, Table 1); it
 * takes them from a code database and states no construction.  The textbook
 * definition written out here: GF(2^m) from a primitive polynomial, zeros
 * alpha^1..alpha^{2t}, generator g(x) = product of the distinct minimal
 * polynomials, check polynomial h(x) = (x^N - 1)/g(x).  The standard
 * parity-check matrix has rows x^i * h~(x) (h~ = reciprocal of h), the
 * banded (N-K) x N form whose row weight wt(h) and column statistics Table 1
 * lists; the generator matrix is systematic: c(x) = x^{N-K} m(x) +
 * (x^{N-K} m(x) mod g(x)), message bits in columns N-K..N-1.
 */
#include <string.h>
#include "oracle.h"

/* exp_tab[i] = alpha^i for 0 <= i < 2N, log_tab[alpha^i] = i. */
int orc_gf_tables(int m, uint32_t prim, int *exp_tab, int *log_tab)
{
    if (m < 2 || m > 7)
        return -1;
    int N = (1 << m) - 1;
    int x = 1;
    for (int i = 0; i <= N; i++)
        log_tab[i] = -1;
    for (int i = 0; i < N; i++) {
        if (log_tab[x] != -1)
            return -2; /* prim is not primitive: alpha has order < N */
        exp_tab[i] = x;
        exp_tab[i + N] = x;
        log_tab[x] = i;
        x <<= 1;
        if (x & (1 << m))
            x ^= (int)prim;
    }
    if (x != 1)
        return -2;
    return 0;
}

static int gf_mul(int a, int b, const int *exp_tab, const int *log_tab)
{
    if (a == 0 || b == 0)
        return 0;
    return exp_tab[log_tab[a] + log_tab[b]];
}

/* g(x) = lcm of minimal polynomials of alpha^1..alpha^{2t}.
 * g[0..deg] coefficients (0/1), lowest degree first. */
int orc_bch_generator(int m, uint32_t prim, int t, uint8_t *g, int *deg)
{
    int exp_tab[2 * ORC_MAXN], log_tab[ORC_MAXN + 1];
    if (orc_gf_tables(m, prim, exp_tab, log_tab))
        return -1;
    int N = (1 << m) - 1;
    if (t < 1 || 2 * t >= N)
        return -1;
    int used[ORC_MAXN];
    memset(used, 0, sizeof used);
    /* poly over GF(2^m), lowest degree first */
    int poly[ORC_MAXN + 1];
    int pdeg = 0;
    poly[0] = 1;
    for (int i = 1; i <= 2 * t; i++) {
        if (used[i % N])
            continue;
        /* cyclotomic coset of i */
        int j = i % N;
        do {
            used[j] = 1;
            /* poly *= (x + alpha^j) */
            int aj = exp_tab[j];
            int np[ORC_MAXN + 1];
            for (int k = 0; k <= pdeg + 1; k++)
                np[k] = 0;
            for (int k = 0; k <= pdeg; k++) {
                np[k + 1] ^= poly[k];
                np[k] ^= gf_mul(poly[k], aj, exp_tab, log_tab);
            }
            pdeg++;
            for (int k = 0; k <= pdeg; k++)
                poly[k] = np[k];
            j = (2 * j) % N;
        } while (j != i % N);
    }
    for (int k = 0; k <= pdeg; k++) {
        if (poly[k] != 0 && poly[k] != 1)
            return -3; /* cannot happen for a union of full cosets */
        g[k] = (uint8_t)poly[k];
    }
    *deg = pdeg;
    return 0;
}

/* Fills N, K, g (N-K+1 coefficients), h (K+1 coefficients), G (K x N),
 * Hstd ((N-K) x N).  Any output pointer may be NULL. */
int orc_bch_matrices(int m, uint32_t prim, int t, int *N_out, int *K_out,
                     uint8_t *g_out, uint8_t *h_out, uint8_t *G, uint8_t *Hstd)
{
    uint8_t g[ORC_MAXN + 1];
    int dg;
    if (orc_bch_generator(m, prim, t, g, &dg))
        return -1;
    int N = (1 << m) - 1;
    int K = N - dg;
    /* h = (x^N + 1) / g by long division over GF(2) */
    uint8_t rem[ORC_MAXN + 1], h[ORC_MAXN + 1];
    memset(rem, 0, sizeof rem);
    memset(h, 0, sizeof h);
    rem[0] = 1;
    rem[N] = 1;
    for (int d = N; d >= dg; d--) {
        if (rem[d]) {
            h[d - dg] = 1;
            for (int k = 0; k <= dg; k++)
                rem[d - dg + k] ^= g[k];
        }
    }
    for (int k = 0; k <= N; k++)
        if (rem[k])
            return -2; /* g does not divide x^N + 1 */
    if (N_out)
        *N_out = N;
    if (K_out)
        *K_out = K;
    if (g_out)
        memcpy(g_out, g, (size_t)dg + 1);
    if (h_out)
        memcpy(h_out, h, (size_t)K + 1);
    if (G) {
        /* row k: x^{N-K+k} + (x^{N-K+k} mod g) */
        for (int k = 0; k < K; k++) {
            uint8_t r[ORC_MAXN + 1];
            memset(r, 0, sizeof r);
            r[N - K + k] = 1;
            for (int d = N - K + k; d >= dg; d--) {
                if (r[d]) {
                    for (int q = 0; q <= dg; q++)
                        r[d - dg + q] ^= g[q];
                }
            }
            uint8_t *row = G + (size_t)k * N;
            for (int i = 0; i < N; i++)
                row[i] = 0;
            for (int i = 0; i < dg; i++)
                row[i] = r[i];
            row[N - K + k] = 1;
        }
    }
    if (Hstd) {
        /* row i = x^i * h~(x), h~_e = h_{K-e} */
        for (int i = 0; i < N - K; i++) {
            uint8_t *row = Hstd + (size_t)i * N;
            for (int c = 0; c < N; c++)
                row[c] = 0;
            for (int e = 0; e <= K; e++)
                if (h[K - e])
                    row[i + e] = 1;
        }
    }
    return 0;
}

/* Weight distribution A[0..N] of the code spanned by the K rows of G
 * (full enumeration of all 2^K messages in Gray-code order). */
int orc_weight_distribution(const uint8_t *G, int K, int N, uint64_t *A)
{
    if (K < 0 || K > 40 || N > ORC_MAXN)
        return -1;
    for (int w = 0; w <= N; w++)
        A[w] = 0;
    /* rows packed in two 64-bit words: bit i of the pair = column i */
    uint64_t rl[64], rh[64];
    for (int k = 0; k < K; k++) {
        rl[k] = rh[k] = 0;
        for (int i = 0; i < N; i++)
            if (G[(size_t)k * N + i]) {
                if (i < 64)
                    rl[k] |= 1ULL << i;
                else
                    rh[k] |= 1ULL << (i - 64);
            }
    }
    uint64_t cl = 0, ch = 0;
    uint64_t total = 1ULL << K;
    A[0]++;
    for (uint64_t n = 1; n < total; n++) {
        int k = __builtin_ctzll(n); /* Gray code: flip row k */
        cl ^= rl[k];
        ch ^= rh[k];
        A[__builtin_popcountll(cl) + __builtin_popcountll(ch)]++;
    }
    return 0;
}

/* All codewords of weight w of the code spanned by the K rows of G (Gray-code
 * enumeration); returns their number (at most cap are written), or < 0. */
int64_t orc_words_of_weight(const uint8_t *G, int K, int N, int w,
                            uint8_t *out, int64_t cap)
{
    if (K < 0 || K > 40 || N > ORC_MAXN)
        return -1;
    uint64_t rl[64], rh[64];
    for (int k = 0; k < K; k++) {
        rl[k] = rh[k] = 0;
        for (int i = 0; i < N; i++)
            if (G[(size_t)k * N + i]) {
                if (i < 64)
                    rl[k] |= 1ULL << i;
                else
                    rh[k] |= 1ULL << (i - 64);
            }
    }
    uint64_t cl = 0, ch = 0, total = 1ULL << K;
    int64_t found = 0;
    for (uint64_t n = 1; n < total; n++) {
        int k = __builtin_ctzll(n);
        cl ^= rl[k];
        ch ^= rh[k];
        if (__builtin_popcountll(cl) + __builtin_popcountll(ch) == w) {
            if (found < cap)
                for (int i = 0; i < N; i++)
                    out[(size_t)found * N + i] =
                        (uint8_t)((i < 64 ? cl >> i : ch >> (i - 64)) & 1);
            found++;
        }
    }
    return found;
}
