/*
 * Oracle: construction of the optimised parity-check matrix H_o
 * (Section III-A, the six-step procedure; Table 1).  Test infrastructure only.
 *
 * Readings of the procedure where the paper is terse (each also listed in the
 * design notes of the repository):
 *   - step 2 "row echelon form" = reduced row echelon form, pivots taken left to
 *     right, zero rows dropped;
 *   - step 3 builds S_f literally (a sum that is the zero vector is skipped: it
 *     is no check); each row then adds to S_g one row, the first member of S_f
 *     whose cyclic class is new, so "excluding any cyclically shifted versions
 *     of existing rows" holds and M_r1 <= M (the padding rule of step 5
 *     presumes M_r1 <= M; collecting every equal-weight sum instead makes the
 *     length-127 matrices grow to thousands of rows);
 *   - step 4 is Q passes of step 3 on the previous H_r1, each pass combining r_i
 *     with every cyclic shift rot^q(r_j), j != i, q = 1..N; S_g starts empty
 *     in every pass; rot^q(r)[c] = r[(c - q) mod N];
 *   - step 5 pads with beta (M - M_r1) copies of H_r1's rows taken in ascending
 *     weight order (stable) and cyclically, M = N - K; alternatively a target
 *     row count M_o is given and M_o - M_r1 copies are added, which keeps Table
 *     1's dimensions when M_r1 differs from the paper's;
 *   - step 6 is simulated annealing on whole-row cyclic shifts driven by a
 *     SplitMix64 stream: a row is drawn with probability proportional to its
 *     length-4-cycle count plus one, a shift q uniform in [1, N-1]; the loss is
 *     C4 + lambda * sum_c (w_c - mean w)^2; a move that would duplicate another
 *     row is rejected; uphill moves are accepted with probability exp(-d/T); T
 *     starts at T0 = (mean uphill delta of 64 trial proposals) / ln 2 and cools
 *     geometrically to 1e-3 T0 over steps_per_row * M_o steps; a result whose
 *     rank is not N - K, or that keeps a duplicated row, is rejected and step 6
 *     is re-run with seed + 1.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

uint64_t orc_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static int weight(const uint8_t *r, int N)
{
    int w = 0;
    for (int i = 0; i < N; i++)
        w += r[i];
    return w;
}

static void rotate(const uint8_t *r, int N, int q, uint8_t *out)
{
    for (int c = 0; c < N; c++)
        out[c] = r[((c - q) % N + N) % N];
}

/* lexicographically smallest rotation = key of the cyclic class */
static void canonical(const uint8_t *r, int N, uint8_t *key)
{
    uint8_t tmp[ORC_MAXN];
    memcpy(key, r, (size_t)N);
    for (int q = 1; q < N; q++) {
        rotate(r, N, q, tmp);
        if (memcmp(tmp, key, (size_t)N) < 0)
            memcpy(key, tmp, (size_t)N);
    }
}

int64_t orc_count_4cycles(const uint8_t *H, int M, int N)
{
    int64_t c4 = 0;
    for (int a = 0; a < M; a++)
        for (int b = a + 1; b < M; b++) {
            int ov = 0;
            for (int c = 0; c < N; c++)
                ov += H[(size_t)a * N + c] & H[(size_t)b * N + c];
            c4 += (int64_t)ov * (ov - 1) / 2;
        }
    return c4;
}

/* In-place reduced row echelon form over GF(2); returns the rank.  Rows
 * beyond the rank are left zero. */
int orc_rref(uint8_t *H, int M, int N)
{
    int r = 0;
    for (int c = 0; c < N && r < M; c++) {
        int p = -1;
        for (int i = r; i < M; i++)
            if (H[(size_t)i * N + c]) {
                p = i;
                break;
            }
        if (p < 0)
            continue;
        if (p != r)
            for (int k = 0; k < N; k++) {
                uint8_t t = H[(size_t)p * N + k];
                H[(size_t)p * N + k] = H[(size_t)r * N + k];
                H[(size_t)r * N + k] = t;
            }
        for (int i = 0; i < M; i++)
            if (i != r && H[(size_t)i * N + c])
                for (int k = 0; k < N; k++)
                    H[(size_t)i * N + k] ^= H[(size_t)r * N + k];
        r++;
    }
    return r;
}

int orc_rank(const uint8_t *H, int M, int N)
{
    uint8_t *tmp = malloc((size_t)M * N);
    if (!tmp)
        return -1;
    memcpy(tmp, H, (size_t)M * N);
    int r = orc_rref(tmp, M, N);
    free(tmp);
    return r;
}

/* A growable list of rows together with their cyclic-class keys. */
typedef struct {
    int n, cap, N;
    uint8_t *rows, *keys;
} rowlist;

static int rl_push(rowlist *L, const uint8_t *row, const uint8_t *key)
{
    if (L->n == L->cap) {
        int nc = L->cap ? 2 * L->cap : 64;
        uint8_t *nr = realloc(L->rows, (size_t)nc * L->N);
        if (!nr)
            return -1;
        L->rows = nr;
        uint8_t *nk = realloc(L->keys, (size_t)nc * L->N);
        if (!nk)
            return -1;
        L->keys = nk;
        L->cap = nc;
    }
    memcpy(L->rows + (size_t)L->n * L->N, row, (size_t)L->N);
    memcpy(L->keys + (size_t)L->n * L->N, key, (size_t)L->N);
    L->n++;
    return 0;
}

static int rl_has_key(const rowlist *L, const uint8_t *key)
{
    for (int i = 0; i < L->n; i++)
        if (!memcmp(L->keys + (size_t)i * L->N, key, (size_t)L->N))
            return 1;
    return 0;
}

/* Step 3 (with_shifts = 0) or one pass of step 4 (with_shifts = 1) on the
 * Mr rows of Hr.  For each row r_i the candidates t = r_i xor r_j (or
 * r_i xor rot^q(r_j)) are scanned in order (j ascending, then q ascending);
 * S_f holds r_i and every candidate of the lowest weight met so far, and is
 * reset when a lighter candidate appears.  Row r_i then contributes to S_g the
 * first member of S_f, in S_f order, whose cyclic class S_g does not yet hold
 * (nothing if every class is present).  Writes the rows of H_r1 to out (cap
 * rows) and returns their number, or a negative value on failure / overflow. */
int orc_min_density(const uint8_t *Hr, int Mr, int N, int with_shifts,
                    uint8_t *out, int cap)
{
    rowlist Sg = {0, 0, N, NULL, NULL};
    rowlist Sf = {0, 0, N, NULL, NULL};
    uint8_t t[ORC_MAXN], rj[ORC_MAXN], key[ORC_MAXN], zero[ORC_MAXN];
    memset(zero, 0, sizeof zero);
    int ret = 0;
    for (int i = 0; i < Mr; i++) {
        const uint8_t *ri = Hr + (size_t)i * N;
        int wg = weight(ri, N);
        Sf.n = 0;
        if (rl_push(&Sf, ri, zero)) {
            ret = -1;
            goto done;
        }
        for (int j = 0; j < Mr; j++) {
            if (j == i)
                continue;
            int qlo = with_shifts ? 1 : 0, qhi = with_shifts ? N : 0;
            for (int q = qlo; q <= qhi; q++) {
                rotate(Hr + (size_t)j * N, N, q % N, rj);
                for (int c = 0; c < N; c++)
                    t[c] = ri[c] ^ rj[c];
                int w = weight(t, N);
                if (w == 0)
                    continue;
                if (w < wg) {
                    Sf.n = 0;
                    wg = w;
                }
                if (w == wg && rl_push(&Sf, t, zero)) {
                    ret = -1;
                    goto done;
                }
            }
        }
        for (int k = 0; k < Sf.n; k++) {
            const uint8_t *cand = Sf.rows + (size_t)k * N;
            canonical(cand, N, key);
            if (!rl_has_key(&Sg, key)) {
                if (rl_push(&Sg, cand, key)) {
                    ret = -1;
                    goto done;
                }
                break;
            }
        }
    }
    if (Sg.n > cap) {
        ret = -2;
        goto done;
    }
    memcpy(out, Sg.rows, (size_t)Sg.n * N);
    ret = Sg.n;
done:
    free(Sg.rows);
    free(Sg.keys);
    free(Sf.rows);
    free(Sf.keys);
    return ret;
}

static double uniform01(uint64_t *st)
{
    return (double)(orc_splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0);
}

static int overlap(const uint8_t *a, const uint8_t *b, int N)
{
    int ov = 0;
    for (int c = 0; c < N; c++)
        ov += a[c] & b[c];
    return ov;
}

static int64_t pairs(int ov) { return (int64_t)ov * (ov - 1) / 2; }

/* Loss change (times N, an integer) of replacing row r by cand. */
static int64_t move_delta(const uint8_t *H, int Mo, int N, int r,
                          const uint8_t *cand, const int *colw, int64_t lam)
{
    const uint8_t *old = H + (size_t)r * N;
    int64_t dc4 = 0;
    for (int k = 0; k < Mo; k++) {
        if (k == r)
            continue;
        const uint8_t *o = H + (size_t)k * N;
        dc4 += pairs(overlap(cand, o, N)) - pairs(overlap(old, o, N));
    }
    /* column weights: sum w_c^2 changes where the row leaves / enters */
    int64_t dsq = 0;
    for (int c = 0; c < N; c++) {
        int w = colw[c] - old[c];
        int w2 = w + cand[c];
        dsq += (int64_t)w2 * w2 - (int64_t)colw[c] * colw[c];
    }
    /* N * (dC4 + lam * d sum (w - mean)^2); the mean is invariant */
    return (int64_t)N * dc4 + lam * (int64_t)N * dsq;
}

static int has_duplicate_rows(const uint8_t *H, int Mo, int N)
{
    for (int a = 0; a < Mo; a++)
        for (int b = a + 1; b < Mo; b++)
            if (!memcmp(H + (size_t)a * N, H + (size_t)b * N, (size_t)N))
                return 1;
    return 0;
}

static int row_equals_other(const uint8_t *H, int Mo, int N, int r,
                            const uint8_t *cand)
{
    for (int k = 0; k < Mo; k++)
        if (k != r && !memcmp(H + (size_t)k * N, cand, (size_t)N))
            return 1;
    return 0;
}

/* Step 6 on H (Mo rows), in place. */
static void anneal(uint8_t *H, int Mo, int N, uint64_t seed, int steps_per_row,
                   double lambda)
{
    uint64_t st = seed;
    int64_t lam = (int64_t)llround(lambda);
    int colw[ORC_MAXN];
    int64_t *c4r = malloc(sizeof(int64_t) * (size_t)Mo);
    uint8_t cand[ORC_MAXN];
    for (int c = 0; c < N; c++) {
        colw[c] = 0;
        for (int r = 0; r < Mo; r++)
            colw[c] += H[(size_t)r * N + c];
    }
    for (int r = 0; r < Mo; r++) {
        c4r[r] = 0;
        for (int k = 0; k < Mo; k++)
            if (k != r)
                c4r[r] += pairs(overlap(H + (size_t)r * N, H + (size_t)k * N, N));
    }
    /* T0 from 64 trial proposals (not applied) */
    double up_sum = 0.0;
    int up_n = 0;
    for (int s = 0; s < 64; s++) {
        int r = (int)(orc_splitmix64_next(&st) % (uint64_t)Mo);
        int q = 1 + (int)(orc_splitmix64_next(&st) % (uint64_t)(N - 1));
        rotate(H + (size_t)r * N, N, q, cand);
        int64_t d = move_delta(H, Mo, N, r, cand, colw, lam);
        if (d > 0) {
            up_sum += (double)d / N;
            up_n++;
        }
    }
    double T0 = up_n ? (up_sum / up_n) / log(2.0) : 1.0;
    int steps = steps_per_row * Mo;
    for (int s = 0; s < steps; s++) {
        double T = T0 * pow(1e-3, (double)s / (double)steps);
        int64_t total = 0;
        for (int r = 0; r < Mo; r++)
            total += c4r[r] + 1;
        uint64_t u = orc_splitmix64_next(&st) % (uint64_t)total;
        int r = 0;
        int64_t acc = 0;
        for (r = 0; r < Mo; r++) {
            acc += c4r[r] + 1;
            if ((uint64_t)acc > u)
                break;
        }
        int q = 1 + (int)(orc_splitmix64_next(&st) % (uint64_t)(N - 1));
        rotate(H + (size_t)r * N, N, q, cand);
        if (row_equals_other(H, Mo, N, r, cand))
            continue;
        int64_t d = move_delta(H, Mo, N, r, cand, colw, lam);
        int accept = 1;
        if (d > 0)
            accept = uniform01(&st) < exp(-((double)d / N) / T);
        if (!accept)
            continue;
        /* apply: update per-row cycle counts, column weights, the row */
        uint8_t *old = H + (size_t)r * N;
        int64_t newc4 = 0;
        for (int k = 0; k < Mo; k++) {
            if (k == r)
                continue;
            const uint8_t *o = H + (size_t)k * N;
            int64_t before = pairs(overlap(old, o, N));
            int64_t after = pairs(overlap(cand, o, N));
            c4r[k] += after - before;
            newc4 += after;
        }
        c4r[r] = newc4;
        for (int c = 0; c < N; c++)
            colw[c] += cand[c] - old[c];
        memcpy(old, cand, (size_t)N);
    }
    free(c4r);
}

/* Steps 2-6.  Hstd: M x N standard parity-check matrix (M = N - K, full rank).
 * Ho receives M_o rows (cap rows); target_rows > 0 overrides beta.
 * Returns M_o or a negative error. */
int orc_build_hopt(const uint8_t *Hstd, int M, int N, int beta, int target_rows,
                   int Q, uint64_t seed, int sa_steps_per_row, double sa_lambda,
                   uint8_t *Ho, int cap, int *Mr1_out, uint64_t *seed_used)
{
    int ret;
    size_t big = 4096;
    uint8_t *Hr = malloc((size_t)M * N);
    uint8_t *H1 = malloc(big * N);
    uint8_t *H2 = malloc(big * N);
    if (!Hr || !H1 || !H2) {
        ret = -1;
        goto out;
    }
    memcpy(Hr, Hstd, (size_t)M * N);
    int rank = orc_rref(Hr, M, N); /* step 2 */
    if (rank != M) {
        ret = -3;
        goto out;
    }
    int m1 = orc_min_density(Hr, M, N, 0, H1, (int)big); /* step 3 */
    if (m1 < 0) {
        ret = -4;
        goto out;
    }
    for (int pass = 0; pass < Q; pass++) { /* step 4 */
        int m2 = orc_min_density(H1, m1, N, 1, H2, (int)big);
        if (m2 < 0) {
            ret = -4;
            goto out;
        }
        uint8_t *sw = H1;
        H1 = H2;
        H2 = sw;
        m1 = m2;
    }
    if (Mr1_out)
        *Mr1_out = m1;
    /* step 5 */
    int pad;
    if (target_rows > 0)
        pad = target_rows > m1 ? target_rows - m1 : 0;
    else
        pad = (m1 <= M) ? beta * (M - m1) : 0;
    int Mo = m1 + pad;
    if (Mo > cap) {
        ret = -2;
        goto out;
    }
    memcpy(Ho, H1, (size_t)m1 * N);
    {
        int order[4096];
        for (int k = 0; k < m1; k++)
            order[k] = k;
        /* stable insertion sort by weight */
        for (int a = 1; a < m1; a++) {
            int v = order[a], wv = weight(H1 + (size_t)v * N, N), b = a - 1;
            while (b >= 0 && weight(H1 + (size_t)order[b] * N, N) > wv) {
                order[b + 1] = order[b];
                b--;
            }
            order[b + 1] = v;
        }
        for (int k = 0; k < pad; k++)
            memcpy(Ho + (size_t)(m1 + k) * N, H1 + (size_t)order[k % m1] * N,
                   (size_t)N);
    }
    /* step 6 */
    {
        uint8_t *start = malloc((size_t)Mo * N);
        memcpy(start, Ho, (size_t)Mo * N);
        uint64_t s = seed;
        int ok = 0;
        for (int attempt = 0; attempt < 64; attempt++, s++) {
            memcpy(Ho, start, (size_t)Mo * N);
            anneal(Ho, Mo, N, s, sa_steps_per_row, sa_lambda);
            if (orc_rank(Ho, Mo, N) == M && !has_duplicate_rows(Ho, Mo, N)) {
                ok = 1;
                break;
            }
        }
        free(start);
        if (!ok) {
            ret = -5;
            goto out;
        }
        if (seed_used)
            *seed_used = s;
    }
    ret = Mo;
out:
    free(Hr);
    free(H1);
    free(H2);
    return ret;
}
