/*
 * Oracle: normalized min-sum decoders (test infrastructure only).
 *
 * Plain NMS is Section II-A: v2c update (eq. 2), c2v normalized min-sum
 * (eq. 3), posterior (eq. 4), syndrome stop (eq. 5).  Enhanced NMS is the
 * algorithm of Section III-B: per iteration the input is dilated into the
 * automorphism block, eqs. 2-3 run on every branch, the per-bit sums of the
 * eq.-3 outputs are mapped back through the inverse permutations and averaged,
 * that average replaces the second term of eq. 4 to give y^(t) and its hard
 * decision, the syndrome decides the stop, and y is replaced by y^(t).
 *
 * Message memory (eq. 2 keeps the previous c2v messages, while the algorithm
 * also replaces y by y^(t)) admits three readings, all implemented:
 *   R2: v = Y_b[i] + sum_{k in C(i)\j} c2v_b^(t-1)[k,i],  y^(t) = y^(t-1) + avg
 *   R3: v = Y_b[i] - c2v_b^(t-1)[j,i],                    y^(t) = L + avg
 *       (the merged posterior minus the branch's own message; with one branch
 *        this is exactly plain NMS)
 *   R1: v = Y_b[i],                                       y^(t) = y^(t-1) + avg
 * where Y_b[i] = y^(t-1)[maps[b][i]] and y^(0) = L, c2v^(0) = 0.
 * sgn(x) = +1 for x >= 0 (also -0.0); the hard decision is c = [y < 0].
 * The average is the sum over branches b = 0..B-1 (ascending) divided by B;
 * per-branch bit sums run over checks in ascending row order.
 *
 * orc_nms_literal evaluates eq. 2 and eq. 3 with explicit exclusion loops
 * (k != j, k != i).  orc_nms_fast uses the min1/min2/sign-product form of
 * eq. 3 (identical values) and S - own for eq. 2 (equal up to rounding).
 * orc_nms_fixed is the integer variant: int8 v2c messages, c2v magnitude
 * (3m + 2) >> 2 (alpha = 3/4 by shift-add), int32 sums, branch average
 * sign(s) * ((|s| + floor(B/2)) / B), posterior saturated to +-32767.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static int syndrome_zero(const uint8_t *Hs, int Ms, int N, const uint8_t *c)
{
    for (int r = 0; r < Ms; r++) {
        int p = 0;
        for (int i = 0; i < N; i++)
            p ^= Hs[(size_t)r * N + i] & c[i];
        if (p)
            return 0;
    }
    return 1;
}

static double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

static int check_args(const uint8_t *H, int M, int N, int B, int max_iter,
                      int mode)
{
    if (M < 1 || N < 2 || N > ORC_MAXN || B < 1 || max_iter < 1)
        return -1;
    if (mode != ORC_R1 && mode != ORC_R2 && mode != ORC_R3)
        return -1;
    for (int j = 0; j < M; j++) {
        int w = 0;
        for (int i = 0; i < N; i++)
            w += H[(size_t)j * N + i];
        if (w < 2)
            return -1; /* a check of weight < 2 has no extrinsic minimum */
    }
    return 0;
}

#define IDX(b, j, i) (((size_t)(b) * M + (j)) * N + (i))

int orc_nms_literal(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                    const double *L, double alpha, int max_iter, int mode,
                    const uint8_t *Hsyn, int Msyn, uint8_t *c_hat, int *iters,
                    int *converged, double *y_trace)
{
    if (check_args(H, M, N, B, max_iter, mode))
        return -1;
    size_t sz = (size_t)B * M * N;
    double *c2v = calloc(sz, sizeof(double));
    double *c2v_new = calloc(sz, sizeof(double));
    double *v = calloc(sz, sizeof(double));
    double *Y = malloc(sizeof(double) * (size_t)B * N);
    double *S = malloc(sizeof(double) * (size_t)B * N);
    double y[ORC_MAXN], ynew[ORC_MAXN], Sbar[ORC_MAXN];
    if (!c2v || !c2v_new || !v || !Y || !S)
        return -2;
    for (int i = 0; i < N; i++)
        y[i] = L[i];
    *converged = 0;
    *iters = max_iter;
    for (int t = 1; t <= max_iter; t++) {
        /* dilation: Y_b = y gathered through branch b's map */
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++)
                Y[b * N + i] = y[maps[b * N + i]];
        /* eq. 2 */
        for (int b = 0; b < B; b++)
            for (int j = 0; j < M; j++)
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    double x = Y[b * N + i];
                    if (mode == ORC_R2) {
                        for (int k = 0; k < M; k++)
                            if (k != j && H[(size_t)k * N + i])
                                x += c2v[IDX(b, k, i)];
                    } else if (mode == ORC_R3) {
                        x -= c2v[IDX(b, j, i)];
                    }
                    v[IDX(b, j, i)] = x;
                }
        /* eq. 3 */
        for (int b = 0; b < B; b++)
            for (int j = 0; j < M; j++)
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    double sp = 1.0, mn = INFINITY;
                    for (int k = 0; k < N; k++) {
                        if (k == i || !H[(size_t)j * N + k])
                            continue;
                        double x = v[IDX(b, j, k)];
                        sp *= sgn(x);
                        if (fabs(x) < mn)
                            mn = fabs(x);
                    }
                    c2v_new[IDX(b, j, i)] = alpha * sp * mn;
                }
        /* per-branch bit sums, inverse permutation, average */
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++) {
                double s = 0.0;
                for (int j = 0; j < M; j++)
                    if (H[(size_t)j * N + i])
                        s += c2v_new[IDX(b, j, i)];
                S[b * N + i] = s;
            }
        for (int u = 0; u < N; u++)
            Sbar[u] = 0.0;
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++)
                Sbar[maps[b * N + i]] += S[b * N + i];
        /* eq. 4 with the averaged term */
        for (int u = 0; u < N; u++) {
            double base = (mode == ORC_R3) ? L[u] : y[u];
            ynew[u] = base + Sbar[u] / (double)B;
            c_hat[u] = ynew[u] < 0.0;
        }
        if (y_trace)
            for (int u = 0; u < N; u++)
                y_trace[(size_t)(t - 1) * N + u] = ynew[u];
        double *sw = c2v;
        c2v = c2v_new;
        c2v_new = sw;
        for (int u = 0; u < N; u++)
            y[u] = ynew[u];
        /* eq. 5 */
        if (syndrome_zero(Hsyn, Msyn, N, c_hat)) {
            *converged = 1;
            *iters = t;
            break;
        }
    }
    free(c2v);
    free(c2v_new);
    free(v);
    free(Y);
    free(S);
    return 0;
}

int orc_nms_fast(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                 const double *L, double alpha, int max_iter, int mode,
                 const uint8_t *Hsyn, int Msyn, uint8_t *c_hat, int *iters,
                 int *converged, double *y_trace)
{
    if (check_args(H, M, N, B, max_iter, mode))
        return -1;
    size_t sz = (size_t)B * M * N;
    double *c2v = calloc(sz, sizeof(double));
    double *v = malloc(sizeof(double) * sz);
    double *S = calloc((size_t)B * N, sizeof(double));
    double y[ORC_MAXN], ynew[ORC_MAXN], Sbar[ORC_MAXN];
    if (!c2v || !v || !S)
        return -2;
    for (int i = 0; i < N; i++)
        y[i] = L[i];
    *converged = 0;
    *iters = max_iter;
    for (int t = 1; t <= max_iter; t++) {
        for (int b = 0; b < B; b++) {
            const int16_t *mp = maps + (size_t)b * N;
            for (int j = 0; j < M; j++) {
                double min1 = INFINITY, min2 = INFINITY, sp = 1.0;
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    double x = y[mp[i]];
                    if (mode == ORC_R2)
                        x += S[b * N + i] - c2v[IDX(b, j, i)];
                    else if (mode == ORC_R3)
                        x -= c2v[IDX(b, j, i)];
                    v[IDX(b, j, i)] = x;
                    double a = fabs(x);
                    if (a < min1) {
                        min2 = min1;
                        min1 = a;
                    } else if (a < min2) {
                        min2 = a;
                    }
                    sp *= sgn(x);
                }
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    double x = v[IDX(b, j, i)];
                    double mag = (fabs(x) == min1) ? min2 : min1;
                    c2v[IDX(b, j, i)] = alpha * (sp * sgn(x)) * mag;
                }
            }
            for (int i = 0; i < N; i++) {
                double s = 0.0;
                for (int j = 0; j < M; j++)
                    if (H[(size_t)j * N + i])
                        s += c2v[IDX(b, j, i)];
                S[b * N + i] = s;
            }
        }
        for (int u = 0; u < N; u++)
            Sbar[u] = 0.0;
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++)
                Sbar[maps[b * N + i]] += S[b * N + i];
        for (int u = 0; u < N; u++) {
            double base = (mode == ORC_R3) ? L[u] : y[u];
            ynew[u] = base + Sbar[u] / (double)B;
            c_hat[u] = ynew[u] < 0.0;
        }
        if (y_trace)
            for (int u = 0; u < N; u++)
                y_trace[(size_t)(t - 1) * N + u] = ynew[u];
        for (int u = 0; u < N; u++)
            y[u] = ynew[u];
        if (syndrome_zero(Hsyn, Msyn, N, c_hat)) {
            *converged = 1;
            *iters = t;
            break;
        }
    }
    free(c2v);
    free(v);
    free(S);
    return 0;
}

static int32_t clampi(int32_t x, int32_t lo, int32_t hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

int orc_nms_fixed(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                  const int8_t *q, int max_iter, int mode, const uint8_t *Hsyn,
                  int Msyn, uint8_t *c_hat, int *iters, int *converged,
                  int32_t *y_trace)
{
    if (check_args(H, M, N, B, max_iter, mode))
        return -1;
    size_t sz = (size_t)B * M * N;
    int32_t *c2v = calloc(sz, sizeof(int32_t));
    int32_t *c2v_new = calloc(sz, sizeof(int32_t));
    int32_t *v = calloc(sz, sizeof(int32_t));
    int32_t *S = malloc(sizeof(int32_t) * (size_t)B * N);
    int32_t y[ORC_MAXN], ynew[ORC_MAXN], Ssum[ORC_MAXN], L[ORC_MAXN];
    if (!c2v || !c2v_new || !v || !S)
        return -2;
    for (int i = 0; i < N; i++) {
        if (q[i] < -127)
            return -1;
        L[i] = q[i];
        y[i] = q[i];
    }
    *converged = 0;
    *iters = max_iter;
    for (int t = 1; t <= max_iter; t++) {
        /* eq. 2, saturated to the int8 message range */
        for (int b = 0; b < B; b++)
            for (int j = 0; j < M; j++)
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    int32_t x = y[maps[b * N + i]];
                    if (mode == ORC_R2) {
                        for (int k = 0; k < M; k++)
                            if (k != j && H[(size_t)k * N + i])
                                x += c2v[IDX(b, k, i)];
                    } else if (mode == ORC_R3) {
                        x -= c2v[IDX(b, j, i)];
                    }
                    v[IDX(b, j, i)] = clampi(x, -127, 127);
                }
        /* eq. 3 with alpha = 3/4: magnitude (3m + 2) >> 2 */
        for (int b = 0; b < B; b++)
            for (int j = 0; j < M; j++)
                for (int i = 0; i < N; i++) {
                    if (!H[(size_t)j * N + i])
                        continue;
                    int neg = 0;
                    int32_t mn = 1 << 30;
                    for (int k = 0; k < N; k++) {
                        if (k == i || !H[(size_t)j * N + k])
                            continue;
                        int32_t x = v[IDX(b, j, k)];
                        neg ^= (x < 0);
                        int32_t a = x < 0 ? -x : x;
                        if (a < mn)
                            mn = a;
                    }
                    int32_t mag = (3 * mn + 2) >> 2;
                    c2v_new[IDX(b, j, i)] = neg ? -mag : mag;
                }
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++) {
                int32_t s = 0;
                for (int j = 0; j < M; j++)
                    if (H[(size_t)j * N + i])
                        s += c2v_new[IDX(b, j, i)];
                S[b * N + i] = s;
            }
        for (int u = 0; u < N; u++)
            Ssum[u] = 0;
        for (int b = 0; b < B; b++)
            for (int i = 0; i < N; i++)
                Ssum[maps[b * N + i]] += S[b * N + i];
        for (int u = 0; u < N; u++) {
            int32_t s = Ssum[u];
            int32_t a = s < 0 ? -s : s;
            int32_t avg = (a + B / 2) / B;
            if (s < 0)
                avg = -avg;
            int32_t base = (mode == ORC_R3) ? L[u] : y[u];
            ynew[u] = clampi(base + avg, -32767, 32767);
            c_hat[u] = ynew[u] < 0;
        }
        if (y_trace)
            for (int u = 0; u < N; u++)
                y_trace[(size_t)(t - 1) * N + u] = ynew[u];
        int32_t *sw = c2v;
        c2v = c2v_new;
        c2v_new = sw;
        for (int u = 0; u < N; u++)
            y[u] = ynew[u];
        if (syndrome_zero(Hsyn, Msyn, N, c_hat)) {
            *converged = 1;
            *iters = t;
            break;
        }
    }
    free(c2v);
    free(c2v_new);
    free(v);
    free(S);
    return 0;
}
