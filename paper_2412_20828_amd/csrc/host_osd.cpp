// Order-p ordered statistics decoding on the host (Section II-B), the second
// stage of the hybrid decoder (run only for frames the NMS stage left with a
// nonzero syndrome).  Steps: hard decision and reliabilities |L|; positions
// sorted by reliability (descending, ties by index); most reliable basis by
// greedy Gaussian elimination on the generator columns; systematic generator
// on the basis; re-encoding of the basis decision with every flip pattern of
// weight <= p (weight-major, then lexicographic in basis order); the candidate
// with the smallest sum of reliabilities over disagreeing positions wins, the
// first one on equality.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.h"

namespace bch {

void osd_frame(const Code &c, const float *llr, int order, uint64_t *bits_out)
{
    const int N = c.N, K = c.K;
    double r[128];
    Row z;
    for (int i = 0; i < N; i++) {
        r[i] = std::fabs((double)llr[i]);
        if (llr[i] < 0.0f)
            z.set(i);
    }
    int perm[128];
    std::iota(perm, perm + N, 0);
    std::stable_sort(perm, perm + N, [&](int a, int b) { return r[a] > r[b]; });
    std::vector<Row> Gs = c.G;
    int mrb[128];
    int piv = 0;
    for (int a = 0; a < N && piv < K; a++) {
        const int col = perm[a];
        int row = -1;
        for (int k = piv; k < K; k++)
            if (Gs[k].get(col)) {
                row = k;
                break;
            }
        if (row < 0)
            continue;
        std::swap(Gs[row], Gs[piv]);
        for (int k = 0; k < K; k++)
            if (k != piv && Gs[k].get(col))
                Gs[k] = Gs[k] ^ Gs[piv];
        mrb[piv++] = col;
    }
    // base candidate: re-encoded basis decision; d0 = its disagreement with z
    Row c0;
    for (int k = 0; k < K; k++)
        if (z.get(mrb[k]))
            c0 = c0 ^ Gs[k];
    auto cost = [&](const Row &diff) {
        double d = 0.0;
        for (int w = 0; w < 2; w++) {
            uint64_t x = diff.w[w];
            while (x) {
                d += r[w * 64 + __builtin_ctzll(x)];
                x &= x - 1;
            }
        }
        return d;
    };
    const Row d0 = c0 ^ z;
    Row best = c0;
    double best_d = cost(d0);
    if (order >= 1)
        for (int k1 = 0; k1 < K; k1++) {
            const Row d1 = d0 ^ Gs[k1];
            const double v1 = cost(d1);
            if (v1 < best_d) {
                best_d = v1;
                best = c0 ^ Gs[k1];
            }
        }
    if (order >= 2)
        for (int k1 = 0; k1 < K; k1++) {
            const Row d1 = d0 ^ Gs[k1];
            for (int k2 = k1 + 1; k2 < K; k2++) {
                const double v2 = cost(d1 ^ Gs[k2]);
                if (v2 < best_d) {
                    best_d = v2;
                    best = c0 ^ Gs[k1] ^ Gs[k2];
                }
            }
        }
    const int W64 = (N + 63) / 64;
    for (int w = 0; w < W64; w++)
        bits_out[w] = best.w[w];
}

}  // namespace bch
