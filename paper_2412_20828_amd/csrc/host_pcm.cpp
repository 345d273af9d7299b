// Optimised parity-check matrix H_o (Section III-A): row echelon form, pairwise
// density minimisation, Q passes over cyclic shifts, redundancy padding and
// simulated annealing on cyclic row shifts that lowers the number of
// length-4 cycles and the column-weight spread (Table 1).
//
// The procedure is deterministic for given parameters and follows these
// readings of the paper's steps:
//  * each row contributes to S_g at most one row: among its lightest sums
//    (kept in scan order, j ascending then shift ascending) the first one whose
//    cyclic class is new; the padding rule then applies because M_r1 <= N - K;
//  * padding repeats H_r1's rows in ascending weight order, cyclically;
//  * annealing uses a SplitMix64 stream: row drawn with probability
//    proportional to (its 4-cycle count + 1), shift uniform in [1, N-1], loss
//    C4 + lambda * sum_c w_c^2 (the mean column weight is invariant), moves
//    that duplicate a row rejected, Metropolis acceptance with T decaying
//    geometrically from T0 (mean uphill loss change of 64 trial proposals /
//    ln 2) to 1e-3 T0; a result without full rank or with a repeated row is
//    discarded and the annealing re-run from seed + 1.
#include <algorithm>
#include <cmath>
#include <unordered_set>

#include "internal.h"

namespace bch {

namespace {

struct RowHash {
    size_t operator()(const Row &r) const
    {
        return (size_t)(r.w[0] * 0x9E3779B97F4A7C15ull ^ (r.w[1] + 0x632BE59BD9B4E019ull));
    }
};

// class representative: numerically smallest rotation (high word first)
Row cyclic_key(const Row &r, int N)
{
    Row best = r;
    for (int q = 1; q < N; q++) {
        Row x = rotate(r, N, q);
        if (x.w[1] < best.w[1] || (x.w[1] == best.w[1] && x.w[0] < best.w[0]))
            best = x;
    }
    return best;
}

uint64_t splitmix_next(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int64_t pair_count(int ov) { return (int64_t)ov * (ov - 1) / 2; }

// reduced row echelon form, pivots left to right, zero rows dropped
std::vector<Row> rref(std::vector<Row> rows, int N)
{
    int r = 0;
    for (int c = 0; c < N && r < (int)rows.size(); c++) {
        int p = -1;
        for (int i = r; i < (int)rows.size(); i++)
            if (rows[i].get(c)) {
                p = i;
                break;
            }
        if (p < 0)
            continue;
        std::swap(rows[p], rows[r]);
        for (int i = 0; i < (int)rows.size(); i++)
            if (i != r && rows[i].get(c))
                rows[i] = rows[i] ^ rows[r];
        r++;
    }
    rows.resize(r);
    return rows;
}

struct Annealer {
    std::vector<Row> H;
    int N, Mo;
    int64_t lam;
    std::vector<int> colw;
    std::vector<int64_t> c4r;

    Annealer(const std::vector<Row> &start, int n, double lambda)
        : H(start), N(n), Mo((int)start.size()), lam((int64_t)std::llround(lambda)),
          colw(n, 0), c4r(start.size(), 0)
    {
        for (int r = 0; r < Mo; r++)
            for (int c = 0; c < N; c++)
                colw[c] += H[r].get(c);
        for (int r = 0; r < Mo; r++)
            for (int k = 0; k < Mo; k++)
                if (k != r)
                    c4r[r] += pair_count(overlap(H[r], H[k]));
    }

    // loss change of replacing row r by cand: C4 change + lam * sum w^2 change
    int64_t delta(int r, const Row &cand) const
    {
        int64_t dc4 = 0;
        for (int k = 0; k < Mo; k++)
            if (k != r)
                dc4 += pair_count(overlap(cand, H[k])) - pair_count(overlap(H[r], H[k]));
        int64_t dsq = 0;
        for (int c = 0; c < N; c++) {
            int before = colw[c];
            int after = before - (int)H[r].get(c) + (int)cand.get(c);
            dsq += (int64_t)after * after - (int64_t)before * before;
        }
        return dc4 + lam * dsq;
    }

    bool duplicates_other(int r, const Row &cand) const
    {
        for (int k = 0; k < Mo; k++)
            if (k != r && H[k] == cand)
                return true;
        return false;
    }

    void apply(int r, const Row &cand)
    {
        int64_t own = 0;
        for (int k = 0; k < Mo; k++) {
            if (k == r)
                continue;
            int64_t after = pair_count(overlap(cand, H[k]));
            c4r[k] += after - pair_count(overlap(H[r], H[k]));
            own += after;
        }
        c4r[r] = own;
        for (int c = 0; c < N; c++)
            colw[c] += (int)cand.get(c) - (int)H[r].get(c);
        H[r] = cand;
    }

    void run(uint64_t seed, int steps_per_row)
    {
        uint64_t st = seed;
        double up_sum = 0.0;
        int up_n = 0;
        for (int s = 0; s < 64; s++) {
            int r = (int)(splitmix_next(st) % (uint64_t)Mo);
            int q = 1 + (int)(splitmix_next(st) % (uint64_t)(N - 1));
            int64_t d = delta(r, rotate(H[r], N, q));
            if (d > 0) {
                up_sum += (double)d;
                up_n++;
            }
        }
        const double T0 = up_n ? (up_sum / up_n) / std::log(2.0) : 1.0;
        const int steps = steps_per_row * Mo;
        for (int s = 0; s < steps; s++) {
            const double T = T0 * std::pow(1e-3, (double)s / (double)steps);
            uint64_t total = 0;
            for (int r = 0; r < Mo; r++)
                total += (uint64_t)(c4r[r] + 1);
            const uint64_t u = splitmix_next(st) % total;
            int r = 0;
            uint64_t acc = 0;
            for (; r < Mo; r++) {
                acc += (uint64_t)(c4r[r] + 1);
                if (acc > u)
                    break;
            }
            const int q = 1 + (int)(splitmix_next(st) % (uint64_t)(N - 1));
            const Row cand = rotate(H[r], N, q);
            if (duplicates_other(r, cand))
                continue;
            const int64_t d = delta(r, cand);
            bool accept = true;
            if (d > 0) {
                const double u01 = (double)(splitmix_next(st) >> 11) * (1.0 / 9007199254740992.0);
                accept = u01 < std::exp(-(double)d / T);
            }
            if (accept)
                apply(r, cand);
        }
    }
};

}  // namespace

int64_t count_4cycles(const std::vector<Row> &H)
{
    int64_t c4 = 0;
    for (size_t a = 0; a < H.size(); a++)
        for (size_t b = a + 1; b < H.size(); b++)
            c4 += pair_count(overlap(H[a], H[b]));
    return c4;
}

std::vector<Row> min_density_pass(const std::vector<Row> &Hr, int N, bool with_shifts)
{
    std::vector<Row> Sg;
    std::unordered_set<Row, RowHash> classes;
    std::vector<Row> Sf;
    const int Mr = (int)Hr.size();
    for (int i = 0; i < Mr; i++) {
        const Row &ri = Hr[i];
        int wg = ri.weight();
        Sf.clear();
        Sf.push_back(ri);
        for (int j = 0; j < Mr; j++) {
            if (j == i)
                continue;
            const int qlo = with_shifts ? 1 : 0, qhi = with_shifts ? N : 0;
            for (int q = qlo; q <= qhi; q++) {
                Row t = ri ^ rotate(Hr[j], N, q);
                int w = t.weight();
                if (w == 0 || w > wg)
                    continue;
                if (w < wg) {
                    Sf.clear();
                    wg = w;
                }
                Sf.push_back(t);
            }
        }
        for (const Row &cand : Sf) {
            Row key = cyclic_key(cand, N);
            if (classes.insert(key).second) {
                Sg.push_back(cand);
                break;
            }
        }
    }
    return Sg;
}

int build_hopt(const Code &c, const bch_pcm_params &p, Pcm &out, std::string &err)
{
    const int N = c.N, M = c.N - c.K;
    if (p.Q < 0 || p.beta < 0 || p.target_rows < 0 || p.sa_steps_per_row < 0) {
        err = "negative construction parameter";
        return BCH_EINVAL;
    }
    std::vector<Row> Hr = rref(c.Hstd, N);
    if ((int)Hr.size() != M) {
        err = "standard PCM is not full rank";
        return BCH_ESTATE;
    }
    std::vector<Row> H1 = min_density_pass(Hr, N, false);
    for (int pass = 0; pass < p.Q; pass++)
        H1 = min_density_pass(H1, N, true);
    const int m1 = (int)H1.size();
    int pad;
    if (p.target_rows > 0)
        pad = std::max(0, p.target_rows - m1);
    else
        pad = m1 <= M ? p.beta * (M - m1) : 0;
    const int Mo = m1 + pad;
    if (Mo > 1024) {
        err = "H_o would exceed 1024 rows";
        return BCH_EUNSUPPORTED;
    }
    std::vector<int> order(m1);
    for (int k = 0; k < m1; k++)
        order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return H1[a].weight() < H1[b].weight(); });
    std::vector<Row> start = H1;
    for (int k = 0; k < pad; k++)
        start.push_back(H1[order[k % m1]]);
    uint64_t s = p.seed;
    for (int attempt = 0; attempt < 64; attempt++, s++) {
        Annealer an(start, N, p.sa_lambda);
        an.run(s, p.sa_steps_per_row);
        bool dup = false;
        for (int a = 0; a < Mo && !dup; a++)
            for (int b = a + 1; b < Mo; b++)
                if (an.H[a] == an.H[b]) {
                    dup = true;
                    break;
                }
        if (!dup && gf2_rank(an.H, N) == M) {
            out.N = N;
            out.M = Mo;
            out.rows = an.H;
            out.E = 0;
            for (const Row &r : out.rows)
                out.E += r.weight();
            out.Mr1 = m1;
            out.seed_used = s;
            return BCH_OK;
        }
    }
    err = "no full-rank H_o without repeated rows after 64 annealing runs";
    return BCH_ESTATE;
}

}  // namespace bch
