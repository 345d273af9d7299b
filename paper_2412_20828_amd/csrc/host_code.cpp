// Code algebra of binary primitive narrow-sense BCH codes: GF(2^m) from a
// primitive polynomial, generator polynomial as the product of the distinct
// minimal polynomials of alpha^1..alpha^{2t}, check polynomial h = (x^N+1)/g,
// systematic generator rows and the banded standard parity-check rows
// x^i h~(x) (Table 1's standard matrices).  Polynomials over GF(2) are held as
// packed rows (bit k = coefficient of x^k).
#include <cstring>

#include "internal.h"

namespace bch {

Row rotate(const Row &r, int N, int q)
{
    q %= N;
    if (q < 0)
        q += N;
    Row out;
    if (q == 0)
        return r;
    for (int c = 0; c < N; c++)
        if (r.get(c))
            out.set((c + q) % N);
    return out;
}

int overlap(const Row &a, const Row &b)
{
    return __builtin_popcountll(a.w[0] & b.w[0]) + __builtin_popcountll(a.w[1] & b.w[1]);
}

namespace {

// polynomial over GF(2) of degree <= 255 as a bit array
struct Poly {
    uint64_t w[4] = {0, 0, 0, 0};
    bool get(int k) const { return (w[k >> 6] >> (k & 63)) & 1u; }
    void flip(int k) { w[k >> 6] ^= 1ull << (k & 63); }
    int degree() const
    {
        for (int k = 255; k >= 0; k--)
            if (get(k))
                return k;
        return -1;
    }
};

// remainder of a(x) modulo b(x), quotient optionally returned
Poly poly_mod(Poly a, const Poly &b, Poly *quot)
{
    int db = b.degree();
    Poly q;
    for (int d = a.degree(); d >= db; d--) {
        if (!a.get(d))
            continue;
        q.flip(d - db);
        for (int k = 0; k <= db; k++)
            if (b.get(k))
                a.flip(d - db + k);
    }
    if (quot)
        *quot = q;
    return a;
}

}  // namespace

int build_code(int m, uint32_t prim, int t, Code &out, std::string &err)
{
    if (m < 3 || m > 7) {
        err = "m must be in [3, 7]";
        return BCH_EUNSUPPORTED;
    }
    const int N = (1 << m) - 1;
    if (t < 1 || 2 * t >= N) {
        err = "t out of range";
        return BCH_EINVAL;
    }
    // antilog table alpha^i, checking that prim is primitive
    std::vector<int> alog(N), lg(N + 1, -1);
    int x = 1;
    for (int i = 0; i < N; i++) {
        if (lg[x] >= 0) {
            err = "polynomial is not primitive";
            return BCH_EINVAL;
        }
        alog[i] = x;
        lg[x] = i;
        x <<= 1;
        if (x >> m)
            x ^= (int)prim;
    }
    if (x != 1 || (prim >> m) != 1) {
        err = "polynomial is not primitive of degree m";
        return BCH_EINVAL;
    }
    auto mul = [&](int a, int b) { return (a && b) ? alog[(lg[a] + lg[b]) % N] : 0; };
    // product of (x - alpha^j) over the union of cyclotomic cosets of 1..2t,
    // coefficients in GF(2^m), lowest degree first
    std::vector<int> poly{1};
    std::vector<char> in_union(N, 0);
    for (int i = 1; i <= 2 * t; i++) {
        int r = i % N;
        if (in_union[r])
            continue;
        int j = r;
        do {
            in_union[j] = 1;
            std::vector<int> next(poly.size() + 1, 0);
            for (size_t k = 0; k < poly.size(); k++) {
                next[k + 1] ^= poly[k];
                next[k] ^= mul(poly[k], alog[j]);
            }
            poly.swap(next);
            j = (2 * j) % N;
        } while (j != r);
    }
    Poly g;
    for (size_t k = 0; k < poly.size(); k++) {
        if (poly[k] > 1) {
            err = "generator coefficient outside GF(2)";
            return BCH_ESTATE;
        }
        if (poly[k])
            g.flip((int)k);
    }
    const int dg = (int)poly.size() - 1;
    const int K = N - dg;
    Poly xn1;
    xn1.flip(0);
    xn1.flip(N);
    Poly h;
    Poly rem = poly_mod(xn1, g, &h);
    if (rem.degree() >= 0) {
        err = "g does not divide x^N + 1";
        return BCH_ESTATE;
    }
    out.m = m;
    out.N = N;
    out.K = K;
    out.t = t;
    out.prim = prim;
    out.g.assign(dg + 1, 0);
    for (int k = 0; k <= dg; k++)
        out.g[k] = g.get(k);
    out.G.assign(K, Row());
    for (int k = 0; k < K; k++) {
        Poly mono;
        mono.flip(N - K + k);
        Poly par = poly_mod(mono, g, nullptr);
        Row row;
        for (int i = 0; i < dg; i++)
            if (par.get(i))
                row.set(i);
        row.set(N - K + k);
        out.G[k] = row;
    }
    // h~(x) = x^K h(1/x); row i = x^i h~(x)
    out.Hstd.assign(N - K, Row());
    for (int i = 0; i < N - K; i++)
        for (int e = 0; e <= K; e++)
            if (h.get(K - e))
                out.Hstd[i].set(i + e);
    return BCH_OK;
}

int gf2_rank(std::vector<Row> rows, int N)
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
    return r;
}

int shift_period(int N)
{
    if (N == 63)
        return 21;
    if (N == 127)
        return 42;
    return N / 3;
}

// Gather maps of the automorphism block: branch b = 3s + p reads
// y[(a_p * (j - sh_s)) mod N], a_p in {1, 2, (N+1)/2}, sh_s = s*d_p + d_o.
int branch_maps(int N, int B, int d_o, int16_t *maps)
{
    const int dp = shift_period(N);
    if (B != 1 && B != 3 && B != 9)
        return BCH_EINVAL;
    if (d_o < 0 || (B > 1 && d_o >= dp))
        return BCH_EINVAL;
    const int mult[3] = {1, 2, (N + 1) / 2};
    const int np = B == 9 ? 3 : 1, ns = B == 1 ? 1 : 3;
    for (int s = 0; s < ns; s++)
        for (int p = 0; p < np; p++) {
            const int b = s * np + p;
            const int sh = B == 1 ? 0 : s * dp + d_o;
            for (int j = 0; j < N; j++) {
                int k = ((j - sh) % N + N) % N;
                maps[b * N + j] = (int16_t)((mult[p] * k) % N);
            }
        }
    return BCH_OK;
}

}  // namespace bch
