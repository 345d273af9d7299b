// Internal declarations of the bchnms library (host side and kernel glue).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bchnms.h"

namespace bch {

// A binary row of length N <= 127 packed into two 64-bit words
// (bit i of the pair = coordinate i).
struct Row {
    uint64_t w[2] = {0, 0};
    bool get(int i) const { return (w[i >> 6] >> (i & 63)) & 1u; }
    void set(int i) { w[i >> 6] |= 1ull << (i & 63); }
    void flip(int i) { w[i >> 6] ^= 1ull << (i & 63); }
    int weight() const { return __builtin_popcountll(w[0]) + __builtin_popcountll(w[1]); }
    bool zero() const { return (w[0] | w[1]) == 0; }
    bool operator==(const Row &o) const { return w[0] == o.w[0] && w[1] == o.w[1]; }
    Row operator^(const Row &o) const { Row r; r.w[0] = w[0] ^ o.w[0]; r.w[1] = w[1] ^ o.w[1]; return r; }
    Row operator&(const Row &o) const { Row r; r.w[0] = w[0] & o.w[0]; r.w[1] = w[1] & o.w[1]; return r; }
};

// Cyclic rotation by q positions: out[c] = in[(c - q) mod N].
Row rotate(const Row &r, int N, int q);
int overlap(const Row &a, const Row &b);

struct Code {
    int m = 0, N = 0, K = 0, t = 0;
    uint32_t prim = 0;
    std::vector<uint8_t> g;    // N-K+1 coefficients
    std::vector<Row> G;        // K systematic generator rows
    std::vector<Row> Hstd;     // N-K standard parity-check rows
    // device copy of Hstd (packed as ceil(N/64) words per row) for syndromes
    uint64_t *d_hsyn = nullptr;
    int d_hsyn_dev = -1;
};

struct Pcm {
    int N = 0, M = 0, E = 0, Mr1 = 0;
    uint64_t seed_used = 0;
    std::vector<Row> rows;
};

// code algebra
int build_code(int m, uint32_t prim, int t, Code &out, std::string &err);
int gf2_rank(std::vector<Row> rows, int N);

// H_o construction
int64_t count_4cycles(const std::vector<Row> &H);
std::vector<Row> min_density_pass(const std::vector<Row> &Hr, int N, bool with_shifts);
int build_hopt(const Code &c, const bch_pcm_params &p, Pcm &out, std::string &err);

// automorphism maps
int branch_maps(int N, int B, int d_o, int16_t *maps);
int shift_period(int N);

// OSD
void osd_frame(const Code &c, const float *llr, int order, uint64_t *bits_out);

void set_error(const std::string &msg);

}  // namespace bch
