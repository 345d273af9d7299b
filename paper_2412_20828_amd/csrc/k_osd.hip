// Order-p ordered statistics decoding on the device (Section II-B), the second
// stage of the hybrid decoder run next to the NMS kernels: one wave per frame,
// frames whose skip byte is set are left alone.
//
// Per frame, exactly the host algorithm:
//   1. reliabilities r_u = |L_u| and hard decisions z;
//   2. positions ordered by reliability, descending, ties by index (each
//      lane counts how many positions precede its own);
//   3. most reliable basis by greedy Gaussian elimination on the generator
//      rows in that column order (row k of the working matrix sits in lane
//      k mod 64, slot k / 64; a row swap moves data between lanes);
//   4. base candidate c0 = sum of the rows whose basis decision is 1;
//   5. candidates c0 + (up to p rows), in the order weight 0, weight 1
//      (ascending), weight 2 (lexicographic); cost = sum of r over the
//      positions where the candidate disagrees with z, in FP64, ascending
//      position; the first candidate of least cost wins.
// The candidates are spread over the lanes and scored in two passes.  The
// first uses r quantised to 16 bits (q_u = round(r_u 2^s), s per frame), an
// integer weighted popcount over bit-planes of q that the wave builds with
// ballots; each candidate's quantised cost is within 63.5 units of 2^s times
// its exact cost, and it is kept in LDS (written and read by the same lane):
// as a word for up to KEEP_MAX candidates, else as a half-word saturated at
// 65535, which the second pass recomputes only when the threshold below
// reaches 65535.  The second pass computes the exact FP64 cost of every
// candidate whose quantised cost is within 128 units of the smallest,
// which includes every candidate of least exact cost, and the wave picks the
// least exact cost, then the first candidate.  The result is therefore the
// host's.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace bch {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t rd(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
// old with lane l's value replaced by v
__device__ __forceinline__ uint32_t wr(uint32_t v, int l, uint32_t old)
{
    return (int)threadIdx.x == l ? v : old;
}

// candidate key -> rows: key 0 = c0, 1..K = one row, then the pairs in
// lexicographic order.  Only for keys below 1 + K + K (K - 1) / 2.
__device__ __forceinline__ void key_rows(int key, int K, int &k1, int &k2)
{
    k1 = -1;
    k2 = -1;
    if (key == 0)
        return;
    if (key <= K) {
        k1 = key - 1;
        return;
    }
    int p = key - 1 - K;
    int a = 0;
    while (p >= K - 1 - a) {  // ends at a <= K - 2 for a valid key
        p -= K - 1 - a;
        a++;
    }
    k1 = a;
    k2 = a + 1 + p;
}

// rows of key, given those of key - WAVE (valid keys only)
__device__ __forceinline__ void next_rows(int key, int K, int &k1, int &k2)
{
    if (key <= K) {
        k1 = key - 1;
        k2 = -1;
        return;
    }
    if (k2 < 0) {
        key_rows(key, K, k1, k2);
        return;
    }
    k2 += WAVE;
    while (k2 >= K) {  // carry into the next row(s); stays below K - 1 for a valid key
        const int over = k2 - K;
        k1++;
        k2 = k1 + 1 + over;
    }
}

// pass-1 costs kept in LDS as words up to this many candidates (9 KB; every
// order-2 search with K <= 67); larger searches keep saturated half-words
// (at most 16.5 KB for K = 128): a word each, 20 KB for K = 99, cut the
// resident waves per CU and measured slower than recomputing.
constexpr int KEEP_MAX = 2304;

// candidates of an order-p search over K basis rows (p = 0, 1 or 2)
__host__ __device__ inline int n_candidates(int order, int K)
{
    return order <= 0 ? 1 : (order == 1 ? 1 + K : 1 + K + K * (K - 1) / 2);
}

__global__ void __launch_bounds__(WAVE) osd_kernel(OsdArgs A)
{
    extern __shared__ uint32_t qv[];  // [n_candidates] quantised costs of pass 1
    __shared__ float r[128];
    __shared__ uint32_t rowl[128][4];  // working generator rows after elimination
    __shared__ int mrb[128];
    const int lane = threadIdx.x;
    const int N = A.N, K = A.K;
    for (int64_t f = blockIdx.x; f < A.F; f += gridDim.x) {
        if ((A.skip && A.skip[f]) || (A.code_idx && A.code_idx[f] != A.code))
            continue;
        const float *L = A.llr + f * A.ld;
        const bool in0 = lane < N, in1 = lane + WAVE < N;
        const float l0 = in0 ? L[lane] : 0.0f, l1 = in1 ? L[lane + WAVE] : 0.0f;
        const float r0 = fabsf(l0), r1 = fabsf(l1);
        const uint64_t z0 = __ballot(in0 && l0 < 0.0f), z1 = __ballot(in1 && l1 < 0.0f);
        r[lane] = r0;
        r[lane + WAVE] = r1;
        __syncthreads();
        // ---- rank of each position: higher reliability first, ties by index
        int rk0 = 0, rk1 = 0;
        for (int j = 0; j < N; j++) {
            const float rj = r[j];
            rk0 += (rj > r0 || (rj == r0 && j < lane)) ? 1 : 0;
            rk1 += (rj > r1 || (rj == r1 && j < lane + WAVE)) ? 1 : 0;
        }
        // ---- greedy elimination; row k in lane k & 63, slot k >> 6
        uint32_t a[4], b[4];
#pragma unroll
        for (int w = 0; w < 4; w++) {
            a[w] = lane < K ? A.G[lane * 4 + w] : 0u;
            b[w] = lane + WAVE < K ? A.G[(lane + WAVE) * 4 + w] : 0u;
        }
        int piv = 0;
        for (int pos = 0; pos < N && piv < K; pos++) {
            // the column of rank pos (one lane holds it)
            const uint64_t m0 = __ballot(in0 && rk0 == pos), m1 = __ballot(in1 && rk1 == pos);
            // (ranks are distinct, so one lane matches; the masks only keep a
            // malformed input inside the arrays)
            const int col = (m0 ? __builtin_ctzll(m0) : WAVE + __builtin_ctzll(m1 | (1ull << 63))) & 127;
            const int cw = (col >> 5) & 3;
            const uint32_t cb = 1u << (col & 31);
            const uint64_t h0 = __ballot(lane < K && lane >= piv && (a[cw] & cb));
            const uint64_t h1 = __ballot(lane + WAVE < K && lane + WAVE >= piv && (b[cw] & cb));
            if (!h0 && !h1)
                continue;
            const int k0 = h0 ? __builtin_ctzll(h0) : WAVE + __builtin_ctzll(h1);
            uint32_t pr[4];
#pragma unroll
            for (int w = 0; w < 4; w++)
                pr[w] = k0 < WAVE ? rd(a[w], k0) : rd(b[w], k0 - WAVE);
            if (k0 != piv) {
                uint32_t qr[4];
#pragma unroll
                for (int w = 0; w < 4; w++)
                    qr[w] = piv < WAVE ? rd(a[w], piv) : rd(b[w], piv - WAVE);
#pragma unroll
                for (int w = 0; w < 4; w++) {
                    if (k0 < WAVE)
                        a[w] = wr(qr[w], k0, a[w]);
                    else
                        b[w] = wr(qr[w], k0 - WAVE, b[w]);
                    if (piv < WAVE)
                        a[w] = wr(pr[w], piv, a[w]);
                    else
                        b[w] = wr(pr[w], piv - WAVE, b[w]);
                }
            }
            if (lane < K && lane != piv && (a[cw] & cb)) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    a[w] ^= pr[w];
            }
            if (lane + WAVE < K && lane + WAVE != piv && (b[cw] & cb)) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    b[w] ^= pr[w];
            }
            if (lane == 0)
                mrb[piv] = col;
            piv++;
        }
        // ---- rows to LDS, base candidate c0 and d0 = c0 + z
#pragma unroll
        for (int w = 0; w < 4; w++) {
            if (lane < K)
                rowl[lane][w] = a[w];
            if (lane + WAVE < K)
                rowl[lane + WAVE][w] = b[w];
        }
        __syncthreads();
        uint32_t c[4] = {0u, 0u, 0u, 0u};
        if (lane < K) {
            const int m = mrb[lane];
            if (((m < WAVE ? z0 : z1) >> (m & 63)) & 1ull)
#pragma unroll
                for (int w = 0; w < 4; w++)
                    c[w] ^= a[w];
        }
        if (lane + WAVE < K) {
            const int m = mrb[lane + WAVE];
            if (((m < WAVE ? z0 : z1) >> (m & 63)) & 1ull)
#pragma unroll
                for (int w = 0; w < 4; w++)
                    c[w] ^= b[w];
        }
#pragma unroll
        for (int w = 0; w < 4; w++)
            for (int s = 1; s < WAVE; s <<= 1)
                c[w] ^= __shfl_xor(c[w], s);
        const uint32_t zw[4] = {(uint32_t)z0, (uint32_t)(z0 >> 32), (uint32_t)z1, (uint32_t)(z1 >> 32)};
        uint32_t d0[4];
#pragma unroll
        for (int w = 0; w < 4; w++)
            d0[w] = __builtin_amdgcn_readfirstlane(c[w] ^ zw[w]);
        // ---- quantised reliabilities and their bit-planes
        float mx = fmaxf(r0, r1);
        for (int s = 1; s < WAVE; s <<= 1)
            mx = fmaxf(mx, __shfl_xor(mx, s));
        const int sc = mx > 0.0f ? 14 - ilogbf(mx) : 0;  // every q below 2^15
        const uint32_t q0 = (uint32_t)rintf(ldexpf(r0, sc)), q1 = (uint32_t)rintf(ldexpf(r1, sc));
        uint32_t pl[16][4];
#pragma unroll
        for (int bp = 0; bp < 16; bp++) {
            const uint64_t p0 = __ballot(in0 && ((q0 >> bp) & 1u)), p1 = __ballot(in1 && ((q1 >> bp) & 1u));
            pl[bp][0] = (uint32_t)p0;
            pl[bp][1] = (uint32_t)(p0 >> 32);
            pl[bp][2] = (uint32_t)p1;
            pl[bp][3] = (uint32_t)(p1 >> 32);
        }
        auto qcost = [&](const uint32_t *x) {
            uint32_t t = 0u;
#pragma unroll
            for (int bp = 0; bp < 16; bp++) {
                const uint32_t n = __builtin_popcount(x[0] & pl[bp][0]) + __builtin_popcount(x[1] & pl[bp][1]) +
                                   __builtin_popcount(x[2] & pl[bp][2]) + __builtin_popcount(x[3] & pl[bp][3]);
                t += n << bp;
            }
            return t;
        };
        const int nk = n_candidates(A.order, K);
        // pass 1: least quantised cost
        uint32_t qmin = 0xffffffffu;
        {
            int k1 = -1, k2 = -1;
            if (lane < nk)
                key_rows(lane, K, k1, k2);
            for (int key = lane; key < nk; key += WAVE) {
                uint32_t x[4];
#pragma unroll
                for (int w = 0; w < 4; w++)
                    x[w] = d0[w] ^ (k1 >= 0 ? rowl[k1][w] : 0u) ^ (k2 >= 0 ? rowl[k2][w] : 0u);
                const uint32_t qc = qcost(x);
                if (A.keep_costs == 1)
                    qv[key] = qc;
                else
                    reinterpret_cast<uint16_t *>(qv)[key] = (uint16_t)(qc < 65535u ? qc : 65535u);
                qmin = qc < qmin ? qc : qmin;
                if (key + WAVE < nk)
                    next_rows(key + WAVE, K, k1, k2);
            }
        }
        for (int s = 1; s < WAVE; s <<= 1) {
            const uint32_t o = __shfl_xor(qmin, s);
            qmin = o < qmin ? o : qmin;
        }
        const uint32_t thr = qmin + 128u;
        // pass 2: exact FP64 cost of the candidates near the least
        double best = 0.0;
        int bkey = 0x7fffffff;
        {
            int k1 = -1, k2 = -1;
            if (lane < nk)
                key_rows(lane, K, k1, k2);
            for (int key = lane; key < nk; key += WAVE) {
                // the stored cost, or 65535 for "at least 65535"
                const uint32_t st = A.keep_costs == 1 ? qv[key] : reinterpret_cast<const uint16_t *>(qv)[key];
                const bool sat = A.keep_costs != 1 && st == 65535u;
                bool near = sat ? thr >= 65535u : st <= thr;
                uint32_t x[4];
                if (near) {
#pragma unroll
                    for (int w = 0; w < 4; w++)
                        x[w] = d0[w] ^ (k1 >= 0 ? rowl[k1][w] : 0u) ^ (k2 >= 0 ? rowl[k2][w] : 0u);
                    if (sat)
                        near = qcost(x) <= thr;
                }
                if (near) {
                    double d = 0.0;
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        uint32_t v = x[w];
                        while (v) {
                            d += (double)r[w * 32 + __builtin_ctz(v)];
                            v &= v - 1u;
                        }
                    }
                    if (bkey == 0x7fffffff || d < best) {
                        best = d;
                        bkey = key;
                    }
                }
                if (key + WAVE < nk)
                    next_rows(key + WAVE, K, k1, k2);
            }
        }
        for (int s = 1; s < WAVE; s <<= 1) {
            const double ob = __shfl_xor(best, s);
            const int ok = __shfl_xor(bkey, s);
            if (ok != 0x7fffffff && (bkey == 0x7fffffff || ob < best || (ob == best && ok < bkey))) {
                best = ob;
                bkey = ok;
            }
        }
        if (lane == 0) {
            int k1 = -1, k2 = -1;
            key_rows(bkey, K, k1, k2);
            uint32_t out[4];
#pragma unroll
            for (int w = 0; w < 4; w++)
                out[w] = d0[w] ^ zw[w] ^ (k1 >= 0 ? rowl[k1][w] : 0u) ^ (k2 >= 0 ? rowl[k2][w] : 0u);
            uint64_t *dst = A.bits + f * A.bits_ld;
            dst[0] = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
            if (N > 64)
                dst[1] = (uint64_t)out[2] | ((uint64_t)out[3] << 32);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_osd(const OsdArgs &args, int n_cu, hipStream_t stream)
{
    OsdArgs A = args;
    if (A.N > 128 || A.K > 128 || A.K < 1)
        return hipErrorInvalidValue;
    int64_t grid = (int64_t)n_cu * 16;
    if (grid > A.F)
        grid = A.F;
    if (grid < 1)
        return hipSuccess;
    const int nk = n_candidates(A.order, A.K);
    A.keep_costs = nk <= KEEP_MAX ? 1 : 2;
    const size_t lds = (A.keep_costs == 1 ? sizeof(uint32_t) : sizeof(uint16_t)) * (size_t)nk;
    hipLaunchKernelGGL(osd_kernel, dim3((unsigned)grid), dim3(WAVE), lds, stream, A);
    return hipGetLastError();
}

}  // namespace bch
