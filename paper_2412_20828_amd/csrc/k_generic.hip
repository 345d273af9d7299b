// Generic HIP kernels for gfx950: normalized min-sum decoding of any
// parity-check matrix in any of the three message-memory modes, the syndrome
// test of eq. 5 and the int8 quantiser of the fixed-point input.
//
// Layout: one lane per frame, 64 frames per workgroup (one wave).  The
// frame's posterior y and the branch-merge accumulator live in LDS as
// structure-of-arrays [coordinate][lane], so a lane gathering y at its own
// permuted coordinate never conflicts with the other lanes (bank = lane).
// The matrix rows (CSR) are wave-uniform and are read through the scalar
// cache.  Edge memories of the memory modes live in the device workspace as
// [branch][edge][frame] so that every access is coalesced.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "philox.h"

namespace bch {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int pmod(int x, int n) { return x < 0 ? x + n : x; }

// frames' codeword bits -> zero syndrome with the packed rows of hsyn
__device__ __forceinline__ bool syndrome_zero(const uint64_t *w, int W64,
                                              const uint64_t *__restrict__ hsyn, int msyn)
{
    uint32_t odd = 0;
    for (int r = 0; r < msyn; r++) {
        uint32_t cnt = 0;
        for (int k = 0; k < W64; k++)
            cnt += __popcll(w[k] & hsyn[r * W64 + k]);
        odd |= cnt;
    }
    return (odd & 1u) == 0;
}

template <int MODE>
__global__ void __launch_bounds__(WAVE) nms_generic_fp32(GenericArgs a)
{
    extern __shared__ float sm[];
    const int N = a.N;
    float *ys = sm;             // [N][64] current posterior y^(t-1)
    float *acc = sm + N * WAVE; // [N][64] sum over branches of c2v at its coordinate
    const int lane = threadIdx.x;
    const int64_t f = (int64_t)blockIdx.x * WAVE + lane;
    const bool live = f < a.F;
    const float *llr = static_cast<const float *>(a.llr);
    for (int u = 0; u < N; u++)
        ys[u * WAVE + lane] = live ? llr[f * a.ld + u] + 0.0f : 1.0f;
    const int B = a.B;
    const int dp = a.dp;
    // d_o is taken modulo d_p, as by the specialised kernels' bucketing
    const int d_o = (live && B > 1) ? (int)a.d_o[f] % dp : 0;
    const int np = (B == 9) ? 3 : 1;
    const int mult[3] = {1, 2, (N + 1) / 2};
    bool done = !live;
    int it_out = a.max_iter;
    uint64_t word[2] = {0, 0};
    const int64_t F = a.F;
    for (int t = 1; t <= a.max_iter; t++) {
        for (int u = 0; u < N; u++)
            acc[u * WAVE + lane] = 0.0f;
        float *s_prev = a.ws_s + (size_t)((t + 1) & 1) * B * N * F;
        float *s_new = a.ws_s + (size_t)(t & 1) * B * N * F;
        for (int b = 0; b < B; b++) {
            const int p = b % np;
            const int s = b / np;
            const int sh = (B == 1) ? 0 : s * dp + d_o;
            const int cb = (mult[p] * sh) % N;
            const uint8_t *colp = a.colp + (size_t)p * a.E;
            if (MODE == BCH_MODE_MEMORY && live)
                for (int i = 0; i < N; i++)
                    s_new[((size_t)b * N + i) * F + f] = 0.0f;
            for (int j = 0; j < a.M; j++) {
                const int e0 = a.rowptr[j], e1 = a.rowptr[j + 1];
                float min1 = INFINITY, min2 = INFINITY;
                uint32_t neg = 0;
                for (int e = e0; e < e1; e++) {
                    const int idx = pmod((int)colp[e] - cb, N);
                    float v = ys[idx * WAVE + lane];
                    if (MODE != BCH_MODE_RESTART && t > 1 && live) {
                        v -= a.ws_c2v[((size_t)b * a.E + e) * F + f];
                        if (MODE == BCH_MODE_MEMORY)
                            v += s_prev[((size_t)b * N + a.colp[e]) * F + f];
                    }
                    const float m = fabsf(v);
                    if (m < min1) {
                        min2 = min1;
                        min1 = m;
                    } else if (m < min2) {
                        min2 = m;
                    }
                    neg ^= (v < 0.0f) ? 1u : 0u;
                }
                for (int e = e0; e < e1; e++) {
                    const int idx = pmod((int)colp[e] - cb, N);
                    float v = ys[idx * WAVE + lane];
                    float *mem = a.ws_c2v + ((size_t)b * a.E + e) * F + f;
                    if (MODE != BCH_MODE_RESTART && t > 1 && live) {
                        v -= *mem;
                        if (MODE == BCH_MODE_MEMORY)
                            v += s_prev[((size_t)b * N + a.colp[e]) * F + f];
                    }
                    const float m = (fabsf(v) == min1) ? min2 : min1;
                    const bool ng = (neg ^ ((v < 0.0f) ? 1u : 0u)) != 0;
                    const float am = a.alpha * m;
                    const float c2v = ng ? -am : am;
                    if (MODE != BCH_MODE_RESTART && live)
                        *mem = c2v;
                    if (MODE == BCH_MODE_MEMORY && live)
                        s_new[((size_t)b * N + a.colp[e]) * F + f] += c2v;
                    acc[idx * WAVE + lane] += c2v;
                }
            }
        }
        // posterior (eq. 4 with the branch average), decision, syndrome
        word[0] = word[1] = 0;
        const float invB = (float)B;
        for (int u = 0; u < N; u++) {
            const float base = (MODE == BCH_MODE_EXTRINSIC) ? (live ? llr[f * a.ld + u] + 0.0f : 1.0f)
                                                            : ys[u * WAVE + lane];
            const float yn = base + acc[u * WAVE + lane] / invB;
            if (!done) {
                ys[u * WAVE + lane] = yn;
                if (a.trace)
                    a.trace[((size_t)f * a.max_iter + (t - 1)) * a.ld_trace + u] = yn;
            }
            if (yn < 0.0f)
                word[u >> 6] |= 1ull << (u & 63);
        }
        if (!done && syndrome_zero(word, a.W64, a.hsyn, a.msyn)) {
            done = true;
            it_out = t;
            for (int k = 0; k < a.W64; k++)
                a.bits[f * a.W64 + k] = word[k];
            a.iters[f] = (uint8_t)t;
            a.flags[f] = 1;
        }
        if (__all(done))
            break;
    }
    if (!done) {
        for (int k = 0; k < a.W64; k++)
            a.bits[f * a.W64 + k] = word[k];
        a.iters[f] = (uint8_t)it_out;
        a.flags[f] = 0;
    }
}

__global__ void syndrome_kernel(const uint64_t *__restrict__ bits, int64_t F, int W64,
                                const uint64_t *__restrict__ hsyn, int msyn,
                                uint8_t *__restrict__ ok)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F)
        return;
    uint64_t w[2] = {0, 0};
    for (int k = 0; k < W64; k++)
        w[k] = bits[f * W64 + k];
    ok[f] = syndrome_zero(w, W64, hsyn, msyn) ? 1 : 0;
}

__global__ void quantize_kernel(const float *__restrict__ llr, int64_t ld, int64_t F, int N,
                                float scale, int8_t *__restrict__ q, int64_t ldq)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t f = idx / ldq;
    const int i = (int)(idx % ldq);
    if (f >= F)
        return;
    int8_t out = 0;
    if (i < N) {
        // roundf rounds half away from zero without forming |x| + 0.5 (which
        // itself rounds, e.g. 0.49999997 + 0.5 = 1.0 in FP32)
        const float r = fminf(fmaxf(roundf(llr[f * ld + i] * scale), -127.0f), 127.0f);
        out = (int8_t)(int)r;
    }
    q[f * ldq + i] = out;
}

__global__ void draw_offsets_kernel(uint64_t seed, uint64_t key_hi, int64_t base, int64_t F, int dp,
                                    uint8_t *__restrict__ d_o)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < F)
        d_o[f] = draw_offset(seed, key_hi, (uint64_t)(base + f), dp);
}

}  // namespace

hipError_t launch_draw_offsets(uint64_t seed, uint64_t key_hi, int64_t base, int64_t F, int dp, uint8_t *d_o,
                               hipStream_t stream)
{
    const dim3 grid((unsigned)((F + 255) / 256));
    hipLaunchKernelGGL(draw_offsets_kernel, grid, dim3(256), 0, stream, seed, key_hi, base, F, dp, d_o);
    return hipGetLastError();
}

hipError_t launch_generic_fp32(const GenericArgs &a, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.F + WAVE - 1) / WAVE));
    const size_t lds = (size_t)2 * a.N * WAVE * sizeof(float);
    switch (a.mode) {
    case BCH_MODE_RESTART:
        hipLaunchKernelGGL(nms_generic_fp32<BCH_MODE_RESTART>, grid, dim3(WAVE), lds, stream, a);
        break;
    case BCH_MODE_MEMORY:
        hipLaunchKernelGGL(nms_generic_fp32<BCH_MODE_MEMORY>, grid, dim3(WAVE), lds, stream, a);
        break;
    default:
        hipLaunchKernelGGL(nms_generic_fp32<BCH_MODE_EXTRINSIC>, grid, dim3(WAVE), lds, stream, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_syndrome(const uint64_t *bits, int64_t F, int W64, const uint64_t *hsyn,
                           int msyn, uint8_t *ok, hipStream_t stream)
{
    const dim3 grid((unsigned)((F + 255) / 256));
    hipLaunchKernelGGL(syndrome_kernel, grid, dim3(256), 0, stream, bits, F, W64, hsyn, msyn, ok);
    return hipGetLastError();
}

hipError_t launch_quantize(const float *llr, int64_t ld, int64_t F, int N, float scale,
                           int8_t *q, int64_t ldq, hipStream_t stream)
{
    const int64_t total = F * ldq;
    const dim3 grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, stream, llr, ld, F, N, scale, q, ldq);
    return hipGetLastError();
}

}  // namespace bch
