// Bucketing prepass of the specialised decoder: frames are grouped by their
// random cyclic offset d_o so that a wave's 64 frames share every branch
// permutation.  Counting sort without global atomics:
//   1. each block of BLK frames counts its frames per bucket;
//   2. one workgroup scans the per-block counts bucket by bucket (bucket
//      starts, per-block offsets, bucket slices [cursor, end));
//   3. each block places its frames at its offsets plus their rank inside the
//      block (LDS counters).
// Frames keep their input order inside a (block, bucket) up to the LDS-atomic
// ranks; no result depends on that order (every frame is decoded on its own).
// With a code index, either only the frames of one code of a mixed batch are
// taken, or (mixed-code kernels) every frame of codes 0..n_codes-1 goes to
// bucket base[code] + d_o mod d_p of its code.
#include <hip/hip_runtime.h>

#include "mix_launch.h"
#include "spec_launch.h"

namespace bch {

namespace {

constexpr int MAXB = 512;
constexpr int BLK = 2048;   // frames per counting block
constexpr int TPB = 256;    // threads per counting block
constexpr int SCAN = 1024;  // threads of the scan workgroup

// which frames go to which bucket: one code (code_idx null, or the frames
// with code_idx == code), bucket (f ranges / F) nofs + d_o mod dp (offset 0
// when !use; nofs = dp, or 1 when !use); or, with n_codes > 0, every frame of
// code c < n_codes to bucket base[c] + d_o mod dps[c]
struct BucketMap {
    const uint8_t *code_idx;
    int code, dp, use, nofs, ranges;
    int64_t F;
    int n_codes;
    int base[MIX_MAXC + 1];
    int dps[MIX_MAXC];
};

// bucket of frame f, or -1 if the map does not take it
__device__ __forceinline__ int bucket_of(const uint8_t *d_o, int64_t f, const BucketMap &m)
{
    if (m.n_codes > 0) {
        const int c = m.code_idx[f];
        return c < m.n_codes ? m.base[c] + (int)d_o[f] % m.dps[c] : -1;
    }
    if (m.code_idx && m.code_idx[f] != m.code)
        return -1;
    const int r = m.ranges > 1 ? (int)((f >> kRangeChunkLog2) % m.ranges) : 0;
    return r * m.nofs + (m.use ? (int)d_o[f] % m.dp : 0);
}

__global__ void __launch_bounds__(TPB) bucket_count(const uint8_t *__restrict__ d_o, BucketMap m, int64_t F,
                                                    int nb, int *__restrict__ blk_hist)
{
    __shared__ int h[MAXB];
    for (int i = threadIdx.x; i < nb; i += TPB)
        h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BLK;
    for (int k = threadIdx.x; k < BLK; k += TPB) {
        const int64_t f = base + k;
        if (f < F) {
            const int b = bucket_of(d_o, f, m);
            if (b >= 0)
                atomicAdd(&h[b], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += TPB)
        blk_hist[(size_t)blockIdx.x * nb + i] = h[i];
}

// one workgroup: per-block offsets in bucket-major order, bucket slices
__global__ void __launch_bounds__(SCAN) bucket_scan(int *__restrict__ blk_hist, int nblk, int dp, BucketWs w)
{
    __shared__ int bucket_total[MAXB];
    __shared__ int bucket_start[MAXB];
    const int tid = threadIdx.x;
    // one wave per bucket: exclusive prefix over the blocks, 64 blocks at a
    // time with a shuffle scan (no workgroup barriers inside)
    const int lane = tid & 63, wave = tid >> 6;
    for (int d = wave; d < dp; d += SCAN / 64) {
        int carry = 0;
        for (int b0 = 0; b0 < nblk; b0 += 64) {
            const int b = b0 + lane;
            const int c = b < nblk ? blk_hist[(size_t)b * dp + d] : 0;
            int v = c;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(v, off);
                if (lane >= off)
                    v += t;
            }
            if (b < nblk)
                blk_hist[(size_t)b * dp + d] = carry + v - c;  // offset inside the bucket
            carry += __shfl(v, 63);
        }
        if (lane == 0)
            bucket_total[d] = carry;
    }
    __syncthreads();
    if (tid == 0) {
        int start = 0;
        for (int d = 0; d < dp; d++) {
            bucket_start[d] = start;
            start += bucket_total[d];
        }
    }
    __syncthreads();
    if (tid < dp) {
        w.counts[tid] = bucket_total[tid];
        w.cursor[tid] = bucket_start[tid];
        w.end[tid] = bucket_start[tid] + bucket_total[tid];
    }
}

__global__ void __launch_bounds__(TPB) bucket_place(const uint8_t *__restrict__ d_o, BucketMap m, int64_t F,
                                                    int nb, const int *__restrict__ blk_off, BucketWs w)
{
    __shared__ int h[MAXB];
    for (int i = threadIdx.x; i < nb; i += TPB)
        h[i] = w.cursor[i] + blk_off[(size_t)blockIdx.x * nb + i];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BLK;
    for (int k = threadIdx.x; k < BLK; k += TPB) {
        const int64_t f = base + k;
        if (f < F) {
            const int b = bucket_of(d_o, f, m);
            if (b >= 0) {
                const int pos = atomicAdd(&h[b], 1);
                w.order[pos] = (int)f;
            }
        }
    }
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

int64_t n_blocks(int64_t F) { return (F + BLK - 1) / BLK; }

}  // namespace

size_t bucket_ws_bytes(int64_t F, int nb)
{
    const size_t head = align16(sizeof(int) * 3 * (size_t)nb);
    const size_t hist = align16(sizeof(int) * (size_t)n_blocks(F) * nb);
    return head + hist + align16((size_t)F * sizeof(int));
}

BucketWs bucket_ws_carve(void *ws, int64_t F, int nb)
{
    BucketWs w;
    char *p = static_cast<char *>(ws);
    int *h = reinterpret_cast<int *>(p);
    w.counts = h;
    w.cursor = h + nb;
    w.end = h + 2 * nb;
    p += align16(sizeof(int) * 3 * (size_t)nb);
    w.blk_hist = reinterpret_cast<int *>(p);
    p += align16(sizeof(int) * (size_t)n_blocks(F) * nb);
    w.order = reinterpret_cast<int *>(p);
    return w;
}

static hipError_t run_bucketing(const uint8_t *d_o, const BucketMap &m, int64_t F, int nb, const BucketWs &w,
                                hipStream_t stream)
{
    if (nb < 1 || nb > MAXB || F <= 0)
        return hipErrorInvalidValue;
    const int nblk = (int)n_blocks(F);
    hipLaunchKernelGGL(bucket_count, dim3(nblk), dim3(TPB), 0, stream, d_o, m, F, nb, w.blk_hist);
    hipLaunchKernelGGL(bucket_scan, dim3(1), dim3(SCAN), 0, stream, w.blk_hist, nblk, nb, w);
    hipLaunchKernelGGL(bucket_place, dim3(nblk), dim3(TPB), 0, stream, d_o, m, F, nb, w.blk_hist, w);
    return hipGetLastError();
}

hipError_t launch_bucketing(const uint8_t *d_o, const uint8_t *code_idx, int code, int64_t F, int dp,
                            int use_offsets, int ranges, const BucketWs &w, hipStream_t stream)
{
    BucketMap m{};
    m.code_idx = code_idx;
    m.code = code;
    m.dp = dp;
    m.use = use_offsets;
    m.nofs = use_offsets ? dp : 1;
    if (ranges < 1 || ranges > kRangeXcds)
        return hipErrorInvalidValue;
    m.ranges = ranges;
    m.F = F;
    m.n_codes = 0;
    return run_bucketing(d_o, m, F, m.ranges * m.nofs, w, stream);
}

hipError_t launch_bucketing_mixed(const uint8_t *d_o, const uint8_t *code_idx, int n_codes, const int *dps,
                                  int64_t F, const BucketWs &w, hipStream_t stream)
{
    if (n_codes < 1 || n_codes > MIX_MAXC || code_idx == nullptr)
        return hipErrorInvalidValue;
    BucketMap m{};
    m.code_idx = code_idx;
    m.n_codes = n_codes;
    m.base[0] = 0;
    for (int c = 0; c < n_codes; c++) {
        m.dps[c] = dps[c];
        m.base[c + 1] = m.base[c] + dps[c];
    }
    return run_bucketing(d_o, m, F, m.base[n_codes], w, stream);
}

}  // namespace bch
