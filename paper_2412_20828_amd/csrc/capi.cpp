// C-ABI of the bchnms library: handle management, argument validation,
// device tables of a decoder and the dispatch to the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "philox.h"
#include "spec_registry.h"

struct bch_code_s {
    bch::Code c;
};
struct bch_pcm_s {
    bch::Pcm p;
};
struct bch_decoder_s {
    int N = 0, K = 0, M = 0, E = 0, W64 = 1;
    bch_dec_params prm{};
    int dev = -1;
    uint16_t *d_rowptr = nullptr;
    uint8_t *d_colp = nullptr;
    uint64_t *d_hsyn = nullptr;
    uint32_t *d_gen = nullptr;  // [K][4] generator rows (device OSD)
    int msyn = 0;
    int n_cu = 0;
    int waves = 0;  // waves per CU of the persistent grid (0: the kernel's default)
    const bch::SpecKernel *spec = nullptr;        // throughput kernel
    const bch::SpecKernel *spec_small = nullptr;  // small-batch kernel (N = 127), or null
    const bch::SpecKernel *spec_packed = nullptr; // fixed point: packed 16-bit kernel for large calls, or null
    uint64_t fingerprint = 0;                     // of the matrix (mixed-code kernel lookup)
};

namespace bch {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

static int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return BCH_EDEVICE;
}

static std::vector<uint64_t> pack_rows(const std::vector<Row> &rows, int W64)
{
    std::vector<uint64_t> out(rows.size() * W64);
    for (size_t r = 0; r < rows.size(); r++)
        for (int w = 0; w < W64; w++)
            out[r * W64 + w] = rows[r].w[w];
    return out;
}

// device copy of a code's standard rows, made once per code and device
static std::mutex g_hsyn_mu;
static int code_hsyn(bch_code_s *code, uint64_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_hsyn_mu);
    Code &c = code->c;
    if (c.d_hsyn && c.d_hsyn_dev == dev) {
        *out = c.d_hsyn;
        return BCH_OK;
    }
    const int W64 = (c.N + 63) / 64;
    std::vector<uint64_t> h = pack_rows(c.Hstd, W64);
    uint64_t *d = nullptr;
    e = hipMalloc(&d, h.size() * sizeof(uint64_t));
    if (e != hipSuccess)
        return hip_fail(e, "hipMalloc");
    e = hipMemcpy(d, h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(d);
        return hip_fail(e, "hipMemcpy");
    }
    c.d_hsyn = d;
    c.d_hsyn_dev = dev;
    *out = d;
    return BCH_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int waves_of(const bch_decoder_s *d)
{
    return d->waves > 0 ? d->waves : d->spec->waves_per_cu;
}

// fixed point: calls of at least this many frames run the packed 16-bit
// kernel (two frames per lane).  It holds 128 frames per wave, so its drain
// at the end of a call is the longest; measured faster than the 32-bit kernel
// from 4,000,000 frames for N = 127 (1.10x) and at 11,000,000 frames for
// N = 63 (1.09x), slower at 1,000,000 frames for N = 63 (0.73x)
static int64_t packed_min_frames(int N) { return N > 64 ? 4000000 : 8000000; }

// the kernel of a decode of F frames: the small-batch kernel (three waves per
// 64 frames) when it is registered and F gives each CU at most 128 frames
// (measured on the 127-bit codes: 2.7x faster up to 64 frames per CU, 1.2x at
// 128, 0.9x at 256), or when the decoder asks for it always; else the
// throughput kernel
static const bch::SpecKernel *spec_for(const bch_decoder_s *d, int64_t F)
{
    if (d->spec_small && ((d->prm.flags & BCH_DEC_SMALL_ALWAYS) || F <= (int64_t)d->n_cu * 128))
        return d->spec_small;
    if (d->spec_packed && F >= packed_min_frames(d->N))
        return d->spec_packed;
    return d->spec;
}

// device workspace of one specialised decode of up to F frames
static int spec_offsets(const bch_decoder_s *d) { return d->prm.n_branches > 1 ? shift_period(d->N) : 1; }

static int spec_ranges(const bch_decoder_s *d, int64_t F)
{
    return bucket_ranges(F, (d->prm.flags & BCH_DEC_CHUNK_BUCKETS) != 0);
}

static size_t spec_ws_bytes(const bch_decoder_s *d, int64_t F)
{
    size_t n = align256(bucket_ws_bytes(F, spec_ranges(d, F) * spec_offsets(d)));
    if (d->spec->y_global)
        n += align256((size_t)d->n_cu * waves_of(d) * d->N * 64 * sizeof(float));
    return n;
}

// prepass + persistent kernel of one decoder; code_idx / code select the
// frames of a mixed batch (code_idx may be null: every frame)
static int spec_decode(const bch_decoder_s *d, const void *llr, int64_t ld, int64_t F, const uint8_t *d_o,
                       const uint8_t *code_idx, int code, uint64_t *bits, int64_t bits_ld, uint8_t *iters,
                       uint8_t *flags, void *trace, void *workspace, hipStream_t stream)
{
    const int dp = shift_period(d->N);
    const int ranges = spec_ranges(d, F);
    const int nb = ranges * spec_offsets(d);
    char *ws = static_cast<char *>(workspace);
    BucketWs w = bucket_ws_carve(ws, F, nb);
    hipError_t e = launch_bucketing(d_o, code_idx, code, F, dp, d->prm.n_branches > 1, ranges, w, stream);
    if (e != hipSuccess)
        return hip_fail(e, "bucketing prepass");
    SpecLaunch s{};
    s.llr = llr;
    s.ld = ld;
    s.order = w.order;
    s.bcur = w.cursor;
    s.bend = w.end;
    s.n_offsets = spec_offsets(d);
    s.n_ranges = ranges;
    s.n_buckets = nb;
    s.bits = bits;
    s.bits_ld = bits_ld;
    s.iters = iters;
    s.flags = flags;
    s.trace = trace;
    s.yscratch = d->spec->y_global
                     ? reinterpret_cast<float *>(ws + align256(bucket_ws_bytes(F, nb)))
                     : nullptr;
    s.max_iter = d->prm.max_iter;
    s.alpha = d->prm.alpha;
    // no more persistent waves than a batch of F frames can keep busy (small
    // batches launch small grids): ceil(F / frames per workgroup) + dp
    // workgroups of wave_group waves.  The tuned waves per CU belong to the
    // throughput kernel.
    const bch::SpecKernel *k = spec_for(d, F);
    const int waves = k == d->spec ? waves_of(d) : k->waves_per_cu;
    const int64_t grid = (int64_t)d->n_cu * waves;
    const int g = k->wave_group;
    const int64_t fw = k->frames_per_wave;
    const int64_t most = g * ((F + fw - 1) / fw + dp);
    if (most < grid)
        e = k->launch(s, 1, (int)most, stream);
    else
        e = k->launch(s, d->n_cu, waves, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "specialised kernel launch");
}

// the mixed-code kernel for decoders decs[0..n) in this order (nine-branch
// restart-mode specialised decoders of one precision), or null
static const bch::MixKernel *mixed_kernel_of(const bch_decoder *decs, int n, int64_t F)
{
    if (n < 2 || n > MIX_MAXC)
        return nullptr;
    uint64_t fps[MIX_MAXC];
    bool forced = false;
    for (int c = 0; c < n; c++) {
        const bch_decoder_s *d = decs[c];
        if (!d || !d->spec || d->prm.n_branches != 9 || d->prm.mode != BCH_MODE_RESTART ||
            d->prm.precision != decs[0]->prm.precision || (d->prm.flags & BCH_DEC_NO_MIXED_KERNEL))
            return nullptr;
        forced = forced || (d->prm.flags & BCH_DEC_MIXED_KERNEL);
        fps[c] = d->fingerprint;
    }
    if (!forced && F >= BCH_MIXED_KERNEL_MAX_FRAMES)
        return nullptr;
    return find_mix_kernel(fps, n, decs[0]->prm.precision);
}

// one code-keyed prepass and one persistent kernel over every frame of the mix
static int mixed_fused(const bch::MixKernel *k, const bch_decoder *decs, int n_codes, const uint8_t *code_idx,
                       const void *llr, int64_t ld, int64_t F, const uint8_t *d_o, uint64_t *bits, int64_t bits_ld,
                       uint8_t *iters, uint8_t *flags, void *workspace, hipStream_t stream)
{
    int dps[MIX_MAXC];
    int nb = 0;
    MixLaunch L{};
    L.n_codes = n_codes;
    L.bbase[0] = 0;
    for (int c = 0; c < n_codes; c++) {
        const bch_decoder_s *d = decs[c];
        dps[c] = shift_period(d->N);
        nb += dps[c];
        L.bbase[c + 1] = nb;
        L.alpha[c] = d->prm.alpha;
        L.max_iter[c] = d->prm.max_iter;
        L.weight[c] = (float)(9 * d->E);
    }
    BucketWs w = bucket_ws_carve(workspace, F, nb);
    hipError_t e = launch_bucketing_mixed(d_o, code_idx, n_codes, dps, F, w, stream);
    if (e != hipSuccess)
        return hip_fail(e, "mixed bucketing prepass");
    L.llr = llr;
    L.ld = ld;
    L.order = w.order;
    L.bcur = w.cursor;
    L.bend = w.end;
    L.counts = w.counts;
    L.n_buckets = nb;
    L.bits = bits;
    L.bits_ld = bits_ld;
    L.iters = iters;
    L.flags = flags;
    // one wave per SIMD, no more waves than the frames can occupy
    const int n_cu = decs[0]->n_cu;
    const int64_t most = (F + 63) / 64 + nb;
    e = most < (int64_t)n_cu * 4 ? k->launch(L, 1, (int)most, stream) : k->launch(L, n_cu, 4, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "mixed-code kernel launch");
}

}  // namespace bch

using namespace bch;

static_assert(BCH_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "scratch size of the header and the library");

extern "C" {

const char *bch_last_error(void) { return g_err.c_str(); }

int bch_load_code(int m, uint32_t prim_poly, int t, bch_code *out)
{
    if (!out)
        return fail(BCH_EINVAL, "out is NULL");
    auto *h = new (std::nothrow) bch_code_s();
    if (!h)
        return fail(BCH_ENOMEM, "allocation failed");
    std::string err;
    int rc = build_code(m, prim_poly, t, h->c, err);
    if (rc) {
        delete h;
        return fail(rc, err);
    }
    *out = h;
    return BCH_OK;
}

int bch_code_info(bch_code code, int *N, int *K, int *t)
{
    if (!code)
        return fail(BCH_EINVAL, "code is NULL");
    if (N)
        *N = code->c.N;
    if (K)
        *K = code->c.K;
    if (t)
        *t = code->c.t;
    return BCH_OK;
}

int bch_code_export(bch_code code, uint8_t *g, uint8_t *G, uint8_t *Hstd)
{
    if (!code)
        return fail(BCH_EINVAL, "code is NULL");
    const Code &c = code->c;
    if (g)
        std::memcpy(g, c.g.data(), c.g.size());
    if (G)
        for (int k = 0; k < c.K; k++)
            for (int i = 0; i < c.N; i++)
                G[(size_t)k * c.N + i] = c.G[k].get(i);
    if (Hstd)
        for (int k = 0; k < c.N - c.K; k++)
            for (int i = 0; i < c.N; i++)
                Hstd[(size_t)k * c.N + i] = c.Hstd[k].get(i);
    return BCH_OK;
}

void bch_code_destroy(bch_code code)
{
    if (!code)
        return;
    if (code->c.d_hsyn)
        (void)hipFree(code->c.d_hsyn);
    delete code;
}

int bch_build_pcm(bch_code code, const bch_pcm_params *params, bch_pcm *out)
{
    if (!code || !params || !out)
        return fail(BCH_EINVAL, "NULL argument");
    auto *h = new (std::nothrow) bch_pcm_s();
    if (!h)
        return fail(BCH_ENOMEM, "allocation failed");
    const Code &c = code->c;
    if (params->kind == BCH_PCM_STD) {
        h->p.N = c.N;
        h->p.M = c.N - c.K;
        h->p.rows = c.Hstd;
        h->p.E = 0;
        for (const Row &r : h->p.rows)
            h->p.E += r.weight();
    } else if (params->kind == BCH_PCM_OPT) {
        std::string err;
        int rc = build_hopt(c, *params, h->p, err);
        if (rc) {
            delete h;
            return fail(rc, err);
        }
    } else {
        delete h;
        return fail(BCH_EINVAL, "unknown PCM kind");
    }
    *out = h;
    return BCH_OK;
}

int bch_pcm_from_dense(bch_code code, const uint8_t *H, int M, bch_pcm *out)
{
    if (!code || !H || !out || M < 1 || M > 1024)
        return fail(BCH_EINVAL, "bad argument");
    const Code &c = code->c;
    std::vector<Row> rows(M);
    for (int r = 0; r < M; r++)
        for (int i = 0; i < c.N; i++) {
            if (H[(size_t)r * c.N + i] > 1)
                return fail(BCH_EINVAL, "matrix entries must be 0 or 1");
            if (H[(size_t)r * c.N + i])
                rows[r].set(i);
        }
    for (int r = 0; r < M; r++) {
        if (rows[r].weight() < 2)
            return fail(BCH_EINVAL, "every row needs weight >= 2");
        for (const Row &g : c.G)
            if (overlap(rows[r], g) & 1)
                return fail(BCH_EINVAL, "row is not a dual codeword");
    }
    if (gf2_rank(rows, c.N) != c.N - c.K)
        return fail(BCH_EINVAL, "matrix rank differs from N-K");
    auto *h = new (std::nothrow) bch_pcm_s();
    if (!h)
        return fail(BCH_ENOMEM, "allocation failed");
    h->p.N = c.N;
    h->p.M = M;
    h->p.rows = rows;
    h->p.E = 0;
    for (const Row &r : rows)
        h->p.E += r.weight();
    *out = h;
    return BCH_OK;
}

int bch_pcm_info(bch_pcm pcm, int *M, int *N, int *E, int64_t *c4, int *Mr1, uint64_t *seed_used)
{
    if (!pcm)
        return fail(BCH_EINVAL, "pcm is NULL");
    if (M)
        *M = pcm->p.M;
    if (N)
        *N = pcm->p.N;
    if (E)
        *E = pcm->p.E;
    if (c4)
        *c4 = count_4cycles(pcm->p.rows);
    if (Mr1)
        *Mr1 = pcm->p.Mr1;
    if (seed_used)
        *seed_used = pcm->p.seed_used;
    return BCH_OK;
}

int bch_pcm_stats(bch_pcm pcm, int *M, int *E, int64_t *c4, double wstats[8])
{
    if (!pcm)
        return fail(BCH_EINVAL, "pcm is NULL");
    const Pcm &p = pcm->p;
    if (M)
        *M = p.M;
    if (E)
        *E = p.E;
    if (c4)
        *c4 = count_4cycles(p.rows);
    if (wstats) {
        // column weights, then row weights: min, max, mean, population std
        std::vector<int> col(p.N, 0), row(p.M, 0);
        for (int r = 0; r < p.M; r++)
            for (int i = 0; i < p.N; i++)
                if (p.rows[r].get(i)) {
                    col[i]++;
                    row[r]++;
                }
        auto fill = [](const std::vector<int> &w, double *o) {
            double s = 0.0, s2 = 0.0;
            int lo = w[0], hi = w[0];
            for (int v : w) {
                s += v;
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            const double mean = s / (double)w.size();
            for (int v : w)
                s2 += (v - mean) * (v - mean);
            o[0] = lo;
            o[1] = hi;
            o[2] = mean;
            o[3] = std::sqrt(s2 / (double)w.size());
        };
        fill(col, wstats);
        fill(row, wstats + 4);
    }
    return BCH_OK;
}

int bch_pcm_export(bch_pcm pcm, uint8_t *dense, size_t cap)
{
    if (!pcm || !dense)
        return fail(BCH_EINVAL, "NULL argument");
    const size_t need = (size_t)pcm->p.M * pcm->p.N;
    if (cap < need)
        return fail(BCH_EINVAL, "buffer too small");
    for (int r = 0; r < pcm->p.M; r++)
        for (int i = 0; i < pcm->p.N; i++)
            dense[(size_t)r * pcm->p.N + i] = pcm->p.rows[r].get(i);
    return BCH_OK;
}

void bch_pcm_destroy(bch_pcm pcm) { delete pcm; }

int bch_make_automorphisms(int N, int n_branches, int d_o, int16_t *maps)
{
    if (!maps || N < 7 || N > 127)
        return fail(BCH_EINVAL, "bad argument");
    int rc = branch_maps(N, n_branches, d_o, maps);
    if (rc)
        return fail(rc, "n_branches must be 1, 3 or 9 and d_o in [0, d_p)");
    return BCH_OK;
}

int bch_draw_offsets(int N, uint64_t seed, uint64_t key_hi, int64_t frame_base, int64_t F, uint8_t *d_o,
                     int on_device, hipStream_t stream)
{
    if (N < 7 || N > 127 || F < 0 || frame_base < 0)
        return fail(BCH_EINVAL, "bad argument (7 <= N <= 127, F >= 0, frame_base >= 0)");
    if (F == 0)
        return BCH_OK;
    if (!d_o)
        return fail(BCH_EINVAL, "d_o is NULL");
    const int dp = shift_period(N);
    if (on_device) {
        hipError_t e = launch_draw_offsets(seed, key_hi, frame_base, F, dp, d_o, stream);
        return e == hipSuccess ? BCH_OK : hip_fail(e, "offset draw kernel launch");
    }
    for (int64_t f = 0; f < F; f++)
        d_o[f] = draw_offset(seed, key_hi, (uint64_t)(frame_base + f), dp);
    return BCH_OK;
}

int bch_draw_offsets_keys(int N, uint64_t seed, int64_t n_keys, const uint64_t *keys, const int64_t *counts,
                          uint8_t *d_o)
{
    if (N < 7 || N > 127 || n_keys < 0)
        return fail(BCH_EINVAL, "bad argument (7 <= N <= 127, n_keys >= 0)");
    if (n_keys == 0)
        return BCH_OK;
    if (!keys || !counts || !d_o)
        return fail(BCH_EINVAL, "NULL argument");
    for (int64_t k = 0; k < n_keys; k++)
        if (counts[k] < 0)
            return fail(BCH_EINVAL, "negative count");
    const int dp = shift_period(N);
    int64_t o = 0;
    for (int64_t k = 0; k < n_keys; k++)
        for (int64_t f = 0; f < counts[k]; f++)
            d_o[o++] = draw_offset(seed, keys[k], (uint64_t)f, dp);
    return BCH_OK;
}

int bch_decoder_create(bch_code code, bch_pcm pcm, const bch_dec_params *params, bch_decoder *out)
{
    if (!code || !pcm || !params || !out)
        return fail(BCH_EINVAL, "NULL argument");
    const Code &c = code->c;
    const Pcm &p = pcm->p;
    if (p.N != c.N)
        return fail(BCH_EINVAL, "PCM and code lengths differ");
    const bch_dec_params &q = *params;
    if (q.n_branches != 1 && q.n_branches != 3 && q.n_branches != 9)
        return fail(BCH_EINVAL, "n_branches must be 1, 3 or 9");
    if (q.mode < BCH_MODE_RESTART || q.mode > BCH_MODE_EXTRINSIC)
        return fail(BCH_EINVAL, "unknown mode");
    if (q.max_iter < 1 || q.max_iter > 64)
        return fail(BCH_EINVAL, "max_iter must be in [1, 64]");
    if (q.precision != BCH_FP32 && q.precision != BCH_FIX8)
        return fail(BCH_EINVAL, "unknown precision");
    if ((q.flags & BCH_DEC_SMALL_ALWAYS) && (q.flags & BCH_DEC_SMALL_NEVER))
        return fail(BCH_EINVAL, "BCH_DEC_SMALL_ALWAYS and BCH_DEC_SMALL_NEVER exclude each other");
    if ((q.flags & BCH_DEC_PACKED16) && (q.flags & BCH_DEC_UNPACKED16))
        return fail(BCH_EINVAL, "BCH_DEC_PACKED16 and BCH_DEC_UNPACKED16 exclude each other");
    if ((q.flags & BCH_DEC_NO_MIXED_KERNEL) && (q.flags & BCH_DEC_MIXED_KERNEL))
        return fail(BCH_EINVAL, "BCH_DEC_NO_MIXED_KERNEL and BCH_DEC_MIXED_KERNEL exclude each other");
    if (q.flags & ~(BCH_DEC_FORCE_GENERIC | BCH_DEC_PACKED16 | BCH_DEC_SMALL_ALWAYS | BCH_DEC_SMALL_NEVER |
                    BCH_DEC_UNPACKED16 | BCH_DEC_NO_MIXED_KERNEL | BCH_DEC_MIXED_KERNEL | BCH_DEC_CHUNK_BUCKETS))
        return fail(BCH_EINVAL, "unknown decoder flags");
    if (p.E > 65535)
        return fail(BCH_EUNSUPPORTED, "too many edges");
    auto *d = new (std::nothrow) bch_decoder_s();
    if (!d)
        return fail(BCH_ENOMEM, "allocation failed");
    d->N = c.N;
    d->K = c.K;
    d->M = p.M;
    d->E = p.E;
    d->W64 = (c.N + 63) / 64;
    d->prm = q;
    // CSR rows (ascending columns) and the three multiplied column tables
    std::vector<uint16_t> rowptr(p.M + 1, 0);
    std::vector<uint8_t> colp(3 * (size_t)p.E);
    const int mult[3] = {1, 2, (c.N + 1) / 2};
    int e = 0;
    for (int r = 0; r < p.M; r++) {
        rowptr[r] = (uint16_t)e;
        for (int i = 0; i < c.N; i++)
            if (p.rows[r].get(i)) {
                for (int k = 0; k < 3; k++)
                    colp[(size_t)k * p.E + e] = (uint8_t)((mult[k] * i) % c.N);
                e++;
            }
    }
    rowptr[p.M] = (uint16_t)e;
    int rc = code_hsyn(code, &d->d_hsyn);
    if (rc) {
        delete d;
        return rc;
    }
    d->msyn = c.N - c.K;
    hipError_t he = hipGetDevice(&d->dev);
    if (he == hipSuccess)
        he = hipMalloc(&d->d_rowptr, rowptr.size() * sizeof(uint16_t));
    if (he == hipSuccess)
        he = hipMalloc(&d->d_colp, colp.size());
    if (he == hipSuccess)
        he = hipMemcpy(d->d_rowptr, rowptr.data(), rowptr.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice);
    if (he == hipSuccess)
        he = hipMemcpy(d->d_colp, colp.data(), colp.size(), hipMemcpyHostToDevice);
    std::vector<uint32_t> gen((size_t)c.K * 4, 0u);
    for (int k = 0; k < c.K; k++)
        for (int w = 0; w < 2; w++) {
            gen[(size_t)k * 4 + 2 * w] = (uint32_t)c.G[k].w[w];
            gen[(size_t)k * 4 + 2 * w + 1] = (uint32_t)(c.G[k].w[w] >> 32);
        }
    if (he == hipSuccess)
        he = hipMalloc(&d->d_gen, gen.size() * sizeof(uint32_t));
    if (he == hipSuccess)
        he = hipMemcpy(d->d_gen, gen.data(), gen.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        bch_decoder_destroy(d);
        return hip_fail(he, "decoder tables");
    }
    if (!(q.flags & BCH_DEC_FORCE_GENERIC)) {
        const bool packed = (q.flags & BCH_DEC_PACKED16) != 0;
        d->spec = find_spec_kernel(p, q, packed ? 1 : 0);
        if (d->spec && !packed && !(q.flags & BCH_DEC_SMALL_NEVER))
            d->spec_small = find_spec_kernel(p, q, 2);
        if (d->spec && !packed && q.precision == BCH_FIX8 && !(q.flags & BCH_DEC_UNPACKED16))
            d->spec_packed = find_spec_kernel(p, q, 1);
    }
    d->fingerprint = pcm_fingerprint(p);
    if (hipDeviceGetAttribute(&d->n_cu, hipDeviceAttributeMultiprocessorCount, d->dev) != hipSuccess ||
        d->n_cu <= 0)
        d->n_cu = 256;
    *out = d;
    return BCH_OK;
}

int bch_decoder_is_specialized(bch_decoder dec) { return dec && dec->spec ? 1 : 0; }

const char *bch_decoder_kernel_name(bch_decoder dec, int64_t F)
{
    if (!dec)
        return "";
    return dec->spec ? spec_for(dec, F)->name : "generic";
}

void bch_decoder_destroy(bch_decoder dec)
{
    if (!dec)
        return;
    if (dec->d_rowptr)
        (void)hipFree(dec->d_rowptr);
    if (dec->d_colp)
        (void)hipFree(dec->d_colp);
    if (dec->d_gen)
        (void)hipFree(dec->d_gen);
    delete dec;
}

size_t bch_decode_workspace_size(bch_decoder dec, int64_t F)
{
    if (!dec || F < 0)
        return 0;
    if (dec->spec)
        return spec_ws_bytes(dec, F);
    if (dec->prm.mode == BCH_MODE_RESTART)
        return 0;
    size_t n = (size_t)dec->prm.n_branches * dec->E * F;
    if (dec->prm.mode == BCH_MODE_MEMORY)
        n += (size_t)2 * dec->prm.n_branches * dec->N * F;
    return n * sizeof(float);
}

int bch_nms_decode_batch(bch_decoder dec, const void *llr, int64_t ld, int64_t F,
                         const uint8_t *d_o, uint64_t *bits, uint8_t *iters, uint8_t *flags,
                         void *y_trace, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!dec)
        return fail(BCH_EINVAL, "decoder is NULL");
    // the frame cursors are 32-bit and may run past a bucket's end by a few
    // grabs of 64; the cap keeps them far from overflow
    if (F < 0 || F > BCH_MAX_FRAMES)
        return fail(BCH_EINVAL, "F out of range");
    if (F == 0)
        return BCH_OK;
    if (!llr || !bits || !iters || !flags)
        return fail(BCH_EINVAL, "NULL buffer");
    if (dec->prm.n_branches > 1 && !d_o)
        return fail(BCH_EINVAL, "d_o required for more than one branch");
    if (ld < dec->N)
        return fail(BCH_EINVAL, "ld < N");
    if (dec->prm.precision != BCH_FP32 && !dec->spec)
        return fail(BCH_EUNSUPPORTED, "fixed-point decoding needs a kernel specialised to this matrix");
    const size_t need = bch_decode_workspace_size(dec, F);
    if (need && (!workspace || ws_bytes < need))
        return fail(BCH_ENOMEM, "workspace too small");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dec->dev)
        return fail(BCH_EINVAL, "decoder belongs to another device");
    if (dec->spec)
        return spec_decode(dec, llr, ld, F, d_o, nullptr, 0, bits, dec->W64, iters, flags, y_trace, workspace,
                           stream);
    GenericArgs a{};
    a.llr = llr;
    a.ld = ld;
    a.F = F;
    a.d_o = d_o;
    a.bits = bits;
    a.iters = iters;
    a.flags = flags;
    a.trace = static_cast<float *>(y_trace);
    a.ld_trace = ld;
    a.rowptr = dec->d_rowptr;
    a.colp = dec->d_colp;
    a.hsyn = dec->d_hsyn;
    a.msyn = dec->msyn;
    a.W64 = dec->W64;
    a.N = dec->N;
    a.M = dec->M;
    a.E = dec->E;
    a.B = dec->prm.n_branches;
    a.dp = shift_period(dec->N);
    a.mode = dec->prm.mode;
    a.max_iter = dec->prm.max_iter;
    a.alpha = dec->prm.alpha;
    float *ws = static_cast<float *>(workspace);
    a.ws_c2v = ws;
    a.ws_s = ws ? ws + (size_t)a.B * a.E * F : nullptr;
    hipError_t e = launch_generic_fp32(a, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "generic kernel launch");
}

int bch_nms_decode_batch_noalloc(bch_decoder dec, const void *llr, int64_t ld, int64_t F, const uint8_t *d_o,
                                 uint64_t *bits, uint8_t *iters, uint8_t *flags, void *y_trace, hipStream_t stream)
{
    if (!dec)
        return fail(BCH_EINVAL, "decoder is NULL");
    if (F < 0 || F > BCH_MAX_FRAMES)
        return fail(BCH_EINVAL, "F out of range");
    const size_t need = bch_decode_workspace_size(dec, F);
    if (need > BCH_NOALLOC_SCRATCH_BYTES)
        return fail(BCH_EINVAL, "decode of " + std::to_string(F) + " frames needs " + std::to_string(need) +
                                    " bytes of workspace, above the " + std::to_string(BCH_NOALLOC_SCRATCH_BYTES) +
                                    "-byte device scratch of the allocation-free entry point");
    void *ws = nullptr;
    if (need) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != dec->dev)
            return fail(BCH_EINVAL, "decoder belongs to another device");
        hipError_t e = noalloc_scratch(&ws);
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress of the decode scratch");
    }
    return bch_nms_decode_batch(dec, llr, ld, F, d_o, bits, iters, flags, y_trace, ws, need, stream);
}

int bch_decoder_set_tuning(bch_decoder dec, int waves_per_cu)
{
    if (!dec)
        return fail(BCH_EINVAL, "decoder is NULL");
    if (waves_per_cu < 0 || waves_per_cu > 16)
        return fail(BCH_EINVAL, "waves_per_cu must be in [0, 16]");
    dec->waves = waves_per_cu;
    return BCH_OK;
}

size_t bch_mixed_workspace_size(const bch_decoder *decs, int n_codes, int64_t F)
{
    if (!decs || n_codes < 1 || n_codes > BCH_MAX_MIX || F < 0)
        return 0;
    size_t n = 0;
    for (int c = 0; c < n_codes; c++) {
        if (!decs[c] || !decs[c]->spec)
            return 0;
        n += spec_ws_bytes(decs[c], F);
    }
    return n;
}

int bch_mixed_decode_batch(const bch_decoder *decs, int n_codes, const uint8_t *code_idx, const void *llr,
                           int64_t ld, int64_t F, const uint8_t *d_o, uint64_t *bits, int64_t bits_ld,
                           uint8_t *iters, uint8_t *flags, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!decs || n_codes < 1 || n_codes > BCH_MAX_MIX)
        return fail(BCH_EINVAL, "n_codes must be in [1, BCH_MAX_MIX]");
    // the frame cursors are 32-bit and may run past a bucket's end by a few
    // grabs of 64; the cap keeps them far from overflow
    if (F < 0 || F > BCH_MAX_FRAMES)
        return fail(BCH_EINVAL, "F out of range");
    if (F == 0)
        return BCH_OK;
    if (!code_idx || !llr || !d_o || !bits || !iters || !flags)
        return fail(BCH_EINVAL, "NULL buffer");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return fail(BCH_EDEVICE, "hipGetDevice failed");
    for (int c = 0; c < n_codes; c++) {
        const bch_decoder_s *d = decs[c];
        if (!d || !d->spec)
            return fail(BCH_EUNSUPPORTED, "every decoder of a mixed batch needs a specialised kernel");
        if (d->dev != cur)
            return fail(BCH_EINVAL, "decoder belongs to another device");
        if (d->prm.precision != decs[0]->prm.precision)
            return fail(BCH_EINVAL, "decoders of a mixed batch must share the precision");
        if (ld < d->N || bits_ld < d->W64)
            return fail(BCH_EINVAL, "ld or bits_ld too small for a code of the mix");
    }
    const size_t need = bch_mixed_workspace_size(decs, n_codes, F);
    if (!workspace || ws_bytes < need)
        return fail(BCH_ENOMEM, "workspace too small");
    if (const bch::MixKernel *k = mixed_kernel_of(decs, n_codes, F))
        return mixed_fused(k, decs, n_codes, code_idx, llr, ld, F, d_o, bits, bits_ld, iters, flags, workspace,
                           stream);
    char *ws = static_cast<char *>(workspace);
    for (int c = 0; c < n_codes; c++) {
        int rc = spec_decode(decs[c], llr, ld, F, d_o, code_idx, c, bits, bits_ld, iters, flags, nullptr, ws,
                             stream);
        if (rc)
            return rc;
        ws += spec_ws_bytes(decs[c], F);
    }
    return BCH_OK;
}

const char *bch_mixed_kernel_name(const bch_decoder *decs, int n_codes, int64_t F)
{
    if (!decs || n_codes < 1 || n_codes > BCH_MAX_MIX || F < 0)
        return "";
    const bch::MixKernel *k = mixed_kernel_of(decs, n_codes, F);
    return k ? k->name : "per-code";
}

int bch_osd_decode_device(bch_decoder dec, const float *llr, int64_t ld, int64_t F, int order,
                          const uint8_t *skip, uint64_t *bits, int64_t bits_ld, hipStream_t stream)
{
    if (!dec || F < 0 || order < 0 || order > 2)
        return fail(BCH_EINVAL, "bad argument (order must be 0, 1 or 2)");
    if (F == 0)
        return BCH_OK;
    if (!llr || !bits)
        return fail(BCH_EINVAL, "NULL buffer");
    if (ld < dec->N || bits_ld < dec->W64)
        return fail(BCH_EINVAL, "ld or bits_ld too small");
    if (dec->N > 128 || dec->K > 128)
        return fail(BCH_EUNSUPPORTED, "device OSD needs N, K <= 128");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dec->dev)
        return fail(BCH_EINVAL, "decoder belongs to another device");
    OsdArgs a{};
    a.llr = llr;
    a.ld = ld;
    a.F = F;
    a.skip = skip;
    a.bits = bits;
    a.bits_ld = bits_ld;
    a.G = dec->d_gen;
    a.N = dec->N;
    a.K = dec->K;
    a.order = order;
    hipError_t e = launch_osd(a, dec->n_cu, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "device OSD launch");
}

int bch_mixed_osd_decode(const bch_decoder *decs, int n_codes, const uint8_t *code_idx, const float *llr,
                         int64_t ld, int64_t F, int order, const uint8_t *skip, uint64_t *bits, int64_t bits_ld,
                         hipStream_t stream)
{
    if (!decs || n_codes < 1 || n_codes > BCH_MAX_MIX)
        return fail(BCH_EINVAL, "n_codes must be in [1, BCH_MAX_MIX]");
    if (!code_idx)
        return fail(BCH_EINVAL, "NULL code_idx");
    for (int c = 0; c < n_codes; c++) {
        if (!decs[c])
            return fail(BCH_EINVAL, "NULL decoder");
        if (F > 0 && (ld < decs[c]->N || bits_ld < decs[c]->W64))
            return fail(BCH_EINVAL, "ld or bits_ld too small for a code of the mix");
    }
    if (F < 0 || order < 0 || order > 2)
        return fail(BCH_EINVAL, "bad argument (order must be 0, 1 or 2)");
    if (F == 0)
        return BCH_OK;
    if (!llr || !bits)
        return fail(BCH_EINVAL, "NULL buffer");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return fail(BCH_EDEVICE, "hipGetDevice failed");
    for (int c = 0; c < n_codes; c++) {
        const bch_decoder_s *d = decs[c];
        if (d->dev != cur)
            return fail(BCH_EINVAL, "decoder belongs to another device");
        if (d->N > 128 || d->K > 128)
            return fail(BCH_EUNSUPPORTED, "device OSD needs N, K <= 128");
        OsdArgs a{};
        a.llr = llr;
        a.ld = ld;
        a.F = F;
        a.skip = skip;
        a.code_idx = code_idx;
        a.code = c;
        a.bits = bits;
        a.bits_ld = bits_ld;
        a.G = d->d_gen;
        a.N = d->N;
        a.K = d->K;
        a.order = order;
        hipError_t e = launch_osd(a, d->n_cu, stream);
        if (e != hipSuccess)
            return hip_fail(e, "device OSD launch");
    }
    return BCH_OK;
}

int bch_syndrome_check(bch_code code, const uint64_t *bits, int64_t F, uint8_t *ok,
                       hipStream_t stream)
{
    if (!code || (F > 0 && (!bits || !ok)) || F < 0)
        return fail(BCH_EINVAL, "bad argument");
    if (F == 0)
        return BCH_OK;
    uint64_t *hs = nullptr;
    int rc = code_hsyn(code, &hs);
    if (rc)
        return rc;
    hipError_t e = launch_syndrome(bits, F, (code->c.N + 63) / 64, hs, code->c.N - code->c.K,
                                   ok, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "syndrome kernel launch");
}

int bch_quantize_llr(const float *llr, int64_t ld, int64_t F, int N, float scale, int8_t *q,
                     int64_t ldq, hipStream_t stream)
{
    if (F < 0 || N < 1 || ld < N || ldq < N || !(scale > 0.0f))
        return fail(BCH_EINVAL, "bad argument");
    if (F == 0)
        return BCH_OK;
    if (!llr || !q)
        return fail(BCH_EINVAL, "NULL buffer");
    hipError_t e = launch_quantize(llr, ld, F, N, scale, q, ldq, stream);
    return e == hipSuccess ? BCH_OK : hip_fail(e, "quantize kernel launch");
}

int bch_osd_decode(bch_code code, const float *llr, int64_t ld, int64_t F, int order,
                   const uint8_t *skip, uint64_t *bits, int n_threads)
{
    if (!code || F < 0 || order < 0 || order > 2 || ld < code->c.N)
        return fail(BCH_EINVAL, "bad argument (order must be 0, 1 or 2)");
    if (F == 0)
        return BCH_OK;
    if (!llr || !bits)
        return fail(BCH_EINVAL, "NULL buffer");
    const Code &c = code->c;
    const int W64 = (c.N + 63) / 64;
    int T = n_threads > 0 ? n_threads : (int)std::thread::hardware_concurrency();
    T = std::max(1, std::min<int>(T, (int)std::min<int64_t>(F, 256)));
    auto work = [&](int64_t lo, int64_t hi) {
        for (int64_t f = lo; f < hi; f++)
            if (!skip || !skip[f])
                osd_frame(c, llr + f * ld, order, bits + f * W64);
    };
    if (T == 1) {
        work(0, F);
        return BCH_OK;
    }
    std::vector<std::thread> pool;
    for (int k = 0; k < T; k++)
        pool.emplace_back(work, F * k / T, F * (k + 1) / T);
    for (auto &th : pool)
        th.join();
    return BCH_OK;
}

}  // extern "C"
