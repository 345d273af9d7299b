// Lookup of PCM-specialised kernels.  The table is produced at build time by
// gen_spec.py for the matrices the library is built for.
#include "spec_registry.h"

namespace bch {

// FNV-1a over N, M and the packed rows in order.
uint64_t pcm_fingerprint(const Pcm &p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; k++) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)p.N);
    mix((uint64_t)p.M);
    for (const Row &r : p.rows) {
        mix(r.w[0]);
        mix(r.w[1]);
    }
    return h;
}

#include "spec_table.inc"

const SpecKernel *find_spec_kernel(const Pcm &p, const bch_dec_params &q, int variant)
{
    const uint64_t fp = pcm_fingerprint(p);
    for (const SpecKernel &k : kSpecKernels) {
        if (k.launch == nullptr)
            continue;
        if (k.fingerprint == fp && k.N == p.N && k.M == p.M && k.B == q.n_branches &&
            k.mode == q.mode && k.precision == q.precision && k.variant == variant)
            return &k;
    }
    return nullptr;
}

const MixKernel *find_mix_kernel(const uint64_t *fps, int n, int precision)
{
    for (const MixKernel &k : kMixKernels) {
        if (k.launch == nullptr || k.n != n || k.precision != precision)
            continue;
        bool same = true;
        for (int c = 0; c < n; c++)
            same = same && k.fp[c] == fps[c];
        if (same)
            return &k;
    }
    return nullptr;
}

}  // namespace bch
