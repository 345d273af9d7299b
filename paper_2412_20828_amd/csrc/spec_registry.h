// Registry of kernels specialised to one parity-check matrix: the matrix is
// compiled into the kernel so that every coordinate of a frame lives in a
// register with a static index.  A decoder uses such a kernel when the
// fingerprint of its matrix and its parameters match an entry.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "internal.h"

namespace bch {

struct SpecArgs {
    const void *llr;
    int64_t ld;
    int64_t F;
    const uint8_t *d_o;
    uint64_t *bits;
    uint8_t *iters;
    uint8_t *flags;
    void *trace;
    int max_iter;
    float alpha;
    const uint64_t *hsyn;
};

struct SpecKernel {
    uint64_t fingerprint;  // of the matrix rows, see pcm_fingerprint()
    int N, M, B, mode, precision;
    const char *name;
    hipError_t (*launch)(const SpecArgs &, hipStream_t);
};

uint64_t pcm_fingerprint(const Pcm &p);
const SpecKernel *find_spec_kernel(const Pcm &p, const bch_dec_params &q);

}  // namespace bch
