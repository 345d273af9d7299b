// Registry of kernels specialised to one parity-check matrix: the matrix is
// compiled into the kernel so that every coordinate of a frame lives in a
// register with a static index.  A decoder uses such a kernel when the
// fingerprint of its matrix and its parameters match an entry.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "internal.h"
#include "mix_launch.h"
#include "spec_launch.h"

namespace bch {

struct SpecKernel {
    uint64_t fingerprint;  // of the matrix rows, see pcm_fingerprint()
    int N, M, B, mode, precision;
    int variant;       // 0; 1: packed 16-bit fixed point; 2: three waves per 64 frames, N = 127 (small batches)
    int waves_per_cu;  // persistent grid = CUs x waves_per_cu wavefronts
    int y_global;      // 1: y lives in device scratch [grid][N][64] floats
    int frames_per_wave;  // frames per workgroup: 64, or 128 for the packed 16-bit kernels
    int wave_group;       // waves per workgroup: 1, or 3 when the branch types share 64 frames
    const char *name;
    hipError_t (*launch)(const SpecLaunch &, int n_cu, int waves_per_cu, hipStream_t);
};

// A kernel over frames of several codes (the matrices compiled in, in this
// order: code k of a mixed call is fingerprint fp[k]), nine branches, restart
// mode.
struct MixKernel {
    int n;                    // codes
    uint64_t fp[MIX_MAXC];    // matrix fingerprints, in code order
    int precision;
    const char *name;
    hipError_t (*launch)(const MixLaunch &, int n_cu, int waves_per_cu, hipStream_t);
};

uint64_t pcm_fingerprint(const Pcm &p);
const SpecKernel *find_spec_kernel(const Pcm &p, const bch_dec_params &q, int variant);
const MixKernel *find_mix_kernel(const uint64_t *fps, int n, int precision);

}  // namespace bch
