"""Generator of PCM-specialised decode kernels (stage 2 of the build).

For every matrix the library is built for, the stage-1 library constructs the
matrix (the construction is deterministic), and a HIP kernel is emitted with
the matrix compiled in.  Returns the generated sources and the lookup table.
"""
from __future__ import annotations

# (code name, target rows of H_o or 0 for the standard matrix, n_branches, mode)
SPECS: list = []


def generate(stage1_lib: str, out_dir: str):
    table = "static const SpecKernel kSpecKernels[] = {{0, 0, 0, 0, 0, 0, nullptr, nullptr}};\n"
    return [], table
