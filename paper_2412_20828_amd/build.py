"""Build of libbchnms.so for gfx950.

Host C++ (code algebra, H_o construction, OSD, C-ABI) is compiled with g++;
HIP sources with hipcc --offload-arch=gfx950.  The build has two stages: stage
1 links the library without PCM-specialised kernels; gen_spec.py then asks that
library for the matrices it is built for (deterministic constructions), emits
one specialised kernel per matrix and a lookup table, and stage 2 links the
final library with them.

Usage: python -m paper_2412_20828_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbchnms.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SRCS = ["host_code.cpp", "host_pcm.cpp", "host_osd.cpp", "capi.cpp", "spec_registry.cpp"]
HIP_SRCS = ["k_generic.hip", "k_bucket.hip", "k_osd.hip", "noalloc.hip"]

CXXFLAGS = ["-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
            "-D__HIP_PLATFORM_AMD__", "-I" + INCLUDE, "-I" + CSRC, "-I" + os.path.join(ROCM, "include")]
HIPFLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + INCLUDE, "-I" + CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def _obj(src, tag=""):
    base = os.path.basename(src)
    return os.path.join(BUILD, tag + base + ".o")


def _compile_host(src, extra_inc=None):
    out = _obj(src)
    cmd = ["g++"] + CXXFLAGS + (["-I" + extra_inc] if extra_inc else []) + ["-c", src, "-o", out]
    _run(cmd)
    return out


# The mixed-code kernels merge each permutation type into the accumulator in
# one of three branches with fixed register indices; SimplifyCFG would sink
# the three branches into one with dynamically indexed arrays, which then live
# in scratch memory.
MIXFLAGS = ["-mllvm", "-simplifycfg-sink-common=false"]


def _compile_hip(src, extra_inc=None):
    out = _obj(src)
    inc = ["-I" + extra_inc] if extra_inc else []
    extra = MIXFLAGS if os.path.basename(src).startswith("mix_") else []
    _run([os.path.join(ROCM, "bin", "hipcc")] + HIPFLAGS + extra + inc + ["-c", src, "-o", out])
    return out


def _link(objs, out):
    tmp = out + ".tmp%d" % os.getpid()
    _run([os.path.join(ROCM, "bin", "hipcc"), "-shared", "-fPIC", "--offload-arch=" + ARCH,
          "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, out)


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as fh:
        fh.write(text)


def build(verbose: bool = True, with_spec: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    gen_dir = os.path.join(BUILD, "gen")
    os.makedirs(gen_dir, exist_ok=True)
    # stage 1: empty specialisation table
    _write_if_changed(os.path.join(gen_dir, "spec_table.inc"),
                      "static const SpecKernel kSpecKernels[] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr}};\n"
                      "static const MixKernel kMixKernels[] = {{0, {0}, 0, nullptr, nullptr}};\n")
    jobs = [(_compile_host, os.path.join(CSRC, s), gen_dir) for s in HOST_SRCS]
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        futs = [ex.submit(fn, src, inc) for fn, src, inc in jobs]
        futs += [ex.submit(_compile_hip, os.path.join(CSRC, s)) for s in HIP_SRCS]
        objs = [f.result() for f in futs]
    stage1 = os.path.join(BUILD, "libbchnms_stage1.so")
    _link(objs, stage1)
    if not with_spec:
        shutil.copyfile(stage1, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
        return LIB
    # stage 2: PCM-specialised kernels
    from . import gen_spec
    spec_srcs, table = gen_spec.generate(stage1, gen_dir)
    _write_if_changed(os.path.join(gen_dir, "spec_table.inc"), table)
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        futs = [ex.submit(_compile_host, os.path.join(CSRC, "spec_registry.cpp"), gen_dir)]
        futs += [ex.submit(_compile_hip, s, gen_dir) for s in spec_srcs]
        new = [f.result() for f in futs]
    objs = [o for o in objs if not o.endswith("spec_registry.cpp.o")] + new
    _link(objs, LIB)
    if verbose:
        print("built", LIB, "with", len(spec_srcs), "specialised kernel sources")
    return LIB


if __name__ == "__main__":
    build(with_spec="--no-spec" not in sys.argv)
