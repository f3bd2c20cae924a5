"""Build librad.so (HIP for gfx950) in-tree with hipcc.

Every device file is compiled with packed-FP32 instruction selection switched off
(`-Xclang -target-feature -Xclang -packed-fp32-ops`)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librad.so")
SOURCES = ["rad_accumulate.hip", "rad_kernels.hip", "rad_runtime.hip", "rad_server.hip"]
# the files that define the accumulate kernels (profiles taken on them are keyed to their hash)
ACCUMULATE_FILES = ["rad_internal.h", "rad_device.h", "rad_accumulate.hip"]
ARCH = os.environ.get("RAD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


# the files that define the auxiliary kernels (fold, read-out, tracked particles)
AUX_FILES = ["rad_internal.h", "rad_device.h", "rad_kernels.hip"]


def source_sha256(files) -> str:
    """sha256 over the given csrc files, in order."""
    import hashlib
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def accumulate_source_sha256() -> str:
    """sha256 over the accumulate kernels' source files, in ACCUMULATE_FILES order."""
    return source_sha256(ACCUMULATE_FILES)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False, extra_flags=()) -> str:
    """extra_flags: more hipcc flags, e.g. -DRAD_CHUNK=16 or -DRAD_W16_WAVES=4."""
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc(), *HIPCC_FLAGS, *extra_flags, "-I", INCLUDE, "-I", CSRC, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # one compiler process per source file, at most four at a time
    from concurrent.futures import ThreadPoolExecutor
    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_c_demo(verbose)
    return LIB


def ensure_built(verbose: bool = False) -> str:
    """The in-tree library (and the C-ABI test harness) as it is, built first only if it is
    not there (after a source change, call build())."""
    if not os.path.exists(LIB) or not os.path.exists(C_DEMO):
        build(verbose)
    return LIB


C_DEMO_SRC = os.path.join(ROOT, "tests", "c_abi", "rad_c_demo.c")
C_DEMO = os.path.join(ROOT, "tests", "c_abi", "rad_c_demo")


def build_c_demo(verbose: bool = False) -> str:
    """The C-ABI test harness: plain C against include/rad.h, the HIP runtime and librad.so."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = C_DEMO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
           "-I", os.path.join(rocm, "include"), C_DEMO_SRC, "-o", tmp, "-L", PKG, "-lrad",
           f"-Wl,-rpath,{PKG}", "-Wl,-rpath,$ORIGIN/../../paper_1802_03972_amd",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, C_DEMO)
    return C_DEMO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, extra_flags=[a for a in sys.argv[1:] if a.startswith("-D")]))
