"""Compile the HIP library ``libyee.so`` in-tree for gfx950 with hipcc."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libyee.so")
RAYMETA_LIB = os.path.join(HERE, "libraymeta.so")

# library -> its HIP sources (each library is one translation unit)
LIBRARIES = {
    LIB: ["yee_runtime.hip"],
    RAYMETA_LIB: ["raymeta.hip"],
}
# per-library flags: the Yee kernels write every fused multiply-add explicitly,
# so that one sample's update is the same instruction sequence in every kernel
LIBRARY_FLAGS = {
    LIB: ["-ffp-contract=off"],
    RAYMETA_LIB: [],
}

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_one(lib: str, sources, verbose: bool = False, extra_flags=()) -> str:
    out_tmp = lib + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *LIBRARY_FLAGS.get(lib, []), *extra_flags, "-I", os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in sources], "-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and r.stderr.strip():
        print(r.stderr)
    os.replace(out_tmp, lib)
    return lib


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every library (always recompiles); returns the Yee library's path."""
    for lib, sources in LIBRARIES.items():
        build_one(lib, sources, verbose, extra_flags)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
