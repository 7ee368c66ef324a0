"""Build libnufft_mi355x.so in-tree with hipcc for gfx950.

    python -m paper_1710_03197_amd.build [-v] [-i]   (-i: only stale objects)
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnufft_mi355x.so")
SOURCES = ["kernels.hip", "kb_host.cpp", "api.cpp"]
ARCH = os.environ.get("NUFFT_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=fast",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: the AGPR form made the compiler
    # copy loop-carried accumulators around every matrix instruction
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def hip_runtime_dir() -> str:
    """Directory of the HIP runtime the process will already hold: torch ships
    its own libamdhip64.so (without a SONAME), so the library links against
    that file rather than /opt/rocm's, keeping one HIP runtime per process."""
    override = os.environ.get("NUFFT_HIP_RUNTIME_DIR")
    if override:
        return override
    try:
        import torch
        d = os.path.join(os.path.dirname(torch.__file__), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    except ImportError:
        pass
    return "/opt/rocm/lib"


def _stale(obj: str, src: str) -> bool:
    """True when obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src, os.path.join(CSRC, "nufft_internal.h"), os.path.join(ROOT, "include", "nufft_mi355x.h")]
    return any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def build(verbose: bool = False, jobs: int = 3, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those whose object is
    older than the source or a header) and link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, os.path.join(CSRC, src)):
            continue
        cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    for src, p in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src}")
    tmp = LIB + ".tmp"
    rt = hip_runtime_dir()
    rtlib = "libamdhip64.so" if os.path.exists(os.path.join(rt, "libamdhip64.so")) else "libamdhip64.so.7"
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    cmd = [clang, "-shared", "-fPIC", *objs, f"-L{rt}", f"-l:{rtlib}", f"-Wl,-rpath,{rt}",
           "-Wl,--no-undefined", "-lstdc++", "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
