"""Build libctm.so (HIP, gfx950) in place: ``python -m paper_2512_14414_amd.build``."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/kernels.hip", "csrc/qr_kernels.hip", "csrc/opt_kernels.hip", "csrc/sur_noalloc.hip", "csrc/engine.cpp",
           "csrc/ctm.cpp", "csrc/surrogate.cpp", "csrc/lbfgs.cpp"]
OUT = os.path.join(HERE, "libctm.so")
C_CHECK = os.path.join(HERE, "c_abi_check")


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # MFMA accumulators in ordinary VGPRs: the FP64 product kernel then needs
           # 212 registers instead of 200 + 128 accumulation registers (two waves per
           # SIMD instead of one) and no longer copies its accumulators out and back
           # in every K step; the arithmetic does not depend on the register file
           "-mllvm", "-amdgpu-mfma-vgpr-form",
           "-I", os.path.join(ROOT, "include"),
           *[os.path.join(HERE, s) for s in SOURCES],
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib",
           "-Wl,--no-undefined", "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs)
    os.replace(OUT + ".tmp", OUT)
    # a plain C program on the C ABI (no Python), run by the GPU tests
    cc = os.environ.get("CC", "gcc")
    cmd = [cc, "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(HERE, "csrc", "c_abi_check.c"), "-L", HERE, "-lctm",
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib", "-lm",
           "-o", C_CHECK]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building the C ABI check failed:\n" + r.stdout + r.stderr)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
