"""Build the bamg HIP library for gfx950 in-tree (hipcc, one translation unit)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbamg.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


def hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


CHECK = os.path.join(HERE, "plan_check_sanitized")
COMMON = ["-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {what}")
    if verbose:
        # host-pass warnings about the packed-fp32 feature are expected
        noise = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
        if noise:
            sys.stderr.write("\n".join(noise) + "\n")


def build(verbose=False, arch="gfx950"):
    """Compile csrc/bamg_all.hip into libbamg.so (always recompiles)."""
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-fPIC", "-shared", *COMMON,
           os.path.join(CSRC, "bamg_all.hip"), "-o", LIB + ".tmp"]
    _run(cmd, "libbamg.so", verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_check(verbose=False, arch="gfx950"):
    """Compile the host-side checker (csrc/check/plan_check.cpp) with the whole
    library into one executable whose host code carries AddressSanitizer and
    UndefinedBehaviorSanitizer; the GPU code is built as usual."""
    cmd = [hipcc(), f"--offload-arch={arch}", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *COMMON,
           os.path.join(CSRC, "bamg_all.hip"), os.path.join(CSRC, "check", "plan_check.cpp"),
           "-o", CHECK + ".tmp"]
    _run(cmd, "plan_check_sanitized", verbose)
    os.replace(CHECK + ".tmp", CHECK)
    return CHECK


if __name__ == "__main__":
    print(build(verbose=True))
    if "--check" in sys.argv:
        print(build_check(verbose=True))
