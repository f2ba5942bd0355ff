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


def build(verbose=False, arch="gfx950"):
    """Compile csrc/bamg_all.hip into libbamg.so (always recompiles)."""
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-munsafe-fp-atomics", "-Wno-unused-result",
           "-I", INCLUDE, "-I", CSRC,
           os.path.join(CSRC, "bamg_all.hip"), "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libbamg.so")
    if verbose:
        # host-pass warnings about the packed-fp32 feature are expected
        noise = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
        if noise:
            sys.stderr.write("\n".join(noise) + "\n")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
