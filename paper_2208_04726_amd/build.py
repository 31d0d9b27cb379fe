"""Builds the gfx950 HIP library libdpba.so (bundle adjustment, the
correlation features, the soft aggregation and the sliding-window driver) in the package directory."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", f) for f in ("dpba.hip", "dpcorr.hip", "dpagg.hip", "dpvo.hip")]
OUT = os.path.join(HERE, "libdpba.so")
ARCH = os.environ.get("DPBA_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile the HIP sources into libdpba.so (always recompiles)."""
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 instructions (v_pk_*_f32) in device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # multiply-add fusion only inside one source expression, so the
           # arithmetic of a window does not depend on which kernel variant ran
           "-ffp-contract=on",
           "-Wno-unused-command-line-argument",
           *SRCS, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libdpba.so")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
