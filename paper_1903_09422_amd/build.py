"""Builds libkadabra.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkadabra.so")
SOURCES = [os.path.join(CSRC, "kadabra_kernels.hip"), os.path.join(CSRC, "kadabra_prep.hip"),
           os.path.join(CSRC, "kadabra_balance.hip"),
           os.path.join(CSRC, "kadabra_host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # loadable by the ROCm 7.0 runtime bundled with PyTorch as well as by /opt/rocm
    "-mcode-object-version=5",
    # the stop check must round exactly like the host expression: no contraction
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (the device code is
# built as usual): every sanitizer flag applies to the host pass only.
SAN_LIB = os.path.join(ROOT, "_build", "libkadabra_san.so")
SAN_FLAGS = ["-O1", "-g"] + [x for f in ("-fsanitize=address", "-fsanitize=undefined",
                                         "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer")
                             for x in ("-Xarch_host", f)]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source into libkadabra.so (always recompiles).  With
    sanitize, a host-sanitized copy goes to _build/libkadabra_san.so instead
    (load it with KADABRA_LIB and the clang ASan runtime preloaded)."""
    out = SAN_LIB if sanitize else LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    flags = [f for f in FLAGS if f != "-O3"] + SAN_FLAGS if sanitize else FLAGS
    cmd = [HIPCC, *flags, "-x", "hip", *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr}")
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
