"""Build the HIP library (libmcpd.so) in-tree for gfx950 with hipcc.

The sampler is compiled once per clone-row format (each instantiation is a
large kernel) and once for its dispatcher, in parallel with the kernels of
the learned weights and the host side of the C ABI, then linked.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmcpd.so")
N_FORMATS = 7

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # only the C ABI is exported
    "-fvisibility=hidden",
    # no FMA contraction anywhere: the host tables must match the FP64
    # reading bit for bit
    "-ffp-contract=off",
    # keep hipcc from emitting packed FP32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def jobs():
    """(source, extra flags, object name) of every compile step."""
    out = [("mcpd_host.cpp", [], "host.o"), ("mcpd_sampler.hip", [], "sampler.o"),
           ("mcpd_mlp.hip", [], "mlp.o"), ("mcpd_mlp_host.cpp", [], "mlp_host.o"),
           ("mcpd_finish.hip", [], "finish.o"), ("mcpd_probe.hip", [], "probe.o"),
           ("mcpd_noalloc.hip", [], "noalloc.o")]
    out += [("mcpd_sampler.hip", [f"-DMCPD_FMT={f}"], f"sampler_f{f}.o") for f in range(N_FORMATS)]
    return out


def build(verbose: bool = False) -> str:
    """Compile every source into libmcpd.so (always rebuilds)."""
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="mcpd_build_") as tmpd:
        procs = []
        objs = []
        for src, extra, obj in jobs():
            o = os.path.join(tmpd, obj)
            cmd = [hipcc(), *HIPCC_FLAGS, *inc, *extra, "-c", os.path.join(CSRC, src), "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(o)
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
