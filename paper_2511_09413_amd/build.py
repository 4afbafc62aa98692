"""Build the HIP library libkmc.so for gfx950 in-tree (paper_2511_09413_amd/_build).

hipcc cross-compiles without a GPU.  Flags:
  -ffp-contract=off      no FMA contraction, so the binary32/binary64 energy and
                         probability expressions round exactly as written;
  -target-feature -packed-fp32-ops
                         no packed FP32 instructions.
"""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libkmc.so")
SOURCES = ["kmc_kernels.hip", "kmc_persistent.hip", "kmc_wave.hip", "kmc_dense.hip", "kmc_api.cpp", "kmc_fit.cpp", "kmc_noalloc.hip", "kmc_zone.hip", "kmc_phifix.hip", "kmc_electrode.hip", "kmc_replay.hip"]
ARCH = os.environ.get("KMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.exists(cand) or cand == "hipcc"):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-command-line-argument"]


def source_hash() -> str:
    """SHA-1 over the build flags and every source and header the library is
    built from (csrc/ and include/), in sorted order.  build() embeds it; the
    loader compares it with the library's kmc_build_hash()."""
    h = hashlib.sha1(" ".join(FLAGS).encode())
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".cpp", ".h")):
                h.update(f.encode())
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-DKMC_SOURCE_HASH=\"%s\"" % source_hash()]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
