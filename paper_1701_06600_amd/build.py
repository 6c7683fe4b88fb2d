"""Compile the gfx950 library libcprand.so in place with hipcc.

Every call recompiles (sources are few); objects go to _build/ next to this
file and the shared library to paper_1701_06600_amd/libcprand.so.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcprand.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["sample.hip", "mttkrp.hip", "mttkrp_stream.hip", "mttkrp_bf16.hip", "mttkrp_full.hip", "solve.hip", "step.hip", "fit.hip", "fitset.hip", "fft.hip", "dct.hip",
           "layout.hip", "proposal.hip", "noalloc.hip", "api.cpp", "api_proposal.cpp", "cpals.cpp", "als.cpp"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # no packed-FP32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _compile(src, incremental=False):
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(out):
        deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
        deps.append(os.path.join(os.path.dirname(HERE), "include", "cprand.h"))
        if max(os.path.getmtime(d) for d in deps) < os.path.getmtime(out):
            return out
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return out


def build(verbose=False, jobs=None, incremental=False):
    """incremental=True skips sources whose object is newer than the source,
    every header and include/cprand.h (a developer shortcut; the default
    recompiles everything)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Wl,-z,defs", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
