"""Builds libhgm.so (the HIP library behind include/hgm.h) for gfx950.

The library carries a digest of the sources and flags it was built from
(hgm_source_digest); the binding refuses a library whose digest differs
from the sources beside it, so a stale build is never run."""
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhgm.so")
SOURCES = ["kernels.hip", "api.hip", "server.cpp", "tune.cpp"]
PROBE_SOURCE = "probe.hip"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-pthread",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def source_digest() -> str:
    """SHA-256 (first 16 hex digits) over the library's sources, the headers
    they include and the compiler flags."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".cpp", ".h")) and f != PROBE_SOURCE)
    for fn in files:
        h.update(fn.encode())
        with open(os.path.join(CSRC, fn), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "include", "hgm.h"), "rb") as f:
        h.update(f.read())
    h.update(" ".join(FLAGS + SOURCES).encode())
    return h.hexdigest()[:16]


def command(out: str):
    return [hipcc()] + FLAGS + [f'-DHGM_SOURCE_DIGEST="{source_digest()}"',
                                "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out] + \
           [os.path.join(CSRC, s) for s in SOURCES]


# Memory-system probes (bench.py --ceilings): their own library, not linked
# into libhgm.so.
PROBE_LIB = os.path.join(HERE, "libhgm_probe.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(command(tmp))
        os.replace(tmp, LIB)
    if force or not os.path.exists(PROBE_LIB):
        tmp = PROBE_LIB + ".tmp"
        subprocess.check_call([hipcc()] + FLAGS + ["-o", tmp, os.path.join(CSRC, PROBE_SOURCE)])
        os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build())
