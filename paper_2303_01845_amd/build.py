"""Compile the HIP library (gfx950) in-tree: paper_2303_01845_amd/libsw_hip.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsw_hip.so")
SOURCES = [os.path.join(CSRC, "sw_device.hip"), os.path.join(CSRC, "sw_kmer.hip"), os.path.join(CSRC, "sw_identity.hip"),
           os.path.join(CSRC, "sw_api.cpp"), os.path.join(CSRC, "sw_server.cpp")]
HEADERS = [os.path.join(CSRC, "sw_internal.h"), os.path.join(CSRC, "kmer_internal.h"),
           os.path.join(CSRC, "identity_internal.h"),
           os.path.join(os.path.dirname(HERE), "include", "sw.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-fvisibility=hidden", "-fvisibility-inlines-hidden",
    # packed FP32 instructions stay off in every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + FLAGS + ["-o", tmp] + SOURCES
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops' is not a recognized" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
