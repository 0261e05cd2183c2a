"""Compile the HIP sources of the package into libfmoxtb.so (gfx950)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmoxtb.so")
SOURCES = ["fx_api.cpp", "fx_grad.cpp", "fx_integrals.hip", "fx_scc.hip", "fx_fmo.hip", "fx_gradk.hip",
           "fx_resp.hip", "fx_mlp.hip", "fx_noalloc.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


LIB_UBSAN = os.path.join(HERE, "libfmoxtb_ubsan.so")


def _sanitizer_runtime_dir():
    """Directory of the compiler's shared undefined-behaviour sanitizer
    runtime (the library's DT_NEEDED entry is found there through the rpath)."""
    name = "libclang_rt.ubsan_standalone-x86_64.so"
    r = subprocess.run(["hipcc", "-print-file-name=" + name], capture_output=True, text=True)
    f = r.stdout.strip()
    if r.returncode != 0 or not os.path.isfile(f):
        raise RuntimeError("the compiler has no " + name)
    return os.path.dirname(os.path.realpath(f))


def build(verbose=False, ubsan=False):
    """ubsan: the host code (not the device code) instrumented with the
    undefined-behaviour sanitizer, linked against the shared runtime, as
    libfmoxtb_ubsan.so (loaded when FX_LIBRARY=ubsan)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    out = LIB_UBSAN if ubsan else LIB
    tmp = out + ".tmp"
    flags = list(FLAGS)
    if ubsan:
        rt = _sanitizer_runtime_dir()
        flags += ["-O1", "-g", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-shared-libsan", "-Wl,-rpath," + rt]
    cmd = ["hipcc"] + flags + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, ubsan="--ubsan" in sys.argv[1:]))
