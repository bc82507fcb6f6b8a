"""Builds libtnmi.so (plan + runtime + HIP kernels for gfx950) in this directory."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtnmi.so")
SOURCES = ["plan.cpp", "tn_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         # no packed-FP32 VALU instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose=False):
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", OUT + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtnmi.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


# Host-sanitizer build of the same sources (AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only; device code is built as
# usual).  Loaded through TNMI_LIB_PATH with the sanitizer runtime preloaded,
# it runs the plan tests on the CPU.
SAN_OUT = os.path.join(os.path.dirname(HERE), "_build", "libtnmi_hostsan.so")
SAN_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def sanitizer_runtime():
    """Path of clang's AddressSanitizer runtime (it also holds the
    UndefinedBehaviorSanitizer handlers)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return cands[-1]


def build_host_sanitized():
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    if os.path.exists(SAN_OUT) and \
            os.path.getmtime(SAN_OUT) >= max(os.path.getmtime(f) for f in deps):
        return SAN_OUT
    os.makedirs(os.path.dirname(SAN_OUT), exist_ok=True)
    r = subprocess.run([HIPCC] + SAN_FLAGS + srcs + ["-o", SAN_OUT + ".tmp"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the host-sanitizer library")
    os.replace(SAN_OUT + ".tmp", SAN_OUT)
    return SAN_OUT


if __name__ == "__main__":
    print(build(verbose=True))
