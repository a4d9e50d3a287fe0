"""Builds libmispectral.so (HIP, gfx950) in the package directory.

    python -m paper_1810_02719_amd.build [--jobs N]

Every translation unit under csrc/ is compiled with hipcc for gfx950 and
linked into one shared library exporting the C ABI of include/mispectral.h.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmispectral.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed FP32 instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources")
    return OUT


# Host-side sanitizer build: every translation unit and the driver under
# tests/native compiled with AddressSanitizer and UndefinedBehaviorSanitizer
# on the host pass only (each flag behind -Xarch_host; the kernels are the
# ordinary gfx950 code), linked into one executable by the LLVM C++ driver.
SAN_DRIVER = os.path.join(os.path.dirname(HERE), "tests", "native", "sanitized_driver.hip")
SAN_OUT = os.path.join(HERE, "mispectral_sanitized")
SAN_BUILD = os.path.join(BUILD, "sanitized")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
CXX_LINK = os.environ.get("MI_CXX_LINK", "/opt/rocm/llvm/bin/clang++")
LINK_SAN = ["-fsanitize=address,undefined"]


def _compile_san(src):
    obj = os.path.join(SAN_BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, *SAN_HOST, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"sanitized build failed for {src}:\n{err}")
    return obj


def build_sanitized(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(SAN_BUILD, exist_ok=True)
    srcs = sources() + [SAN_DRIVER]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile_san, srcs))
    rocm = os.path.dirname(os.path.dirname(HIPCC))
    tmp = SAN_OUT + ".tmp"
    cmd = [CXX_LINK, *LINK_SAN, "-o", tmp, *objs, f"-L{rocm}/lib", "-lamdhip64",
           f"-Wl,-rpath,{rocm}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stderr)
    os.replace(tmp, SAN_OUT)
    if verbose:
        print(f"built {SAN_OUT} (host ASan/UBSan) from {len(srcs)} sources")
    return SAN_OUT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--sanitized", action="store_true",
                    help="also build the host-sanitized test executable")
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True)
    if a.sanitized:
        build_sanitized(a.jobs, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
