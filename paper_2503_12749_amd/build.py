"""Builds libmpgbs.so (the HIP/C++ library behind include/mpgbs.h) in-tree
for gfx950 with hipcc.  Run: python -m paper_2503_12749_amd.build
(--host-check: the sanitized host self-check executable instead)."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpgbs.so")
SOURCES = ["api.cpp", "sample.hip", "propagate.hip", "counts.hip", "jointd.hip", "pairs.hip", "plan.hip",
           "mlp.hip", "diag.hip"]
ARCH = os.environ.get("MPGBS_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compiles every source and links the shared library; returns its path."""
    with tempfile.TemporaryDirectory(prefix="mpgbs_build_") as tmp:
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            # hipcc's host pass does not know the packed-fp32 feature: harmless
            lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
            if lines and (verbose or p.returncode):
                print("\n".join(lines), file=sys.stderr)
            if p.returncode:
                failed.append(src)
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        tmp_lib = LIB + ".tmp"
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib]
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


# Host-side self-check (csrc/host_check.cpp) with AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only; the device code is built
# as for the library.
HOST_CHECK = os.path.join(os.path.dirname(HERE), "_build", "host_check")
SANITIZE_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def build_host_check(verbose: bool = False) -> str:
    """Builds the sanitized host check executable (skipped while it is newer
    than every source and header); returns its path."""
    srcs = [os.path.join(CSRC, f) for f in SOURCES + ["host_check.cpp"]]
    deps = srcs + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "mpgbs.h"))
    if os.path.exists(HOST_CHECK) and all(os.path.getmtime(HOST_CHECK) > os.path.getmtime(d)
                                          for d in deps):
        return HOST_CHECK
    os.makedirs(os.path.dirname(HOST_CHECK), exist_ok=True)
    flags = ["-O2", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-Xarch_host", "-g", "-Xarch_host",
             "-fno-omit-frame-pointer", *SANITIZE_HOST]
    with tempfile.TemporaryDirectory(prefix="mpgbs_hostcheck_") as tmp:
        objs, procs = [], []
        for src in srcs:
            obj = os.path.join(tmp, os.path.splitext(os.path.basename(src))[0] + ".o")
            cmd = [HIPCC, *flags, "-x", "hip", "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode:
                print(out.decode(errors="replace"), file=sys.stderr)
                failed.append(src)
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        subprocess.run([HIPCC, f"--offload-arch={ARCH}", *SANITIZE_HOST, *objs, "-o",
                        HOST_CHECK + ".tmp"], check=True)
        os.replace(HOST_CHECK + ".tmp", HOST_CHECK)
    return HOST_CHECK


if __name__ == "__main__":
    if "--host-check" in sys.argv:
        print(build_host_check(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
