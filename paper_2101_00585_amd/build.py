"""Build the HIP library ``libupslam.so`` for gfx950 with hipcc.

Each ``csrc/*.hip`` file is compiled to an object in parallel and the objects
are linked into one shared library next to this file.  Packed FP32 vector
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libupslam.so")
ARCH = os.environ.get("UPS_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I",
         os.path.join(HERE, "csrc")]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Host code only, instrumented with AddressSanitizer and UBSan (device code
# is built as usual); the sanitizers' runtime is preloaded into the process
# that loads the library (tests/run_cpu_sanitized.sh).
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
                 "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
SO_SANITIZED = os.path.join(HERE, "libupslam_san.so")
# The same library with phase timestamps in the single-registration launches
# (paper_2101_00585_amd.phase_split reads them); for profiling only.
SO_PHASES = os.path.join(HERE, "libupslam_phases.so")


def build(verbose: bool = False, sanitize: bool = False, phases: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build_phases" if phases else "_build")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    flags = FLAGS + (HOST_SANITIZE if sanitize else []) + (["-DUPS_PHASE_TIMESTAMPS"] if phases else [])

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *flags, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if verbose and out.strip():
            print(out)
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    so = SO_SANITIZED if sanitize else SO_PHASES if phases else SO
    tmp = so + ".tmp%d" % os.getpid()
    if sanitize:
        # the objects already hold their device code: a host link against the HIP runtime
        cmd = ["/opt/rocm/llvm/bin/clang++", "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan",
               "-o", tmp, *objs, "-L/opt/rocm/lib", "-lamdhip64"]
    else:
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, so)
    return so


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv, phases="--phases" in sys.argv))
