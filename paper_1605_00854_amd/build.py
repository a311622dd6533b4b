"""Compile the HIP/C++ sources of the library into an in-tree shared object.

Every source is compiled for gfx950 with hipcc; host-only files are plain
C++17.  The result is paper_1605_00854_amd/libpbn_amd.so, loaded by the
ctypes binding.
"""
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpbn_amd.so")
ARCH = "gfx950"

HOST_SOURCES = ["host_net.cpp", "host_plan.cpp", "host_stats.cpp"]
DEVICE_SOURCES = ["device.hip", "probe.hip"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
# host-only sources: plain C++ (hipcc would otherwise also compile them for a
# default device target)
HOST_FLAGS = ["-x", "c++"]
# never emit packed FP32 instructions (none are needed: the path is integer only)
DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-munsafe-fp-atomics"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=4):
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="pbn_build_")
    try:
        procs, objs = [], []
        for src in HOST_SOURCES + DEVICE_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc] + COMMON + (DEVICE_FLAGS if src.endswith(".hip") else HOST_FLAGS) + \
                  ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        errors = []
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                errors.append(f"--- {src} ---\n{out}")
            elif verbose and out.strip():
                print(out)
        if errors:
            raise RuntimeError("compilation failed:\n" + "\n".join(errors))
        out_tmp = os.path.join(tmp, "libpbn_amd.so")
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", out_tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
        shutil.move(out_tmp, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
