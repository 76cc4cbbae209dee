"""Build libperiodic_sum.so (HIP for gfx950 + host C++) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib", "libperiodic_sum.so")
SOURCES = ["ps_setup.cpp", "ps_kernels.hip", "ps_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PS_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled on purpose; host code is built without
# FMA contraction so that its FP64 set phase is reproducible.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fopenmp"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False, jobs=3):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(os.path.dirname(OUT), src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, *COMMON, "-x", "c++", "-c", path, "-o", obj]
        objs.append(obj)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    for cmd, p in procs:
        out, _ = p.communicate()
        lines = [l for l in out.splitlines() if "is not a recognized feature for this target" not in l]
        if p.returncode != 0:
            sys.stderr.write("\n".join(lines) + "\n")
            raise RuntimeError("compilation failed: " + " ".join(cmd))
        if verbose and lines:
            print("\n".join(lines))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
