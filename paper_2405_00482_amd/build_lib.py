"""Build the HIP library libpvfl.so in-tree for gfx950 with hipcc.

Every HIP source is compiled with -ffp-contract=off (the exact binary64
modular arithmetic relies on uncontracted products) and with packed FP32
instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpvfl.so")
PROBE_OUT = os.path.join(HERE, "libpvfl_probe.so")
SOURCES = ["he_kernels.hip", "encode_kernels.hip", "batch.hip", "mlp.hip", "capi.cpp", "plan.cpp", "codec.cpp",
           "batch.cpp", "mlp_capi.cpp", "planner.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
         "-Werror=return-type", "-Werror=uninitialized"]


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(build_dir, src + ".o")
        objs.append(obj)
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = ["hipcc"] + FLAGS + lang + ["-c", path, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        if pr.returncode != 0:
            sys.stderr.write(text)
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if verbose:
            sys.stderr.write(text)
    tmp = OUT + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    # the arithmetic-throughput probe (measurement only, its own library)
    tmp = PROBE_OUT + ".tmp"
    subprocess.check_call(["hipcc"] + FLAGS + ["-shared", os.path.join(CSRC, "alu_probe.hip"), "-o", tmp])
    os.replace(tmp, PROBE_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
