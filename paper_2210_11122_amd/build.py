"""Build libme.so for gfx950: generate the process sources, compile every HIP source with
hipcc, link the shared library next to this file."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(CSRC, "generated")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libme.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions (v_pk_{add,mul,fma}_f32) are switched off for all device code
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

SUPPORTED = ["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg", "ee_mumu_z"]


def generate(names=None):
    sys.path.insert(0, ROOT)
    from paper_2210_11122_amd.gen import emit
    return emit.generate(GEN, names or SUPPORTED)


def _compile(src, obj, log):
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    if log:
        print("compiled", os.path.basename(src), flush=True)
    return obj


def build(verbose=True, jobs=None, names=None):
    os.makedirs(BUILD, exist_ok=True)
    generate(names)
    srcs = [os.path.join(CSRC, "me_abi.cpp")]
    srcs += [os.path.join(GEN, f"proc_{n}.hip") for n in SUPPORTED]
    # segment kernels of the large processes live in files of their own
    srcs += sorted(os.path.join(GEN, f) for f in os.listdir(GEN)
                   if f.endswith(".hip") and "_amp_seg" in f and f.split("_amp_seg")[0][5:] in SUPPORTED)
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    # the biggest sources first
    order = sorted(range(len(srcs)), key=lambda i: -os.path.getsize(srcs[i]))
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, srcs[i], objs[i], verbose) for i in order]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("linked", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build()
