"""Build libpagani.so (HIP, gfx950) in-tree with hipcc: one object per
source file, compiled in parallel, then linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", s) for s in
           ("pg_evaluate.hip", "pg_list.hip", "pg_batch.hip", "pg_adjoint.hip",
            "pg_api.hip", "pg_noalloc.hip")]
# the EVALUATE kernels, one object per integrand family (pg_family ids)
FAMILY_SOURCE = os.path.join(HERE, "csrc", "pg_eval_family.hip")
N_FAMILIES = 8
LIB = os.path.join(HERE, "libpagani.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PAGANI_OFFLOAD_ARCH", "gfx950")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off in every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    units = [(s, os.path.join(OBJ_DIR, os.path.basename(s) + ".o"), [])
             for s in SOURCES]
    units += [(FAMILY_SOURCE, os.path.join(OBJ_DIR, f"pg_eval_family{k}.o"),
               [f"-DPG_EVAL_FAMILY={k}"]) for k in range(N_FAMILIES)]

    def compile_one(unit):
        src, obj, extra = unit
        cmd = ["hipcc", *FLAGS, *extra, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = min(len(units), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, units))
    objs = [u[1] for u in units]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
