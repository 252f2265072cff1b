"""Build ``librlbm.so`` (the HIP/gfx950 RLBM library) in-tree with hipcc.

    python -m paper_2101_06187_amd.build [--jobs N] [--verbose]

Compiles every translation unit under ``csrc/`` for gfx950 (one step-kernel
object per population storage form) and links the shared library next to
this file.  Always rebuilds.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librlbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # keep the compiler away from packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
]

STORAGE_FORMS = {0: "f64", 1: "f32", 2: "f16s", 3: "bf16s"}


def _units():
    units = []
    for sid, name in STORAGE_FORMS.items():
        units.append((os.path.join(CSRC, "kernels_step.hip"),
                      os.path.join(BUILD, f"kernels_step_{name}.o"),
                      [f"-DRLBM_STORAGE_ID={sid}"]))
    units.append((os.path.join(CSRC, "kernels_aux.hip"), os.path.join(BUILD, "kernels_aux.o"), []))
    units.append((os.path.join(CSRC, "api.hip"), os.path.join(BUILD, "api.o"), []))
    return units


def _compile(unit, verbose):
    src, obj, extra = unit
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    t = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)} {extra}:\n{p.stderr}")
    return obj, time.time() - t, p.stderr


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, (os.cpu_count() or 4)))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, err in ex.map(lambda u: _compile(u, verbose), units):
            objs.append(obj)
            if verbose:
                print(f"  {os.path.basename(obj)}: {dt:.1f} s", flush=True)
            if err.strip() and verbose:
                print(err, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    t = time.time()
    lib = build(a.jobs, a.verbose)
    print(f"built {lib} in {time.time() - t:.1f} s")


if __name__ == "__main__":
    sys.exit(main())
