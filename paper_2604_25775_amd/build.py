"""Build the scalevmc C-ABI library (libscalevmc.so) in-tree for gfx950.

    python -m paper_2604_25775_amd.build [--jobs N] [--debug]

Every translation unit under csrc/ is compiled by hipcc into an object in
_build/, then linked into paper_2604_25775_amd/libscalevmc.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libscalevmc.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = os.environ.get("SVMC_ARCH", "gfx950")

# Packed-FP32 ops are switched off for all device code (stability of those
# instructions on this hardware); hipcc's host pass warns that it does not
# know the feature, which is harmless.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# (precision, channels) instances of the templated conv kernels; must match
# SVMC_FOR_EACH_PREC_C in csrc/svmc_launch.h.
INSTANCES = [(p, c) for p in ("PREC_F64", "PREC_F32", "PREC_BF16", "PREC_BF16X3", "PREC_F16X2") for c in (8, 16, 24, 32)]


def units():
    """(source, defines, object name): files that contain per-instance code
    are compiled once as a base unit and once per instance."""
    out = []
    for f in sorted(os.listdir(CSRC)):
        if not (f.endswith(".hip") or f.endswith(".cpp")):
            continue
        src = os.path.join(CSRC, f)
        out.append((src, [], f + ".o"))
        with open(src) as fh:
            if "SVMC_INST_P" in fh.read():
                for p, c in INSTANCES:
                    out.append((src, [f"-DSVMC_INST_P={p}", f"-DSVMC_INST_C={c}"], f"{f}.{p}_{c}.o"))
    return out


def compile_one(unit, debug: bool) -> str:
    src, defs, name = unit
    obj = os.path.join(BUILD, name)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-c", src, "-o", obj,
           "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"] + defs
    cmd += ["-O1", "-g"] if debug else ["-O3"]
    if src.endswith(".hip"):
        cmd += DEVICE_FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, debug: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    us = units()
    jobs = jobs or max(1, min(16, os.cpu_count() or 4))
    # longest units first
    us.sort(key=lambda u: (0 if u[1] else 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: compile_one(u, debug), us))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    return OUT


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.debug)


if __name__ == "__main__":
    main()
