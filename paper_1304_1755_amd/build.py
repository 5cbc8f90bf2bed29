"""Build libsgbt.so for gfx950 in-tree (hipcc, parallel per source file), and beside it the
LDS-poison debug build libsgbt_poison.so (-DSG_LDS_POISON: kernels with LDS tiles fill their LDS
with NaN before use, so that a read before write shows up as NaN in their output)."""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsgbt.so")
LIB_POISON = os.path.join(HERE, "libsgbt_poison.so")
SOURCES = ["sg_setup.cpp", "sg_apply.hip", "sg_apply_p1.hip", "sg_mg.hip", "sg_vec.hip", "sg_split.hip", "sg_api.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(job):
    src, poison = job
    out_dir = os.path.join(BUILD, "poison") if poison else BUILD
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, *(["-DSG_LDS_POISON"] if poison else []), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose=False, poison=True):
    os.makedirs(os.path.join(BUILD, "poison"), exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + ([(src, True) for src in SOURCES] if poison else [])
    # the longest translation units first, so that they do not finish last
    jobs.sort(key=lambda j: j[0] != "sg_mg.hip")
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(_compile, jobs))
    _link([o for o, j in zip(objs, jobs) if not j[1]], LIB)
    if poison:
        _link([o for o, j in zip(objs, jobs) if j[1]], LIB_POISON)
    if verbose:
        print("built", LIB, *( [LIB_POISON] if poison else []))
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
