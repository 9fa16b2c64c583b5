"""Build libstencil.so (HIP kernels for gfx950 + the C++ host runtime) in-tree.

    python -m paper_1004_1741_amd.build [--jobs N] [--save-temps DIR]

Every source under csrc/ is compiled with hipcc for gfx950 only, then linked
into paper_1004_1741_amd/libstencil.so.  Compilation flags that matter for
the numerics: -ffp-contract=off (no FMA contraction: results match a
sequential evaluation bit for bit) and no fast-math.  Packed FP32 math is
disabled (the packed-fp32-ops target feature is switched off).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import pathlib
import shutil
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = PKG / "_build"
LIB = PKG / "libstencil.so"
ARCH = os.environ.get("STENCIL_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function", "-I" + str(ROOT / "include")]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and pathlib.Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libstencil")


def sources():
    return sorted(list(CSRC.glob("*.hip")) + list(CSRC.glob("*.cpp")))


def _compile(src: pathlib.Path, save_temps: str | None):
    obj = BUILD / (src.stem + ".o")
    cmd = [hipcc(), *COMMON]
    if src.suffix == ".hip":
        cmd += HIP_FLAGS + ["-x", "hip"]
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    if save_temps and src.suffix == ".hip":
        cmd += ["-save-temps=obj"]
    cmd += ["-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=str(BUILD))
    # the host pass does not know the packed-fp32-ops feature: drop that note
    noise = "'-packed-fp32-ops' is not a recognized feature"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    return obj, err


def build(jobs: int | None = None, save_temps: str | None = None, verbose: bool = False):
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, save_temps), srcs))
    for obj, err in results:
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", str(tmp),
           *[str(o) for o, _ in results], "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--save-temps", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, "1" if a.save_temps else None, a.verbose))


if __name__ == "__main__":
    main()
