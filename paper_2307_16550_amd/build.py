"""Build step of the gfx950 library: hipcc -> paper_2307_16550_amd/libgridhop.so (in-tree).

Run as `python -m paper_2307_16550_amd.build`.  Each csrc/*.hip is compiled to
an object of its own (in parallel: every kernel is launched from the file that
defines it, so no relocatable device code is needed), then the objects are
linked into the shared library.  The library links the HIP runtime by soname
(libamdhip64.so.7); when torch is imported first, its already-loaded runtime
is the one the library binds to.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libgridhop.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMPILE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# per-source additions: the direct decision keeps its matrix-core accumulators in
# VGPRs (without this the BF16 loops copy them between AGPRs every step)
FILE_FLAGS = {"direct.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}
LINK_FLAGS = ["--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _filtered(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())


def build(verbose: bool = False, extra=None, jobs: int | None = None) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    tmpdir = tempfile.mkdtemp(prefix="gridhop_build_")
    try:
        objs, cmds = [], []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([HIPCC, *COMPILE_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), *(extra or []), *inc, "-c",
                         src, "-o", obj])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
        with cf.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        failed = False
        for c, res in zip(cmds, results):
            msg = _filtered(res.stdout + res.stderr)
            if res.returncode != 0:
                failed = True
                sys.stderr.write(res.stdout + res.stderr)
            elif verbose and msg:
                print(msg)
        if failed:
            raise RuntimeError("hipcc failed building libgridhop.so")
        tmp = LIB + ".tmp"
        link = [HIPCC, *LINK_FLAGS, *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libgridhop.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
