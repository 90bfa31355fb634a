"""Build of the native library ``libprobestream.so`` for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libprobestream.so")
SOURCES = ["trace.hip", "blend.hip", "batched.hip", "bounce.hip", "select.hip", "pack.hip", "entropy.hip", "receive.hip", "yuv.hip", "ceilings.hip", "bvh.cpp", "pv_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are not generated (compiler-formed v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-value", "-Wno-unused-result",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source to an object (in parallel), then links."""
    import concurrent.futures
    import tempfile
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="pvbuild") as tmpd:
        objs, cmds = [], []
        for s in SOURCES:
            obj = os.path.join(tmpd, s + ".o")
            objs.append(obj)
            cmds.append([HIPCC, *[f for f in FLAGS if f != "-shared"], *inc, "-c", os.path.join(CSRC, s), "-o", obj])
        workers = jobs or min(len(cmds), os.cpu_count() or 1)
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            for cmd, rc in zip(cmds, ex.map(_run(verbose), cmds)):
                if rc != 0:
                    raise subprocess.CalledProcessError(rc, cmd)
        tmp = SO + ".tmp"
        link = [HIPCC, *FLAGS, *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), file=sys.stderr)
        subprocess.check_call(link)
        os.replace(tmp, SO)
    return SO


def _run(verbose):
    def go(cmd):
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        return subprocess.call(cmd)
    return go


if __name__ == "__main__":
    print(build(verbose=True))
