"""Build libtm.so (the HIP library behind include/tm.h) for gfx950.

Compiles every .hip source in csrc/ (the per-grid kernel file once per
compiled grid) with hipcc in parallel into ./_build at the repository root
and links paper_2302_13524_amd/libtm.so. Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtm.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
] + os.environ.get("TM_EXTRA_FLAGS", "").split()


def grids() -> list[tuple[int, int]]:
    txt = open(os.path.join(CSRC, "grids.hpp")).read()
    body = txt[txt.index("#define TM_GRID_LIST"):]
    body = body[: body.index("namespace")]
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", body)]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _run(cmd: list[str]) -> tuple[list[str], int, str]:
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return cmd, r.returncode, err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    units = []
    for a, b in grids():
        units.append(([cc, *FLAGS, f"-DGL1={a}", f"-DGL2={b}", "-c", os.path.join(CSRC, "grid_inst.hip"),
                       "-o", os.path.join(BUILD, f"grid_{a}_{b}.o")]))
    for src in sorted(os.listdir(CSRC)):
        if src == "grid_inst.hip" or not (src.endswith(".hip") or src.endswith(".cpp")):
            continue
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        units.append([cc, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(16, os.cpu_count() or 4)
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, rc, err in ex.map(_run, units):
            if rc != 0:
                failed.append((cmd, err))
            elif verbose and err:
                print(err, file=sys.stderr)
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + e for c, e in failed)
        raise RuntimeError("hipcc failed:\n" + msg)
    objs = [u[-1] for u in units]
    tmp = LIB + ".tmp"
    cmd, rc, err = _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
                         "-Wl,-rpath,/opt/rocm/lib"])
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
