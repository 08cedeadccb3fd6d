"""Build the HIP library libjk.so for gfx950 (hipcc), in-tree.

One object per bra angular pair (kern_bra.hip compiled with -DJK_LI/-DJK_LJ)
so the class kernels compile in parallel, plus the planner/API unit.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libjk.so")

LMAX_BUILT = 3
BRAS = [(i, j) for i in range(LMAX_BUILT + 1) for j in range(i + 1)]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stderr[-4000:])
    return r


# sources a kernel unit (kern_bra.hip) depends on; the other units depend on
# every source
_KERN_DEPS = ("kern_bra.hip", "jk_registry.h", "jk_device.h", "jk_common.h", "tables/jk_tables_meta.h",
              "tables/jk_tables_mom_meta.h")


def _stale(obj: str, kernel_unit: bool) -> bool:
    """True when obj is older than a source it depends on (incremental
    builds during development; build() without incremental compiles all)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    if kernel_unit:
        deps = [os.path.join(CSRC, d) for d in _KERN_DEPS]
    else:
        deps = [os.path.join(d, f) for d, _, fs in os.walk(CSRC) for f in fs]
        deps.append(os.path.join(ROOT, "include", "jk.h"))
    deps.append(__file__)
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, extra=(), verbose=False, incremental=False) -> str:
    """Compile every unit (incremental: only units older than a source) and
    link libjk.so."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = [("jk_api", os.path.join(CSRC, "jk_api.hip"), []), ("jk_batch", os.path.join(CSRC, "jk_batch.hip"), [])]
    for (i, j) in BRAS:
        units.append((f"kern_{i}{j}", os.path.join(CSRC, "kern_bra.hip"), [f"-DJK_LI={i}", f"-DJK_LJ={j}"]))
    # heaviest units first
    units.sort(key=lambda u: -sum(int(c) for c in u[0][-2:]) if u[0].startswith("kern") else 0)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {}
        for name, src, defs in units:
            obj = os.path.join(BUILD, name + ".o")
            objs.append(obj)
            if incremental and not _stale(obj, name.startswith("kern")):
                continue
            cmd = [hipcc, *FLAGS, *extra, *defs, "-c", src, "-o", obj]
            futs[ex.submit(_run, cmd)] = name
        for f in cf.as_completed(futs):
            f.result()
            if verbose:
                print("built", futs[f], file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
