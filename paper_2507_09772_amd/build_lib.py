"""Build the HIP library libjk.so for gfx950 (hipcc), in-tree.

One object per bra angular pair (kern_bra.hip compiled with -DJK_LI/-DJK_LJ)
so the class kernels compile in parallel, plus the planner/API unit.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libjk.so")

LMAX_BUILT = 4
BRAS = [(i, j) for i in range(LMAX_BUILT + 1) for j in range(i + 1)]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the kernel units also print each kernel's resource usage, checked below
RESOURCE_FLAGS = ["-Rpass-analysis=kernel-resource-usage"]
# Private memory (scratch) per lane.  Two family-2 (ff|ff) kernels once
# returned wrong values at 2736 and 2848 bytes per lane, while the same
# classes at about 800 bytes were right; the cause was not found.  So every
# kernel that spills is held to the scratch size recorded in KNOWN_GOOD (the
# sizes of the build whose kernels passed the parity tests on the device),
# and a kernel missing from that record to SCRATCH_LIMIT: a build whose
# register allocation moves further into scratch fails here instead of
# shipping.  `build_lib.py --record-scratch` rewrites the record from the
# current build (only after that build has passed the parity tests).
SCRATCH_LIMIT = 1024
KNOWN_GOOD = os.path.join(HERE, "kernel_scratch_gfx950.txt")
RESOURCES = os.path.join(BUILD, "kernel_resources.txt")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stderr[-4000:])
    return r


def kernel_resources(stderr: str) -> list:
    """(kernel, scratch bytes per lane, dynamic stack, VGPRs, LDS bytes) from
    the compiler's kernel-resource-usage remarks."""
    out, cur = [], None
    for line in stderr.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass")[0].strip()
        if body.startswith("Function Name:"):
            cur = {"name": body.split(":", 1)[1].strip(), "scratch": 0, "dynstack": False, "vgpr": 0, "lds": 0}
            out.append(cur)
        elif cur is not None:
            key, _, val = body.partition(":")
            val = val.strip()
            if key.startswith("ScratchSize"):
                cur["scratch"] = int(val)
            elif key.startswith("Dynamic Stack"):
                cur["dynstack"] = val == "True"
            elif key == "VGPRs":
                cur["vgpr"] = int(val)
            elif key.startswith("LDS Size"):
                cur["lds"] = int(val)
    return out


def known_good() -> dict:
    """Recorded scratch bytes per lane of the kernels that spill (name -> bytes)."""
    out = {}
    if os.path.exists(KNOWN_GOOD):
        with open(KNOWN_GOOD) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 2 and not line.startswith("#"):
                    out[f[1]] = int(f[0])
    return out


def check_resources(res: list, known: dict) -> None:
    """Refuses kernels with a dynamic stack, or with more scratch than their
    recorded size (SCRATCH_LIMIT for a kernel without a record)."""
    bad = [r for r in res if r["dynstack"] or r["scratch"] > known.get(r["name"], SCRATCH_LIMIT)]
    if bad:
        raise RuntimeError("kernels over their private-memory limit (the recorded size, else %d bytes per lane):\n"
                           % SCRATCH_LIMIT +
                           "\n".join(f"  {r['name']}: scratch {r['scratch']} B (limit "
                                      f"{known.get(r['name'], SCRATCH_LIMIT)}), dynamic stack {r['dynstack']}"
                                      for r in bad))


def record_scratch(res: list) -> None:
    with open(KNOWN_GOOD, "w") as fh:
        fh.write("# scratch bytes per lane of each spilling kernel in the build that passed the parity tests\n")
        fh.write("# (written by build_lib.py --record-scratch; checked by every build)\n")
        for r in sorted(res, key=lambda r: r["name"]):
            if r["scratch"] > 0:
                fh.write(f"{r['scratch']} {r['name']}\n")


# sources a kernel unit (kern_bra.hip) depends on; the other units depend on
# every source
_KERN_DEPS = ("kern_bra.hip", "kern_persist.hip", "jk_registry.h", "jk_device.h", "jk_common.h",
              "tables/jk_tables_meta.h", "tables/jk_tables_mom_meta.h")


def _stale(obj: str, kernel_unit: bool) -> bool:
    """True when obj is older than a source it depends on (incremental
    builds during development; build() without incremental compiles all)."""
    if not os.path.exists(obj) or (kernel_unit and not os.path.exists(obj[:-2] + ".res.json")):
        return True
    t = os.path.getmtime(obj)
    if kernel_unit:
        deps = [os.path.join(CSRC, d) for d in _KERN_DEPS]
    else:
        deps = [os.path.join(d, f) for d, _, fs in os.walk(CSRC) for f in fs]
        deps.append(os.path.join(ROOT, "include", "jk.h"))
    deps.append(__file__)
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, extra=(), verbose=False, incremental=False, record=False) -> str:
    """Compile every unit (incremental: only units older than a source) and
    link libjk.so."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = [("jk_api", os.path.join(CSRC, "jk_api.hip"), []), ("jk_batch", os.path.join(CSRC, "jk_batch.hip"), []),
             ("jk_noalloc", os.path.join(CSRC, "jk_noalloc.hip"), []),
             ("kern_persist", os.path.join(CSRC, "kern_persist.hip"), [])]
    for (i, j) in BRAS:
        units.append((f"kern_{i}{j}", os.path.join(CSRC, "kern_bra.hip"), [f"-DJK_LI={i}", f"-DJK_LJ={j}"]))
    # heaviest units first
    units.sort(key=lambda u: -sum(int(c) for c in u[0][-2:]) if u[0][-2:].isdigit() else 0)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {}
        for name, src, defs in units:
            obj = os.path.join(BUILD, name + ".o")
            objs.append(obj)
            if incremental and not _stale(obj, name.startswith("kern")):
                continue
            rflags = RESOURCE_FLAGS if name.startswith("kern") else []
            cmd = [hipcc, *FLAGS, *rflags, *extra, *defs, "-c", src, "-o", obj]
            futs[ex.submit(_run, cmd)] = name
        for f in cf.as_completed(futs):
            name = futs[f]
            if name.startswith("kern"):
                # each kernel unit's resource remarks, kept beside its object
                with open(os.path.join(BUILD, name + ".res.json"), "w") as fh:
                    json.dump(kernel_resources(f.result().stderr), fh)
            if verbose:
                print("built", name, file=sys.stderr)
    res = []
    for name, _, _ in units:
        if name.startswith("kern"):
            with open(os.path.join(BUILD, name + ".res.json")) as fh:
                res += json.load(fh)
    with open(RESOURCES, "w") as fh:
        for r in sorted(res, key=lambda r: -r["scratch"]):
            fh.write(f"{r['scratch']:6d} B scratch  {r['vgpr']:4d} VGPRs  {r['lds']:6d} B LDS  {r['name']}\n")
    if record:
        record_scratch(res)
    check_resources(res, known_good())
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv, record="--record-scratch" in sys.argv))
