"""Autotuner for the per-device kernel tuning table (tune_gfx950.txt).

For each workload and precision it times every class kernel once per
available family (HIP events around each launch, through the library's
per-kernel timing), sums each angular class's time over its primitive-count
variants and over the workloads, and keeps the faster family.  The chosen
table is written next to the library, which loads it at start-up.

Run on the GPU: python -m paper_2507_09772_amd.autotune [--workloads c1 c2]
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

OUT = os.path.join(HERE, "tune_gfx950.txt")
ROWNAME = {1: "row", 2: "tile", 3: "allrow"}


def measure(jk, synth, torch, names, precision, family, row, steps=2):
    """Per angular class total ms with every class forced to ``family``
    where built (default elsewhere) and row mode on (1) or off (2)."""
    for c in jk.canonical_classes():
        _, avail = jk.tune_get(*c, precision)
        jk.tune_set(*c, precision, family if avail & family else 0)
        jk.tune_set_row(*c, precision, row)
    tot = collections.defaultdict(float)
    for name in names:
        wl = synth.workload(name)
        plan = jk.Plan(wl.mol, wl.cutoff)
        D = torch.from_numpy(wl.D).cuda()
        J, K = plan.execute(D, precision=precision)
        torch.cuda.synchronize()
        plan.profile(True)
        for _ in range(steps):
            plan.execute(D, J, K, precision=precision)
        torch.cuda.synchronize()
        for t in plan.timings():
            # every (class, precision, kind) entry has one launch per build
            tot[(t.li, t.lj, t.lk, t.ll)] += t.ms / steps
        plan.close()
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["c1", "c2"])
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    import torch

    from paper_2507_09772_amd import jk, synth
    lines = ["# kernel family per (class, precision), chosen by paper_2507_09772_amd/autotune.py",
             f"# workloads: {' '.join(args.workloads)}; columns: li lj lk ll precision(0 fp64, 2 fp32) family "
             "row(1 long bras, 2 off, 3 all bras)"]
    report = {}
    for precision in ("fp64", "fp32"):
        t = {(f, r): measure(jk, synth, torch, args.workloads, precision, f, r) for f in (1, 2) for r in (1, 2, 3)}
        for c in jk.canonical_classes():
            _, avail = jk.tune_get(*c, precision)
            opts = {k: v.get(c) for k, v in t.items() if avail & k[0] and v.get(c) is not None}
            if not opts:
                continue
            (fam, row), best = min(opts.items(), key=lambda kv: kv[1])
            report[f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]})"] = {f"f{k[0]}r{k[1]}": v for k, v in opts.items()}
            lines.append(f"{c[0]} {c[1]} {c[2]} {c[3]} {jk.PRECISION[precision]} {fam} {row}")
            print(f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]}): " +
                  "  ".join(f"f{k[0]}/{ROWNAME[k[1]]} {v:8.3f}" for k, v in sorted(opts.items())) +
                  f"  -> family {fam} {ROWNAME[row]}", flush=True)
        for c in jk.canonical_classes():
            jk.tune_set(*c, precision, 0)
            jk.tune_set_row(*c, precision, 0)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
