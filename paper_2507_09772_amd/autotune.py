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


def measure(jk, synth, torch, names, precision, family, steps=2):
    """Per angular class total ms with every class forced to ``family``
    where built (default elsewhere)."""
    for c in jk.canonical_classes():
        _, avail = jk.tune_get(*c, precision)
        jk.tune_set(*c, precision, family if avail & family else 0)
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
        want = jk.JK_FP32 if precision == "fp32" else jk.JK_FP64
        for t in plan.timings():
            if t.precision == want:
                tot[(t.li, t.lj, t.lk, t.ll)] += t.ms / t.launches
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
             f"# workloads: {' '.join(args.workloads)}; columns: li lj lk ll precision(0 fp64, 2 fp32) family"]
    report = {}
    for precision in ("fp64", "fp32"):
        t1 = measure(jk, synth, torch, args.workloads, precision, 1)
        t2 = measure(jk, synth, torch, args.workloads, precision, 2)
        for c in jk.canonical_classes():
            _, avail = jk.tune_get(*c, precision)
            a, b = t1.get(c), t2.get(c)
            if avail != 3 or a is None or b is None:
                continue
            fam = 1 if a <= b else 2
            report[f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]})"] = {"family1_ms": a, "family2_ms": b, "chosen": fam}
            lines.append(f"{c[0]} {c[1]} {c[2]} {c[3]} {jk.PRECISION[precision]} {fam}")
            print(f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]}): family1 {a:8.3f} ms  family2 {b:8.3f} ms -> {fam}",
                  flush=True)
        for c in jk.canonical_classes():
            jk.tune_set(*c, precision, 0)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
