"""Autotuner for the per-device kernel tuning table (tune_gfx950.txt).

Three searches, each timing every class kernel through the library's
per-kernel timing (HIP events around each launch) on the given workloads:

1. family and row mode: for each precision, every class forced to each
   built family (1, 2, 3) with row mode for long bras, off, or for every
   bra; per angular class the fastest (family, row) pair is kept;
2. task shape (the fragmentation of Section 3.2): with those choices, the
   long-bra threshold (min_kets) and the kets per row task (chunk) from a
   small grid around the defaults; per class the fastest pair is kept;
3. mixed split: with those choices, each class's time in mixed builds
   (its single- and double-precision passes) against its FP64 time; a
   class whose mixed time is not at least 3 % lower runs in double
   precision in mixed builds ("split li lj lk ll 0").

Each class's time is summed over its primitive-count variants, the
workloads and both kinds of launch (row tasks and tiles).  The table is
written next to the library, which loads it at start-up.

Run on the GPU: python -m paper_2507_09772_amd.autotune [--workloads c1 c2]
(--split-only: keep the shipped table's families and shapes and redo the
third search only).
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
# shape grid: (min_kets, chunk scale against the family default)
SHAPES = [(m, s) for m in (96, 192, 384) for s in (0.5, 1.0, 2.0)]


def default_chunk(fam, li):
    """Kets per row task of a family (row_chunk in the library)."""
    if fam == 1:
        return 2048
    nci = (li + 1) * (li + 2) // 2
    return 256 * max(1, 64 // nci)  # families 2 and 3 step by their quartets per wave


def split_lines(jk, synth, torch, names):
    """The third search: classes whose mixed builds are not faster."""
    for c in jk.canonical_classes():
        jk.tune_set_split(*c, 1)
    t64 = timed_classes(jk, synth, torch, names, "fp64")
    tmx = timed_classes(jk, synth, torch, names, "mixed")
    lines, report = [], {}
    for c in jk.canonical_classes():
        if c not in t64 or c not in tmx:
            continue
        report[f"split ({c[0]}{c[1]}|{c[2]}{c[3]})"] = {"fp64": t64[c], "mixed": tmx[c]}
        off = tmx[c] > 0.97 * t64[c]
        print(f"split ({c[0]}{c[1]}|{c[2]}{c[3]}): fp64 {t64[c]:8.3f} mixed {tmx[c]:8.3f} ms -> "
              f"{'off' if off else 'on'}", flush=True)
        if off:
            lines.append(f"split {c[0]} {c[1]} {c[2]} {c[3]} 0")
    return lines, report


def timed_classes(jk, synth, torch, names, precision, steps=2):
    """Per angular class total ms of one build (summed over the workloads)."""
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
            tot[(t.li, t.lj, t.lk, t.ll)] += t.ms / steps
        plan.close()
    return tot


def force(jk, precision, family, row):
    for c in jk.canonical_classes():
        _, avail = jk.tune_get(*c, precision)
        jk.tune_set(*c, precision, family if avail & (1 << (family - 1)) else 0)
        jk.tune_set_row(*c, precision, row)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["c1", "c2"])
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--no-shapes", action="store_true")
    ap.add_argument("--split-only", action="store_true")
    args = ap.parse_args()
    import torch

    from paper_2507_09772_amd import jk, synth
    if args.split_only:
        keep = [l.rstrip("\n") for l in open(OUT) if not l.startswith("split")]
        if not any(l.startswith("# split lines") for l in keep):
            keep.insert(next(i for i, l in enumerate(keep) if not l.startswith("#")),
                        "# split lines: li lj lk ll 0 (the class runs in double precision in mixed builds)")
        lines, report = split_lines(jk, synth, torch, args.workloads)
        with open(args.out, "w") as f:
            f.write("\n".join(keep + lines) + "\n")
        print(json.dumps(report), flush=True)
        return
    lines = ["# kernel family per (class, precision), chosen by paper_2507_09772_amd/autotune.py",
             f"# workloads: {' '.join(args.workloads)}; columns: li lj lk ll precision(0 fp64, 2 fp32) family "
             "row(1 long bras, 2 off, 3 all bras)",
             "# shape lines: li lj lk ll min_kets chunk (the long-bra threshold and kets per row task)",
             "# split lines: li lj lk ll 0 (the class runs in double precision in mixed builds)"]
    report = {}
    choice = {}
    for precision in ("fp64", "fp32"):
        t = {}
        for f in (1, 2, 3):
            for r in (1, 2, 3):
                if f == 3 and r == 2:
                    continue
                force(jk, precision, f, r)
                t[(f, r)] = timed_classes(jk, synth, torch, args.workloads, precision)
        for c in jk.canonical_classes():
            _, avail = jk.tune_get(*c, precision)
            opts = {k: v.get(c) for k, v in t.items() if avail & (1 << (k[0] - 1)) and v.get(c) is not None}
            if not opts:
                continue
            (fam, row), best = min(opts.items(), key=lambda kv: kv[1])
            choice[(c, precision)] = (fam, row)
            report[f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]})"] = {f"f{k[0]}r{k[1]}": v for k, v in opts.items()}
            lines.append(f"{c[0]} {c[1]} {c[2]} {c[3]} {jk.PRECISION[precision]} {fam} {row}")
            print(f"{precision} ({c[0]}{c[1]}|{c[2]}{c[3]}): " +
                  "  ".join(f"f{k[0]}/{ROWNAME[k[1]]} {v:8.3f}" for k, v in sorted(opts.items())) +
                  f"  -> family {fam} {ROWNAME[row]}", flush=True)
    # the chosen families and row modes, then the task-shape grid (FP64 timings)
    for (c, precision), (fam, row) in choice.items():
        jk.tune_set(*c, precision, fam)
        jk.tune_set_row(*c, precision, row)
    if not args.no_shapes:
        ts = {}
        for mk, sc in SHAPES:
            for c in jk.canonical_classes():
                fam = choice.get((c, "fp64"), (1, 1))[0]
                jk.tune_set_shape(*c, mk, int(default_chunk(fam, c[0]) * sc))
            ts[(mk, sc)] = timed_classes(jk, synth, torch, args.workloads, "fp64")
        for c in jk.canonical_classes():
            opts = {k: v.get(c) for k, v in ts.items() if v.get(c) is not None}
            if not opts:
                continue
            (mk, sc), best = min(opts.items(), key=lambda kv: kv[1])
            base = opts.get((192, 1.0), best)
            fam = choice.get((c, "fp64"), (1, 1))[0]
            print(f"shape ({c[0]}{c[1]}|{c[2]}{c[3]}): best min_kets {mk} chunk x{sc} {best:.3f} ms "
                  f"(default {base:.3f} ms)", flush=True)
            if (mk, sc) != (192, 1.0) and best < 0.97 * base:
                lines.append(f"shape {c[0]} {c[1]} {c[2]} {c[3]} {mk} {int(default_chunk(fam, c[0]) * sc)}")
            report[f"shape ({c[0]}{c[1]}|{c[2]}{c[3]})"] = {f"m{k[0]}x{k[1]}": v for k, v in opts.items()}
    split, rs = split_lines(jk, synth, torch, args.workloads)
    lines += split
    report.update(rs)
    for c in jk.canonical_classes():
        jk.tune_set_shape(*c, 0, 0)
        jk.tune_set_split(*c, 1)
        for precision in ("fp64", "fp32"):
            jk.tune_set(*c, precision, 0)
            jk.tune_set_row(*c, precision, 0)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
