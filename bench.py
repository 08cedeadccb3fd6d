#!/usr/bin/env python
"""J/K build benchmark on one MI355X.

Workload (default): 64 waters on a 4x4x4 lattice, split-valence +
polarisation Cartesian basis (6-31G*-shaped), 1216 AOs, one density,
Schwarz cutoff 1e-13.  Inputs are seeded and synthetic and resident in HBM
before the timed region; a step is one full J+K build (every hot-path
kernel: density transform when spherical, all class kernels, finalize).

Prints one JSON line: FP64 builds/s as ``value``, ERI quartets/s, the mixed
FP32/FP64 rate and its energy error against the FP64 GPU build, the
roofline of the dominant kernel from HIP events over the timed region, and
the CPU reference timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J/K builds/s + ERI quartets/s, FP64 vs mixed FP32/FP64 at |dE|<=1e-6 Eh"
PEAK_FP64_VECTOR = 78.6   # TFLOP/s, MI355X FP64 vector
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X FP32 vector

WORKLOAD_TEXT = {
    "c0": "3 waters, basis A (6-31G*-shaped, Cartesian), 57 AOs, 1 density, cutoff 1e-13",
    "c1": "64 waters 4x4x4 lattice, basis A (6-31G*-shaped, Cartesian), 1216 AOs, 1 density, cutoff 1e-13",
    "c2": "32 waters, basis B (TZ2P-shaped, spherical, up to f), 1376 AOs, 1 density, cutoff 1e-13",
}
BATCH_TEXT = ("256 molecules of 1-8 waters, half basis A (Cartesian), half basis B (spherical), "
              "4 densities each, cutoff 1e-13")


COUNTERS = os.path.join(ROOT, "profiles", "jk_c1_fp64_hbm_counters.txt")


def source_sha256():
    """Fingerprint of the kernel sources and build flags (matches the one
    recorded in the profiles)."""
    import glob
    import hashlib
    pkg = os.path.join(ROOT, "paper_2507_09772_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "**", "*.h"), recursive=True) +
                   glob.glob(os.path.join(pkg, "csrc", "*.hip")) + [os.path.join(pkg, "build_lib.py")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by the
    copy-kernel calibration), or (None, reason) when the summary is missing,
    does not cover the kernel, or was taken from other kernel sources."""
    if not os.path.exists(COUNTERS):
        return None, "no counter summary"
    text = open(COUNTERS).read()
    m = re.search(r"kernel sources sha256[^:]*: ([0-9a-f]+)", text)
    if not m or m.group(1) != source_sha256():
        return None, "kernel sources changed since the counters were taken"
    cal = re.search(r"^calibration fetch_factor ([0-9.]+) write_factor ([0-9.]+)", text, re.M)
    got = {}
    for line in text.splitlines():
        f = line.split(None, 4)
        if len(f) == 5 and f[3] in ("FETCH_SIZE", "WRITE_SIZE") and f"jk::{kernel}(" in f[4]:
            got[f[3]] = float(f[2])
    if not cal or len(got) != 2:
        return None, "kernel not in the counter summary"
    fetch = got["FETCH_SIZE"] * float(cal.group(1)) * 1024
    write = got["WRITE_SIZE"] * float(cal.group(2)) * 1024
    return fetch + write, f"rocprofv3 FETCH_SIZE+WRITE_SIZE per dispatch, {os.path.relpath(COUNTERS, ROOT)}"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(plan, D, J, K, precision, steps, warmup, torch, profile=False):
    for _ in range(warmup):
        plan.execute(D, J, K, precision=precision)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(D, J, K, precision=precision)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tim = plan.timings() if profile else []
    if profile:
        plan.profile(False)
    return dt, tim


def kernel_name(t):
    """Name of the kernel instantiation a timing entry belongs to (the
    profiler's kernel name without namespace)."""
    prec = "double" if t.precision == 0 else "float"
    cls = f"{t.li}, {t.lj}, {t.lk}, {t.ll}"
    if t.kind in (1, 3):
        return f"jk_k{t.family}_row<{cls}, {prec}, {256 if t.kind == 1 else 64}, false>"
    return f"jk_k{t.family}<{cls}, {prec}, {0 if t.kind == 0 else 2}>"


def kernel_groups(timings):
    out = {}
    for t in timings:
        g = out.setdefault(kernel_name(t), {"ms": 0.0, "launches": 0, "flops": 0.0, "quartets": 0})
        g["ms"] += t.ms
        g["launches"] += t.launches
        g["flops"] += t.model_flops
        g["quartets"] += t.nquartets
    return out


def cpu_baseline(wl, target_s: float):
    """Time the oracle's eight-fold build over a random sample of bra shell
    pairs (all canonical kets of each) and scale to one full build."""
    import numpy as np

    from oracle import oracle as orc
    orc.build_oracle(force=False)
    Q = orc.schwarz(wl.mol)
    ns = wl.mol.nshell
    npair = ns * (ns + 1) // 2
    rng = np.random.default_rng(12345)
    order = rng.permutation(npair)
    n = 32
    used, spent = 0, 0.0
    while True:
        sel = order[used:used + n]
        t0 = time.perf_counter()
        orc.jk_subset(wl.mol, wl.D, Q, sel, wl.cutoff)
        spent += time.perf_counter() - t0
        used += sel.size
        if spent >= target_s or used >= npair:
            break
        # aim the next chunk at the remaining time
        n = int(min(npair - used, max(32, used * (target_s - spent) / max(spent, 1e-3))))
    full_s = spent * npair / used
    return {"value": 1.0 / full_s, "unit": "builds/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"eight-fold oracle over {used} random bra shell pairs of {npair} (each with all its "
                      f"canonical kets), {spent:.1f} s, scaled by {npair}/{used} to one build "
                      f"({full_s:.0f} s per build)"}


def bench_batch(args, torch, jk, synth):
    """Batched builds over the 256-molecule set: one graph replay per step
    against the same molecules built one jk_execute at a time."""
    import numpy as np
    wls = synth.batch_workload()
    t0 = time.perf_counter()
    plans = [jk.Plan(w.mol, w.cutoff) for w in wls]
    t_plan = time.perf_counter() - t0
    Ds = [torch.from_numpy(w.D).cuda() for w in wls]
    Js = [torch.empty_like(D) for D in Ds]
    Ks = [torch.empty_like(D) for D in Ds]
    nset = Ds[0].shape[0]
    nq = sum(p.stats().nquartets for p in plans)
    res = {"config": BATCH_TEXT, "nmol": len(wls), "nset": nset, "plan_seconds": t_plan, "nquartets": nq}
    log(f"batch: {len(wls)} plans in {t_plan:.1f} s, {nq} quartets")
    # mixed batches only on request: their FP64 list pass is slow for small
    # molecules (most quartets are above the threshold)
    for precision in ("fp64",) + (("mixed",) if args.batch_mixed else ()):
        b = jk.Batch(plans, nset=nset, precision=precision, mix_threshold=args.mix_threshold)
        for _ in range(max(args.warmup, 1)):
            b.execute(Ds, Js, Ks)
        torch.cuda.synchronize()
        log(f"batch {precision}: warm")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.execute(Ds, Js, Ks)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        e = [2.0 * float(np.sum(w.D * J.cpu().numpy())) for w, J in zip(wls, Js)]
        log(f"batch {precision}: {dt * 1e3:.1f} ms per batch; now one jk_execute per molecule")
        # the same molecules one jk_execute each
        for p, D, J, K in zip(plans, Ds, Js, Ks):
            p.execute(D, J, K, precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for p, D, J, K in zip(plans, Ds, Js, Ks):
                p.execute(D, J, K, precision=precision)
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t0) / args.steps
        e1 = [2.0 * float(np.sum(w.D * J.cpu().numpy())) for w, J in zip(wls, Js)]
        res[precision] = {"ms_per_step": dt * 1e3, "molecule_builds_per_s": len(wls) / dt,
                          "density_builds_per_s": len(wls) * nset / dt, "quartets_per_s": nq / dt,
                          "one_by_one_ms": dts * 1e3, "speedup_vs_one_by_one": dts / dt,
                          "max_dE_J_vs_one_by_one": float(np.abs(np.subtract(e, e1)).max())}
        log(f"batch {precision}: {dt * 1e3:.2f} ms/step ({len(wls) / dt:.0f} molecule builds/s), one by one "
            f"{dts * 1e3:.2f} ms")
        b.close()
    return res


def bench_dscreen(args, torch, plan, wl, dt_full):
    """Incremental build as in a late direct-SCF iteration: the density
    change dD = 1e-4 * (a fresh seeded density - D) with density screening
    at --dscreen; reports its time against the full build, and its error
    against the same dD built unscreened."""
    import numpy as np
    from paper_2507_09772_amd import synth
    nocc = int(np.rint(np.trace(wl.D[0])))  # D = C C^T with orthonormal C
    D2 = synth.random_density(wl.mol.nao, nocc, [999, 1], wl.D.shape[0])
    dD = torch.from_numpy(1e-4 * (D2 - wl.D)).cuda()
    J = torch.empty_like(dD)
    K = torch.empty_like(dD)
    plan.set_density_screening(0.0)
    plan.execute(dD, J, K)
    torch.cuda.synchronize()
    J0, K0 = J.cpu().numpy(), K.cpu().numpy()
    plan.set_density_screening(args.dscreen)
    for _ in range(max(args.warmup, 1)):
        plan.execute(dD, J, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute(dD, J, K)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    plan.set_density_screening(0.0)
    err_j = float(np.abs(J.cpu().numpy() - J0).max())
    err_k = float(np.abs(K.cpu().numpy() - K0).max())
    log(f"incremental (dD ~ 1e-4, dscreen {args.dscreen:g}): {dt * 1e3:.2f} ms/build, max|dJ| {err_j:.1e} "
        f"max|dK| {err_k:.1e} vs unscreened")
    return {"threshold": args.dscreen, "delta_D": "1e-4 * (seeded density - D)", "ms_per_step": dt * 1e3,
            "builds_per_s": 1.0 / dt, "speedup_vs_full_build": dt_full / dt,
            "max_dJ_vs_unscreened": err_j, "max_dK_vs_unscreened": err_k}


def bench_micro(args, torch, jk, synth):
    """Micro-benchmarks after the paper's appendix B, on the c1 / c2
    geometries with one uniform shell per atom:
      * (ss|ss) with 1..8 identical primitives per shell (the same contracted
        function, so the same quartets): FP64 and FP32 time and their ratio;
      * (dd|dd) and (ff|ff) with 1..4 densities: time against the number of
        densities, fitted to integral generation + per-density contraction."""
    import numpy as np
    out = {"ssss_nprim": [], "ndm": {}}
    ref = None
    for npr in range(1, 9):
        wl = synth.uniform_shell_workload("c1", 0, npr, 0.2700058226)
        plan = jk.Plan(wl.mol, wl.cutoff)
        D = torch.from_numpy(wl.D).cuda()
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        row = {"nprim": npr, "nquartets": plan.stats().nquartets}
        for prec in ("fp64", "fp32"):
            dt, _ = timed_steps(plan, D, J, K, prec, args.steps, args.warmup, torch)
            row[prec + "_ms"] = dt * 1e3
            if prec == "fp64":
                Jh = J.cpu().numpy()
                ref = Jh if ref is None else ref
                row["max_dJ_vs_nprim1"] = float(np.abs(Jh - ref).max())
        row["fp32_speedup"] = row["fp64_ms"] / row["fp32_ms"]
        log(f"(ss|ss) nprim {npr}: fp64 {row['fp64_ms']:.3f} ms  fp32 {row['fp32_ms']:.3f} ms  "
            f"ratio {row['fp32_speedup']:.2f}  (|dJ| vs nprim 1: {row['max_dJ_vs_nprim1']:.1e})")
        out["ssss_nprim"].append(row)
        plan.close()
    for l, lab in ((2, "dddd"), (3, "ffff")):
        wl = synth.uniform_shell_workload("c2", l, 1, 1.2700058226, nset=4)
        plan = jk.Plan(wl.mol, wl.cutoff)
        ts = []
        J1 = None
        for n in range(1, 5):
            D = torch.from_numpy(np.ascontiguousarray(wl.D[:n])).cuda()
            J = torch.empty_like(D)
            K = torch.empty_like(D)
            dt, _ = timed_steps(plan, D, J, K, "fp64", args.steps, args.warmup, torch)
            ts.append(dt * 1e3)
            if n == 1:
                J1 = J[0].cpu().numpy()
            dj = float(np.abs(J[0].cpu().numpy() - J1).max())
            log(f"({lab[:2]}|{lab[2:]}) ndm {n}: {dt * 1e3:.2f} ms (|dJ[0]| vs ndm 1: {dj:.1e})")
        slope, icpt = np.polyfit(np.arange(1, 5), ts, 1)
        out["ndm"][lab] = {"ms": ts, "integral_ms": float(icpt), "per_density_ms": float(slope),
                           "nquartets": plan.stats().nquartets}
        plan.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOAD_TEXT) + ["c4"],
                    help="c4: only the 256-molecule batched builds")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-molecule batched builds")
    ap.add_argument("--no-dscreen", action="store_true", help="skip the incremental (density-screened) build")
    ap.add_argument("--micro", action="store_true", help="only the appendix-B style micro-benchmarks")
    ap.add_argument("--batch-mixed", action="store_true", help="also time mixed-precision batches")
    ap.add_argument("--dscreen", type=float, default=1e-10, help="density screening threshold")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mix-threshold", type=float, default=1e-4)
    ap.add_argument("--top", type=int, default=12, help="kernels listed per build")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scales the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); multi-GPU sharding is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_09772_amd import jk, synth

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8}), flush=True)
        return

    torch.cuda.set_device(0)
    if args.micro:
        print(json.dumps({"micro": bench_micro(args, torch, jk, synth)}), flush=True)
        return
    if args.workload == "c4":
        res = bench_batch(args, torch, jk, synth)
        r64 = res["fp64"]
        out = {"metric": METRIC, "value": r64["molecule_builds_per_s"], "unit": "molecule builds/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic (seeded water clusters, random orthonormal C)",
               "config": {"workload": f"c4: {BATCH_TEXT}", "precision": "fp64"}, "batch": res,
               "roofline": None, "cpu_baseline": None}
        print(json.dumps(out), flush=True)
        return
    wl = synth.workload(args.workload)
    log(f"workload {args.workload}: {wl.mol.nshell} shells, {wl.mol.nao} AOs")
    t0 = time.perf_counter()
    plan = jk.Plan(wl.mol, wl.cutoff)
    st = plan.stats()
    log(f"plan: {time.perf_counter() - t0:.2f} s, {st.nquartets} quartets, {st.nprim_quartets} primitive "
        f"quartets, {st.nclasses} classes")
    D = torch.from_numpy(wl.D).cuda()
    J = torch.empty_like(D)
    K = torch.empty_like(D)

    dt64, tim64 = timed_steps(plan, D, J, K, "fp64", args.steps, args.warmup, torch, profile=True)
    log(f"fp64: {dt64 * 1e3:.2f} ms/build")
    D_h = wl.D
    J64, K64 = J.cpu().numpy(), K.cpu().numpy()
    ej64 = 2.0 * float(np.sum(D_h * J64))
    ek64 = float(np.sum(D_h * K64))

    # dominant kernel: group the per-launch timings by kernel instantiation
    # (class, family, precision, kind), as the profiler groups by name
    kern = kernel_groups(tim64)
    dom_name, dom = max(kern.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    traffic, traffic_src = hbm_traffic(dom_name) if args.workload == "c1" else (None, "counters taken for c1 only")
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic, "traffic_source": traffic_src,
                "kernel": dom_name,
                "avg_launch_ms": avg_ms, "launches_per_build": dom["launches"] / args.steps,
                "model_flops_per_launch": dom["flops"] / dom["launches"],
                "share_of_build": dom["ms"] / args.steps / (dt64 * 1e3)}
    whole = st.model_flops / dt64 / 1e12
    for name, k in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])[:args.top]:
        log(f"  {name:44s} {k['ms'] / args.steps:8.3f} ms/build  {k['launches'] / args.steps:4.0f} launches  "
            f"{k['flops'] / (k['ms'] * 1e-3) / 1e12 if k['ms'] > 0 else 0:6.2f} TF/s")

    out = {"metric": METRIC, "value": 1.0 / dt64, "unit": "builds/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt64 * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded water lattice, random orthonormal C)",
           "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", "nset": 1,
                      "precision": "fp64", "cutoff": wl.cutoff},
           "quartets_per_s": st.nquartets / dt64, "prim_quartets_per_s": st.nprim_quartets / dt64,
           "nquartets": st.nquartets, "model_tflops": whole, "model_frac_fp64_peak": whole / PEAK_FP64_VECTOR,
           "E_J": ej64, "E_K": ek64, "roofline": roofline}

    if not args.no_mixed:
        dtm, timm = timed_steps(plan, D, J, K, "mixed", args.steps, args.warmup, torch, profile=True)
        Jm, Km = J.cpu().numpy(), K.cpu().numpy()
        ejm, ekm = 2.0 * float(np.sum(D_h * Jm)), float(np.sum(D_h * Km))
        f32 = sum(t.ms for t in timm if t.precision == jk.JK_FP32)
        f64 = sum(t.ms for t in timm if t.precision == jk.JK_FP64)
        log(f"mixed: {dtm * 1e3:.2f} ms/build (fp64 kernels {f64 / args.steps:.2f} ms, fp32 kernels "
            f"{f32 / args.steps:.2f} ms), dE_J {ejm - ej64:.2e} dE_K {ekm - ek64:.2e}")
        out["mixed"] = {"builds_per_s": 1.0 / dtm, "quartets_per_s": st.nquartets / dtm, "ms_per_step": dtm * 1e3,
                        "speedup_vs_fp64": dt64 / dtm, "dE_J_vs_fp64_gpu": ejm - ej64, "dE_K_vs_fp64_gpu": ekm - ek64,
                        "max_dJ_vs_fp64_gpu": float(np.abs(Jm - J64).max()),
                        "max_dK_vs_fp64_gpu": float(np.abs(Km - K64).max()),
                        "threshold": args.mix_threshold}
    if not args.no_dscreen:
        out["density_screening"] = bench_dscreen(args, torch, plan, wl, dt64)
    if not args.no_batch:
        out["batch"] = bench_batch(args, torch, jk, synth)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
