#!/usr/bin/env python
"""J/K build benchmark on one MI355X.

Headline workload: 64 waters on a 4x4x4 lattice, split-valence +
polarisation Cartesian basis (6-31G*-shaped), 1216 AOs, one density,
Schwarz cutoff 1e-13.  Inputs are seeded and synthetic and resident in HBM
before the timed region; a step is one full J+K build (every hot-path
kernel: density transform when spherical, all class kernels, finalize).

The same run measures every configuration of the workload set:
  c1  the headline molecule, FP64 and mixed FP32/FP64;
  c2  32 waters in the spherical triple-zeta-shaped basis up to f, FP64 and
      mixed;
  c3  the mixed-precision split (threshold 1e-4 on Q_IJ Q_KL max|D_block|)
      on the c1 and c2 molecules: FP32 quartet fraction, speedup over FP64
      and the error against the oracle's stored values;
  c4  256 molecules of 1-8 waters with 4 densities each in one batched
      build (recorded hipGraph), FP64 and mixed;
  qz8 8 waters in the quadruple-zeta-shaped basis up to g shells, FP64 and
      mixed.
Per build: builds/s and quartets/s from a plain timed loop (no per-kernel
events), then a separate profiled pass (HIP events around every class
kernel) for the per-kernel breakdown and the dominant kernel's roofline.
Errors are taken against the oracle's stored values (tests/golden/, written
by the oracle alone).  The CPU oracle is timed on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import functools
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J/K builds/s + ERI quartets/s, FP64 vs mixed FP32/FP64 at |dE|<=1e-6 Eh"
PEAK_FP64_VECTOR = 78.6   # TFLOP/s, MI355X FP64 vector
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X FP32 vector (published, packed issue)

WORKLOAD_TEXT = {
    "c0": "3 waters, basis A (6-31G*-shaped, Cartesian), 57 AOs, 1 density, cutoff 1e-13",
    "c1": "64 waters 4x4x4 lattice, basis A (6-31G*-shaped, Cartesian), 1216 AOs, 1 density, cutoff 1e-13",
    "c2": "32 waters, basis B (TZ2P-shaped, spherical, up to f), 1376 AOs, 1 density, cutoff 1e-13",
    "qz8": "8 waters, basis C (QZ-shaped, spherical, up to g), 920 AOs, 1 density, cutoff 1e-13",
}
BATCH_TEXT = ("256 molecules of 1-8 waters, half basis A (Cartesian), half basis B (spherical), "
              "4 densities each, cutoff 1e-13")
GOLDEN = os.path.join(ROOT, "tests", "golden")
COUNTERS = {"c1": os.path.join(ROOT, "profiles", "jk_c1_fp64_hbm_counters.txt"),
            "c2": os.path.join(ROOT, "profiles", "jk_c2_fp64_hbm_counters.txt")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def hbm_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by the
    copy-kernel calibration), or (None, reason) when the summary is missing,
    does not cover the kernel, or was taken from other kernel sources."""
    path = COUNTERS.get(workload)
    if not path or not os.path.exists(path):
        return None, "no counter summary for this workload"
    text = open(path).read()
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
    return fetch + write, f"rocprofv3 FETCH_SIZE+WRITE_SIZE per dispatch, {os.path.relpath(path, ROOT)}"


def counter_flops(workload: str, kernel: str):
    """Hardware FP64 FLOP rate of `kernel` and of the whole build from the
    committed rocprofv3 FLOP-counter summary (64 x SQ_INSTS_VALU_FLOPS_FP64
    per dispatch over the traced average duration), or None while the
    summary is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"jk_{workload}_fp64_flop_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel sources sha256[^:]*: ([0-9a-f]+)", text)
    if not m or m.group(1) != source_sha256():
        return None
    whole = re.search(r"counter FP64 FLOP rate ([0-9.]+) TFLOP/s", text)
    kern = None
    for line in text.splitlines():
        f = line.split(None, 5)
        if len(f) == 6 and f"jk::{kernel}(" in f[5]:
            kern = float(f[3])
    return {"kernel_tflops": kern, "build_tflops": float(whole.group(1)) if whole else None,
            "source": os.path.relpath(path, ROOT)}


def golden(name):
    path = os.path.join(GOLDEN, f"{name}_jk.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


STEP_MS = {}  # per-step device times (ms) of the last timed_loop, by id(run)


def timed_loop(run, steps, warmup, torch):
    """Mean seconds per call of run() over `steps` calls after `warmup`,
    bracketed by device synchronisations; nothing else in the loop but an
    event on the stream between calls (for the median and minimum)."""
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        run()
        ev[k + 1].record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    STEP_MS[id(run)] = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    return dt


def step_stats(run):
    """Median and minimum device ms per call of the last timed_loop(run)."""
    v = STEP_MS.get(id(run), [])
    if not v:
        return {}
    return {"ms_median": v[len(v) // 2], "ms_min": v[0]}


def profiled(plan, run, steps, torch):
    """Per-launch HIP-event timings of `steps` builds (a separate pass)."""
    plan.profile(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    tim = plan.timings()
    plan.profile(False)
    return tim


def kernel_name(t):
    """Name of the kernel instantiation a timing entry belongs to (the
    profiler's kernel name without namespace)."""
    prec = "double" if t.precision == 0 else "float"
    cls = f"{t.li}, {t.lj}, {t.lk}, {t.ll}"
    if t.kind in (1, 3):
        return f"jk_k{t.family}_row<{cls}, {prec}, {256 if t.kind == 1 else 64}, false>"
    return f"jk_k{t.family}<{cls}, {prec}, 0>"


def kernel_groups(timings):
    out = {}
    for t in timings:
        g = out.setdefault(kernel_name(t), {"ms": 0.0, "launches": 0, "flops": 0.0, "quartets": 0,
                                            "precision": "fp64" if t.precision == 0 else "fp32"})
        g["ms"] += t.ms
        g["launches"] += t.launches
        g["flops"] += t.model_flops
        g["quartets"] += t.nquartets
    return out


def roofline_of(workload, kern, steps):
    """Dominant kernel (most time) of a profiled pass, against the vector
    peak of its precision."""
    name, k = max(kern.items(), key=lambda kv: kv[1]["ms"])
    peak = PEAK_FP64_VECTOR if k["precision"] == "fp64" else PEAK_FP32_VECTOR
    achieved = k["flops"] / (k["ms"] * 1e-3) / 1e12
    traffic, src = hbm_traffic(workload, name)
    out = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": traffic, "traffic_source": src, "kernel": name, "avg_launch_ms": k["ms"] / k["launches"],
           "launches_per_build": k["launches"] / steps, "model_flops_per_launch": k["flops"] / k["launches"]}
    cf = counter_flops(workload, name) if k["precision"] == "fp64" else None
    if cf:
        # the same kernel's hardware FLOP rate (rocprofv3 counters), and the whole build's
        out["counter_achieved"] = cf["kernel_tflops"]
        out["counter_frac"] = cf["kernel_tflops"] / peak if cf["kernel_tflops"] else None
        out["counter_build_tflops"] = cf["build_tflops"]
        out["counter_source"] = cf["source"]
    return out


def errors_vs_golden(g, D, J, K):
    """max |dJ|, |dK| over the stored elements and dE_J, dE_K (closed-shell
    reading E_J = 2 Tr(DJ), E_K = Tr(DK)) against the oracle's values."""
    import numpy as np
    if g is None:
        return None
    Jh, Kh, Dh = J[0].cpu().numpy(), K[0].cpu().numpy(), D[0]
    ej, ek = 2.0 * float(np.sum(Dh * Jh)), float(np.sum(Dh * Kh))
    return {"max_dJ": float(np.abs(Jh.ravel()[::g["stride"]] - np.asarray(g["J"])).max()),
            "max_dK": float(np.abs(Kh.ravel()[::g["stride"]] - np.asarray(g["K"])).max()),
            "dE_J": ej - g["E_J"], "dE_K": ek - g["E_K"], "E_J": ej, "E_K": ek}


def bench_molecule(name, args, torch, jk, synth, steps, warmup):
    """FP64 and mixed builds of one molecule: timed loop, profiled pass,
    errors against the oracle's stored values."""
    wl = synth.workload(name)
    g = golden(name)
    t0 = time.perf_counter()
    plan = jk.Plan(wl.mol, wl.cutoff)
    st = plan.stats()
    log(f"{name}: {wl.mol.nshell} shells, {wl.mol.nao} AOs; plan {time.perf_counter() - t0:.2f} s, "
        f"{st.nquartets} quartets, {st.nprim_quartets} primitive quartets, {st.nclasses} classes")
    D = torch.from_numpy(wl.D).cuda()
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    psteps = max(1, min(steps, 5))
    # the mixed split threshold: ten times lower with g shells, whose
    # single-precision transfers lose about ten times more digits per quartet
    mix = args.mix_threshold * (0.1 if name == "qz8" else 1.0)
    res = {"workload": f"{name}: {WORKLOAD_TEXT[name]}", "nquartets": st.nquartets,
           "nprim_quartets": st.nprim_quartets, "plan_seconds": time.perf_counter() - t0,
           "model_flops_per_build": st.model_flops, "steps": steps, "warmup": warmup, "mix_threshold": mix}
    for prec in args.precisions.split(","):
        def run():
            plan.execute(D, J, K, precision=prec, mix_threshold=mix)
        dt = timed_loop(run, steps, warmup, torch)
        err = errors_vs_golden(g, wl.D, J, K)
        stp = plan.stats()
        tim = profiled(plan, run, psteps, torch)
        kern = kernel_groups(tim)
        f64 = sum(k["flops"] for k in kern.values() if k["precision"] == "fp64") / psteps
        f32 = sum(k["flops"] for k in kern.values() if k["precision"] == "fp32") / psteps
        ms64 = sum(k["ms"] for k in kern.values() if k["precision"] == "fp64") / psteps
        ms32 = sum(k["ms"] for k in kern.values() if k["precision"] == "fp32") / psteps
        t_bound = f64 / (PEAK_FP64_VECTOR * 1e12) + f32 / (PEAK_FP32_VECTOR * 1e12)
        r = {"ms_per_step": dt * 1e3, **step_stats(run), "builds_per_s": 1.0 / dt, "quartets_per_s": st.nquartets / dt,
             "prim_quartets_per_s": st.nprim_quartets / dt, "model_tflops": st.model_flops / dt / 1e12,
             "frac_of_vector_roofline": t_bound / dt, "fp32_quartets": stp.nquartets_fp32,
             "fp32_fraction": stp.nquartets_fp32 / st.nquartets, "kernel_ms_fp64": ms64, "kernel_ms_fp32": ms32,
             "roofline": roofline_of(name, kern, psteps), "vs_oracle": err}
        top = sorted(kern.items(), key=lambda kv: -kv[1]["ms"])[:args.top]
        r["top_kernels"] = [{"kernel": n, "ms_per_build": k["ms"] / psteps,
                             "tflops": k["flops"] / (k["ms"] * 1e-3) / 1e12 if k["ms"] > 0 else 0.0}
                            for n, k in top]
        ev = (f"vs oracle max|dJ| {err['max_dJ']:.1e} max|dK| {err['max_dK']:.1e} dE_J {err['dE_J']:.1e} "
              f"dE_K {err['dE_K']:.1e}") if err else "no stored oracle values"
        log(f"{name} {prec}: {dt * 1e3:.2f} ms/build, {st.nquartets / dt:.3e} quartets/s, fp32 fraction "
            f"{r['fp32_fraction']:.3f}; kernels fp64 {ms64:.1f} ms fp32 {ms32:.1f} ms; {ev}")
        for n, k in top:
            log(f"  {n:46s} {k['ms'] / psteps:8.3f} ms/build  {k['launches'] / psteps:4.0f} launches  "
                f"{k['flops'] / (k['ms'] * 1e-3) / 1e12 if k['ms'] > 0 else 0:6.2f} TF/s")
        res[prec] = r
    if "fp64" in res and "mixed" in res:
        res["mixed"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    if name in ("c1", "c2") and "fp64" in res and not args.no_deterministic:
        res["deterministic"] = bench_deterministic(torch, jk, plan, D, g, wl, res["fp64"]["ms_per_step"] * 1e-3,
                                                   min(steps, 3), 1)
    if name == "c1" and not args.no_dscreen:
        res["density_screening"] = bench_dscreen(args, torch, plan, wl, res["fp64"]["ms_per_step"] * 1e-3, steps,
                                                 warmup)
    plan.close()
    return res


def bench_batch(args, torch, jk, synth, steps, warmup):
    """Batched builds over the 256-molecule set (one graph replay per step),
    FP64 and mixed, against the oracle's stored per-molecule values, and the
    same molecules built one jk_execute at a time."""
    import numpy as np
    wls = synth.batch_workload()
    g = golden("c4")
    t0 = time.perf_counter()
    plans = [jk.Plan(w.mol, w.cutoff) for w in wls]
    t_plan = time.perf_counter() - t0
    Ds = [torch.from_numpy(w.D).cuda() for w in wls]
    Js = [torch.empty_like(D) for D in Ds]
    Ks = [torch.empty_like(D) for D in Ds]
    nset = Ds[0].shape[0]
    nq = sum(p.stats().nquartets for p in plans)
    res = {"workload": f"c4: {BATCH_TEXT}", "nmol": len(wls), "nset": nset, "plan_seconds": t_plan,
           "nquartets": nq, "steps": steps, "warmup": warmup}
    log(f"c4: {len(wls)} plans in {t_plan:.1f} s, {nq} quartets")

    def errors():
        dj = dk = de = 0.0
        for w, J, K, gm in zip(wls, Js, Ks, g["molecules"]):
            Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
            dj = max(dj, float(np.abs(Jh.ravel()[::g["stride"]] - np.asarray(gm["J"])).max()))
            dk = max(dk, float(np.abs(Kh.ravel()[::g["stride"]] - np.asarray(gm["K"])).max()))
            ej = 2.0 * np.einsum("sij,sij->s", w.D, Jh)
            ek = np.einsum("sij,sij->s", w.D, Kh)
            de = max(de, float(np.abs(ej - np.asarray(gm["E_J"])).max()), float(np.abs(ek - np.asarray(gm["E_K"])).max()))
        return {"max_dJ": dj, "max_dK": dk, "max_dE": de}

    for precision in args.precisions.split(","):
        b = jk.Batch(plans, nset=nset, precision=precision, mix_threshold=args.mix_threshold)
        def run():
            b.execute(Ds, Js, Ks)
        dt = timed_loop(run, steps, warmup, torch)
        nev, n32 = b.stats()
        err = errors()
        res[precision] = {"ms_per_step": dt * 1e3, **step_stats(run), "molecule_builds_per_s": len(wls) / dt,
                          "density_builds_per_s": len(wls) * nset / dt, "quartets_per_s": nq / dt,
                          "fp32_quartets": n32, "fp32_fraction": n32 / max(nev, 1), "vs_oracle": err}
        log(f"c4 {precision}: {dt * 1e3:.1f} ms per batch ({len(wls) / dt:.0f} molecule builds/s), fp32 fraction "
            f"{n32 / max(nev, 1):.3f}, vs oracle max|dJ| {err['max_dJ']:.1e} max|dK| {err['max_dK']:.1e} "
            f"max|dE| {err['max_dE']:.1e}")
        b.close()
        # the same molecules one jk_execute each (one warm-up pass, one timed)
        def one_by_one():
            for p, D, J, K in zip(plans, Ds, Js, Ks):
                p.execute(D, J, K, precision=precision, mix_threshold=args.mix_threshold)
        dts = timed_loop(one_by_one, 1, 1, torch)
        res[precision]["one_by_one_ms"] = dts * 1e3
        res[precision]["speedup_vs_one_by_one"] = dts / dt
        log(f"c4 {precision}: one by one {dts * 1e3:.1f} ms")
    if "fp64" in res and "mixed" in res:
        res["mixed"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    for p in plans:
        p.close()
    return res


def bench_deterministic(torch, jk, plan, D, g, wl, dt_full, steps, warmup):
    """The fixed-order FP64 build (JK_DETERMINISTIC): its time against the
    default build, whether two builds agree bit for bit, and its error
    against the oracle's stored values."""
    import numpy as np
    flags = jk.JK_DO_J | jk.JK_DO_K | jk.JK_DETERMINISTIC
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    dt = timed_loop(lambda: plan.execute(D, J, K, flags=flags), steps, warmup, torch)
    J1, K1 = J.cpu().numpy(), K.cpu().numpy()
    plan.execute(D, J, K, flags=flags)
    torch.cuda.synchronize()
    same = bool(np.array_equal(J1, J.cpu().numpy()) and np.array_equal(K1, K.cpu().numpy()))
    err = errors_vs_golden(g, wl.D, J, K)
    log(f"deterministic fp64: {dt * 1e3:.2f} ms/build ({dt / dt_full:.2f} x the default build), "
        f"bitwise repeatable {same}" + (f", max|dJ| {err['max_dJ']:.1e} max|dK| {err['max_dK']:.1e}" if err else ""))
    return {"ms_per_step": dt * 1e3, "vs_default_build": dt / dt_full, "bitwise_repeatable": same, "vs_oracle": err}


def bench_dscreen(args, torch, plan, wl, dt_full, steps, warmup):
    """Incremental build as in a late direct-SCF iteration: the density
    change dD = 1e-4 * (a fresh seeded density - D) with density screening
    at --dscreen; its time against the full build, and its error against
    the same dD built unscreened."""
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
    dt = timed_loop(lambda: plan.execute(dD, J, K), steps, warmup, torch)
    st = plan.stats()
    plan.set_density_screening(0.0)
    err_j = float(np.abs(J.cpu().numpy() - J0).max())
    err_k = float(np.abs(K.cpu().numpy() - K0).max())
    log(f"c1 incremental (dD ~ 1e-4, dscreen {args.dscreen:g}): {dt * 1e3:.2f} ms/build, "
        f"{st.nquartets_evaluated} of {st.nquartets} quartets, max|dJ| {err_j:.1e} max|dK| {err_k:.1e} vs unscreened")
    return {"threshold": args.dscreen, "delta_D": "1e-4 * (seeded density - D)", "ms_per_step": dt * 1e3,
            "builds_per_s": 1.0 / dt, "speedup_vs_full_build": dt_full / dt,
            "quartets_evaluated": st.nquartets_evaluated,
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
            row[prec + "_ms"] = 1e3 * timed_loop(lambda: plan.execute(D, J, K, precision=prec), args.steps,
                                                 args.warmup, torch)
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
            dt = timed_loop(lambda: plan.execute(D, J, K), args.steps, args.warmup, torch)
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
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / full_s, "unit": "builds/s", "cores": orc.num_threads(), "kind": "oracle",
            "host_cpus": os.cpu_count(), "host_cpu_model": model,
            "sample": f"c1 eight-fold oracle over {used} random bra shell pairs of {npair} (each with all its "
                      f"canonical kets), {spent:.1f} s, scaled by {npair}/{used} to one build "
                      f"({full_s:.0f} s per build)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps of the headline (c1) builds")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--configs", default="c1,c2,c4,qz8", help="comma list of c1, c2, c4, qz8 (c1 is always run)")
    ap.add_argument("--steps-other", type=int, default=5, help="most timed steps of c2 and c4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=sorted(WORKLOAD_TEXT) + ["c4"], default=None,
                    help="time one molecule alone and print its result (for profiler runs)")
    ap.add_argument("--precisions", default="fp64,mixed",
                    help="builds timed per molecule (fp64 is needed for the headline value)")
    ap.add_argument("--no-dscreen", action="store_true", help="skip the incremental (density-screened) build")
    ap.add_argument("--no-deterministic", action="store_true", help="skip the fixed-order (JK_DETERMINISTIC) builds")
    ap.add_argument("--micro", action="store_true", help="only the appendix-B style micro-benchmarks")
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
    which = [c.strip() for c in args.configs.split(",") if c.strip()]
    so, wo = max(1, min(args.steps, args.steps_other)), max(1, min(args.warmup, 2))

    if args.only:
        # one molecule alone (the profiler runs): its result, not the headline line
        f = bench_batch if args.only == "c4" else functools.partial(bench_molecule, args.only)
        print(json.dumps({args.only: f(args, torch, jk, synth, args.steps, args.warmup)}), flush=True)
        return
    c1 = bench_molecule("c1", args, torch, jk, synth, args.steps, args.warmup)
    r64 = c1["fp64"]
    out = {"metric": METRIC, "value": r64["builds_per_s"], "unit": "builds/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded water lattice, random orthonormal C)",
           "config": {"workload": c1["workload"], "nset": 1, "precision": "fp64", "cutoff": 1e-13},
           "quartets_per_s": r64["quartets_per_s"], "prim_quartets_per_s": r64["prim_quartets_per_s"],
           "nquartets": c1["nquartets"], "model_tflops": r64["model_tflops"],
           "model_frac_fp64_peak": r64["frac_of_vector_roofline"], "roofline": r64["roofline"],
           "configs": {"c1": c1}}
    if "c2" in which:
        out["configs"]["c2"] = bench_molecule("c2", args, torch, jk, synth, so, wo)
    # config 3: the mixed split on the c1 and c2 molecules
    c3 = {}
    for n in ("c1", "c2"):
        if n in out["configs"] and "mixed" in out["configs"][n]:
            m = out["configs"][n]["mixed"]
            c3[n] = {"fp32_fraction": m["fp32_fraction"], "speedup_vs_fp64": m["speedup_vs_fp64"],
                     "builds_per_s": m["builds_per_s"], "quartets_per_s": m["quartets_per_s"],
                     "frac_of_vector_roofline": m["frac_of_vector_roofline"],
                     "vs_oracle": m["vs_oracle"],
                     "threshold": args.mix_threshold}
    out["configs"]["c3"] = c3
    if "c4" in which:
        out["configs"]["c4"] = bench_batch(args, torch, jk, synth, so, wo)
    if "qz8" in which:
        out["configs"]["qz8"] = bench_molecule("qz8", args, torch, jk, synth, so, wo)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(synth.workload("c1"), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
