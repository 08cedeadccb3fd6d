"""Batched builds (jk_batch_*): many molecules in one recorded hipGraph.

Each molecule's J and K from the batch must equal the single-molecule
build (jk_execute, same kernels in another launch shape) to atomic-order
rounding, and the CPU oracle within 1e-10 (FP64).  The graph is replayed
several times with eager work and synchronisations in between, every
replay checked.  At the full 256-molecule size the stored oracle values
(tests/golden/c4_jk.json) are checked for every molecule.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as o
from paper_2507_09772_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2507_09772_amd import jk
    assert torch.cuda.is_available()
    return torch, jk


def _setup(torch, jk, wls):
    plans = [jk.Plan(w.mol, w.cutoff) for w in wls]
    Ds = [torch.from_numpy(w.D).cuda() for w in wls]
    return plans, Ds


def _singles(torch, plans, Ds, precision):
    out = [p.execute(D, precision=precision) for p, D in zip(plans, Ds)]
    torch.cuda.synchronize()
    return [(J.cpu().numpy(), K.cpu().numpy()) for J, K in out]


# Single precision: the batch runs the short bras of a class as 64-lane row
# tasks where the single build runs tiles of another family, and the FP32
# rounding of one quartet's elements differs between kernels by ~1e-7
# relative.  Mixed: FP32 quartets have bounds below 1e-4, so an element of J
# or K built from many of them differs by up to ~1e-10 between the two;
# all-FP32: elements of order one differ by up to ~1e-8.
MIXED_TOL = 1e-9
FP32_TOL = 1e-7


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", MIXED_TOL), ("fp32", FP32_TOL)])
def test_batch_matches_single_and_replays(env, precision, tol):
    torch, jk = env
    wls = synth.batch_workload(nmol=24, nset=2, seed=11)
    say("batch", precision, [w.mol.nwater for w in wls])
    plans, Ds = _setup(torch, jk, wls)
    ref = _singles(torch, plans, Ds, precision)
    b = jk.Batch(plans, nset=2, precision=precision)
    Js = [torch.full_like(D, np.nan) for D in Ds]
    Ks = [torch.full_like(D, np.nan) for D in Ds]
    for rep in range(3):
        b.execute(Ds, Js, Ks)
        torch.cuda.synchronize()
        for m, (J, K) in enumerate(zip(Js, Ks)):
            dj = np.abs(J.cpu().numpy() - ref[m][0]).max()
            dk = np.abs(K.cpu().numpy() - ref[m][1]).max()
            assert dj <= tol and dk <= tol, (rep, m, dj, dk)
        # eager work between replays
        _singles(torch, plans[:3], Ds[:3], "fp64")
    if precision == "fp64":
        for m, w in enumerate(wls):
            if w.mol.nwater > 3:
                continue
            J0, K0, _ = o.jk(w.mol, w.D, w.cutoff, mode=1)
            assert np.abs(Js[m].cpu().numpy() - J0).max() <= 1e-10, m
            assert np.abs(Ks[m].cpu().numpy() - K0).max() <= 1e-10, m
    b.close()


@pytest.mark.parametrize("fam,persist,branches", [(1, "0", "4"), (1, "1", "4"), (1, "1", "1"), (2, "0", "1")])
def test_batch_row_tasks(env, fam, persist, branches):
    """Every class forced to row mode on all bras (the batch then runs row
    tasks instead of tiles) and to one family, FP64 and mixed, against the
    single-molecule builds and the oracle; with family 1 also in the
    persistent form (one work queue for the one- and two-root classes) and
    on one or four graph branches."""
    torch, jk = env
    wls = synth.batch_workload(nmol=12, nset=2, seed=13)
    say("batch rows", fam, persist, branches, [w.mol.nwater for w in wls])
    saved = {k: os.environ.get(k) for k in ("JK_BATCH_PERSIST", "JK_BATCH_BRANCHES")}
    os.environ["JK_BATCH_PERSIST"] = persist
    os.environ["JK_BATCH_BRANCHES"] = branches
    try:
        for c in jk.canonical_classes():
            for p in ("fp64", "fp32"):
                _, avail = jk.tune_get(*c, p)
                jk.tune_set(*c, p, fam if avail & fam else 0)
                jk.tune_set_row(*c, p, 3)
        plans, Ds = _setup(torch, jk, wls)
        for precision, tol in (("fp64", 1e-12), ("mixed", MIXED_TOL)):
            ref = _singles(torch, plans, Ds, precision)
            b = jk.Batch(plans, nset=2, precision=precision)
            Js = [torch.full_like(D, np.nan) for D in Ds]
            Ks = [torch.full_like(D, np.nan) for D in Ds]
            for rep in range(2):
                b.execute(Ds, Js, Ks)
                torch.cuda.synchronize()
                for m in range(len(wls)):
                    assert np.abs(Js[m].cpu().numpy() - ref[m][0]).max() <= tol, (precision, rep, m)
                    assert np.abs(Ks[m].cpu().numpy() - ref[m][1]).max() <= tol, (precision, rep, m)
            b.close()
        for m, w in enumerate(wls):
            if w.mol.nwater <= 2:
                J0, K0, _ = o.jk(w.mol, w.D, w.cutoff, mode=1)
                assert np.abs(ref[m][0] - J0).max() <= 1e-6  # mixed reference vs FP64 oracle
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        for c in jk.canonical_classes():
            for p in ("fp64", "fp32"):
                jk.tune_set(*c, p, 0)
                jk.tune_set_row(*c, p, 0)
        jk.tune_load(os.path.join(os.path.dirname(jk.__file__), "tune_gfx950.txt"))


def test_batch_pointer_change(env):
    torch, jk = env
    wls = synth.batch_workload(nmol=6, nset=1, seed=12)
    plans, Ds = _setup(torch, jk, wls)
    ref = _singles(torch, plans, Ds, "fp64")
    b = jk.Batch(plans, nset=1)
    Js = [torch.zeros_like(D) for D in Ds]
    Ks = [torch.zeros_like(D) for D in Ds]
    b.execute(Ds, Js, Ks)
    # new outputs and a new (scaled) density for every molecule
    D2 = [2.0 * D for D in Ds]
    J2 = [torch.zeros_like(D) for D in Ds]
    K2 = [torch.zeros_like(D) for D in Ds]
    b.execute(D2, J2, K2)
    torch.cuda.synchronize()
    for m in range(len(wls)):
        assert np.abs(Js[m].cpu().numpy() - ref[m][0]).max() <= 1e-12
        assert np.abs(J2[m].cpu().numpy() - 2 * ref[m][0]).max() <= 1e-12
        assert np.abs(K2[m].cpu().numpy() - 2 * ref[m][1]).max() <= 1e-12
    with pytest.raises(ValueError):
        b.execute(Ds[:-1], Js[:-1], Ks[:-1])


@pytest.mark.skipif(not os.path.exists(os.path.join(HERE, "golden", "c4_jk.json")), reason="no stored c4 values")
def test_batch_full_size_golden(env):
    torch, jk = env
    with open(os.path.join(HERE, "golden", "c4_jk.json")) as f:
        g = json.load(f)
    wls = synth.batch_workload()
    assert len(wls) == len(g["molecules"])
    say("batch full", len(wls))
    plans, Ds = _setup(torch, jk, wls)
    for m, (p, gm) in enumerate(zip(plans, g["molecules"])):
        assert p.stats().nquartets == gm["nsig"], m
    Js = [torch.empty_like(D) for D in Ds]
    Ks = [torch.empty_like(D) for D in Ds]
    st = g["stride"]
    for precision in ("fp64", "mixed"):
        b = jk.Batch(plans, nset=Ds[0].shape[0], precision=precision)
        b.execute(Ds, Js, Ks)
        torch.cuda.synchronize()
        worst = [0.0, 0.0, 0.0]
        for m, (w, gm) in enumerate(zip(wls, g["molecules"])):
            J, K = Js[m].cpu().numpy(), Ks[m].cpu().numpy()
            ej, ek = o.energies(w.D, J, K)
            de = max(np.abs(ej - gm["E_J"]).max(), np.abs(ek - gm["E_K"]).max())
            dj = np.abs(J.ravel()[::st] - np.asarray(gm["J"])).max()
            dk = np.abs(K.ravel()[::st] - np.asarray(gm["K"])).max()
            worst = [max(worst[0], dj), max(worst[1], dk), max(worst[2], de)]
            if precision == "fp64":
                assert dj <= 1e-10 and dk <= 1e-10 and de <= 1e-8, (m, dj, dk, de)
            else:
                assert de <= 1e-6, (m, de)
        say(precision, "max|dJ| %.2e max|dK| %.2e max|dE| %.2e" % tuple(worst))
        b.close()
