"""Full-size parity against stored oracle values (tests/golden/*_jk.json,
written by tests/golden/make_golden.py from the CPU oracle alone).

FP64: every stored element (every 97th of J and K) within 1e-10, energies
E_J = 2 Tr(DJ) and E_K = Tr(DK) within 1e-8 Eh, and the same number of
significant unique quartets.  Mixed FP32/FP64 (threshold 1e-4 on
Q_IJ Q_KL max|D_block|): |dE_J|, |dE_K| <= 1e-6 Eh.  With g shells (the
QZ-shaped workload) the single-precision transfers lose about ten times more
digits per quartet (up to 2e-4 relative against 2e-5 without g), so the
split is taken at 1e-5 there to hold the same energy bar.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2507_09772_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    with open(os.path.join(HERE, "golden", f"{name}_jk.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def torch_jk():
    import torch

    from paper_2507_09772_amd import jk
    assert torch.cuda.is_available()
    return torch, jk


MIX_THRESHOLD = {"c1": 1e-4, "c2": 1e-4, "qz8": 1e-5}


@pytest.mark.parametrize("name", ["c1", "c2", "qz8"])
def test_full_size_against_golden(torch_jk, name):
    torch, jk = torch_jk
    g = golden(name)
    wl = synth.workload(name)
    print("golden", name, flush=True)
    plan = jk.Plan(wl.mol, wl.cutoff)
    assert plan.stats().nquartets == g["nsig"]
    D = torch.from_numpy(wl.D).cuda()
    Dh = wl.D[0]
    for precision in ("fp64", "mixed"):
        J, K = plan.execute(D, precision=precision, mix_threshold=MIX_THRESHOLD[name])
        torch.cuda.synchronize()
        Jh, Kh = J[0].cpu().numpy(), K[0].cpu().numpy()
        ej, ek = 2.0 * float(np.sum(Dh * Jh)), float(np.sum(Dh * Kh))
        dj = np.abs(Jh.ravel()[::g["stride"]] - np.asarray(g["J"])).max()
        dk = np.abs(Kh.ravel()[::g["stride"]] - np.asarray(g["K"])).max()
        print(f"{name} {precision}: max|dJ| {dj:.2e} max|dK| {dk:.2e} dE_J {ej - g['E_J']:.2e} "
              f"dE_K {ek - g['E_K']:.2e}", flush=True)
        if precision == "fp64":
            assert dj <= 1e-10 and dk <= 1e-10
            assert abs(ej - g["E_J"]) <= 1e-8 and abs(ek - g["E_K"]) <= 1e-8
        else:
            assert abs(ej - g["E_J"]) <= 1e-6 and abs(ek - g["E_K"]) <= 1e-6
