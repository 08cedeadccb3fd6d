"""Class kernels of one build spread over several streams: results for every
stream count against the oracle, and a build captured into a graph (the
fork and join of the plan's streams inside the capture) replayed several
times against eager builds."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as o
from paper_2507_09772_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def jkmod(torch_cuda):
    from paper_2507_09772_amd import jk
    jk.lib()
    return jk


def plan_with_streams(jkmod, wl, n):
    """A plan created with JK_STREAMS=n (None: the library default)."""
    saved = os.environ.get("JK_STREAMS")
    try:
        if n is None:
            os.environ.pop("JK_STREAMS", None)
        else:
            os.environ["JK_STREAMS"] = str(n)
        return jkmod.Plan(wl.mol, wl.cutoff)
    finally:
        if saved is None:
            os.environ.pop("JK_STREAMS", None)
        else:
            os.environ["JK_STREAMS"] = saved


@pytest.mark.parametrize("basis,nw", [("B", 4), ("C", 1)])
def test_stream_counts(jkmod, torch_cuda, basis, nw):
    wl = synth.small_workload(nw, basis, seed=71 + nw, nset=2)
    J0, K0, _ = o.jk(wl.mol, wl.D, wl.cutoff, mode=1)
    D = torch_cuda.from_numpy(wl.D).cuda()
    for n in (1, 2, None, 8):
        say("streams", basis, nw, n)
        plan = plan_with_streams(jkmod, wl, n)
        for prec in ("fp64", "mixed"):
            J, K = plan.execute(D, precision=prec, mix_threshold=1e-5)
            torch_cuda.cuda.synchronize()
            J, K = J.cpu().numpy(), K.cpu().numpy()
            if prec == "fp64":
                assert np.abs(J - J0).max() <= TOL and np.abs(K - K0).max() <= TOL, (n, prec)
            else:
                assert np.abs(J - J0).max() <= 1e-6 and np.abs(K - K0).max() <= 1e-6, (n, prec)
        plan.close()


def test_graph_capture(jkmod, torch_cuda):
    torch = torch_cuda
    wl = synth.small_workload(4, "B", seed=81, nset=1)
    D2 = synth.random_density(wl.mol.nao, synth.OCC_PER_WATER * 4, 83, 1)  # another density, same geometry
    say("graph capture")
    plan = plan_with_streams(jkmod, wl, 4)
    D = torch.from_numpy(wl.D).cuda()
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    plan.execute(D, J, K)  # allocates the plan's scratch before the capture
    torch.cuda.synchronize()
    refs = []
    for Dh in (wl.D, D2):
        Je, Ke = plan.execute(torch.from_numpy(Dh).cuda())
        torch.cuda.synchronize()
        refs.append((Je.cpu().numpy(), Ke.cpu().numpy()))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(D, J, K)
    torch.cuda.synchronize()
    for rep in range(4):
        which = rep % 2
        D.copy_(torch.from_numpy((wl.D, D2)[which]).cuda())
        J.fill_(7.0)
        K.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        Jr, Kr = refs[which]
        dj = np.abs(J.cpu().numpy() - Jr).max()
        dk = np.abs(K.cpu().numpy() - Kr).max()
        say("replay", rep, dj, dk)
        assert dj <= 1e-12 and dk <= 1e-12, (rep, dj, dk)
        # eager work on the same plan between replays
        Je, Ke = plan.execute(torch.from_numpy(D2).cuda())
        torch.cuda.synchronize()
        assert np.abs(Je.cpu().numpy() - refs[1][0]).max() <= 1e-12
    g.reset()
    plan.close()
