"""JK_DETERMINISTIC: the fixed-order build against the oracle, and bitwise
equal J and K across repeated builds, stream counts, plans and profiling;
the no-allocation entry point refuses the flag."""
import ctypes
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
    saved = os.environ.get("JK_STREAMS")
    try:
        os.environ["JK_STREAMS"] = str(n)
        return jkmod.Plan(wl.mol, wl.cutoff)
    finally:
        if saved is None:
            os.environ.pop("JK_STREAMS", None)
        else:
            os.environ["JK_STREAMS"] = saved


def det_build(jkmod, torch, plan, D, precision="fp64", extra=0, J=None, K=None):
    flags = jkmod.JK_DO_J | jkmod.JK_DO_K | jkmod.JK_DETERMINISTIC | extra
    J, K = plan.execute(D, J, K, precision=precision, mix_threshold=1e-5, flags=flags)
    torch.cuda.synchronize()
    return J.cpu().numpy(), K.cpu().numpy()


@pytest.mark.parametrize("basis,nw,nset", [("A", 5, 1), ("B", 3, 2), ("C", 1, 1)])
def test_deterministic_vs_oracle(jkmod, torch_cuda, basis, nw, nset):
    wl = synth.small_workload(nw, basis, seed=90 + nw, nset=nset)
    say("deterministic vs oracle", basis, nw, nset)
    J0, K0, _ = o.jk(wl.mol, wl.D, wl.cutoff, mode=1)
    plan = jkmod.Plan(wl.mol, wl.cutoff)
    D = torch_cuda.from_numpy(wl.D).cuda()
    J, K = det_build(jkmod, torch_cuda, plan, D)
    assert np.abs(J - J0).max() <= TOL and np.abs(K - K0).max() <= TOL
    # mixed precision in the fixed-order mode: within the split's error
    ej0, ek0 = o.energies(wl.D, J0, K0)
    Jm, Km = det_build(jkmod, torch_cuda, plan, D, precision="mixed")
    ej, ek = o.energies(wl.D, Jm, Km)
    assert np.abs(ej - ej0).max() <= 1e-6 and np.abs(ek - ek0).max() <= 1e-6
    plan.close()


def test_deterministic_bitwise(jkmod, torch_cuda):
    """Every build of the same inputs gives the same bits: repeated builds,
    one and eight streams, a second plan, profiled builds, and mixed
    precision; the default (atomic-order) build differs from it only by
    rounding."""
    torch = torch_cuda
    wl = synth.small_workload(6, "B", seed=97, nset=2)
    D = torch.from_numpy(wl.D).cuda()
    say("deterministic bitwise")
    p1 = plan_with_streams(jkmod, wl, 1)
    p8 = plan_with_streams(jkmod, wl, 8)
    for prec in ("fp64", "mixed"):
        ref = det_build(jkmod, torch, p8, D, prec)
        runs = [det_build(jkmod, torch, p8, D, prec) for _ in range(3)]
        runs.append(det_build(jkmod, torch, p1, D, prec))
        p8.profile(True)
        runs.append(det_build(jkmod, torch, p8, D, prec))
        p8.profile(False)
        for k, (J, K) in enumerate(runs):
            assert np.array_equal(J, ref[0]) and np.array_equal(K, ref[1]), (prec, k)
        # the default build sums in another order (row kernels, atomics):
        # FP64 elements up to about 10 from about 1e5 additions each differ
        # by rounding (1e-11); in mixed builds the single-precision quartets
        # of the row and tile kernels round differently (1e-9, as between
        # batched and single mixed builds)
        Jd, Kd = p8.execute(D, precision=prec, mix_threshold=1e-5)
        torch.cuda.synchronize()
        tol = 1e-11 if prec == "fp64" else 1e-9
        assert np.abs(Jd.cpu().numpy() - ref[0]).max() <= tol, prec
        assert np.abs(Kd.cpu().numpy() - ref[1]).max() <= tol, prec
    p1.close()
    p8.close()


def test_deterministic_accumulate(jkmod, torch_cuda):
    torch = torch_cuda
    wl = synth.small_workload(3, "A", seed=98, nset=1)
    D = torch.from_numpy(wl.D).cuda()
    plan = jkmod.Plan(wl.mol, wl.cutoff)
    say("deterministic accumulate")
    J1, K1 = det_build(jkmod, torch, plan, D)
    J = torch.from_numpy(J1).cuda()
    K = torch.from_numpy(K1).cuda()
    J2, K2 = det_build(jkmod, torch, plan, D, extra=jkmod.JK_ACCUMULATE, J=J, K=K)
    assert np.array_equal(J2, J1 + J1) and np.array_equal(K2, K1 + K1)
    plan.close()


def test_noalloc_refuses_deterministic(jkmod, torch_cuda):
    torch = torch_cuda
    L = jkmod.lib()
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.jk_execute_noalloc.argtypes = [vp, vp, i32, i32, i32, f64, f64, vp, vp, vp]
    wl = synth.small_workload(1, "A", seed=99, nset=1)
    plan = jkmod.Plan(wl.mol, wl.cutoff)
    D = torch.from_numpy(wl.D).cuda()
    J = torch.zeros_like(D)
    K = torch.zeros_like(D)
    flags = jkmod.JK_DO_J | jkmod.JK_DO_K | jkmod.JK_DETERMINISTIC
    rc = L.jk_execute_noalloc(plan.h, ctypes.c_void_p(D.data_ptr()), 1, flags, 0, 1e-4, 0.0,
                              ctypes.c_void_p(J.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == -1  # JK_EINVAL
    assert float(J.abs().max()) == 0.0
    plan.close()
