"""jk_execute_noalloc (scratch in the library's fixed per-GPU array, no
allocation) against jk_execute on the same inputs, through the C ABI: two
calls in a row, the second with a smaller input, FP64 to 1e-13 (both run the
same kernels; only the order of atomic additions differs) and mixed, plus the
size limit."""
import ctypes

import numpy as np
import pytest

from paper_2507_09772_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_09772_amd import jk
    L = jk.lib()
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.jk_execute_noalloc.argtypes = [vp, vp, i32, i32, i32, f64, f64, vp, vp, vp]
    return torch, jk, L


def noalloc(env, plan, D, precision="fp64", flags=None):
    torch, jk, L = env
    J = torch.full_like(D, float("nan"))
    K = torch.full_like(D, float("nan"))
    flags = jk.JK_DO_J | jk.JK_DO_K if flags is None else flags
    rc = L.jk_execute_noalloc(plan.h, ctypes.c_void_p(D.data_ptr()), D.shape[0], flags, jk.PRECISION[precision],
                              1e-4, 0.0, ctypes.c_void_p(J.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, J, K


def test_noalloc_matches_execute_twice(env):
    torch, jk, L = env
    cases = [synth.small_workload(4, "B", seed=301, nset=2), synth.small_workload(2, "A", seed=302, nset=1)]
    for wl in cases:  # the second call has the smaller input
        print("noalloc", wl.mol.nao, wl.D.shape[0], flush=True)
        plan = jk.Plan(wl.mol, wl.cutoff)
        D = torch.from_numpy(wl.D).cuda()
        for prec in ("fp64", "mixed"):
            J0, K0 = plan.execute(D, precision=prec)
            torch.cuda.synchronize()
            n0 = plan.stats().nquartets_fp32
            rc, J, K = noalloc(env, plan, D, prec)
            assert rc == 0, jk.lib().jk_last_error().decode()
            dj = float((J - J0).abs().max())
            dk = float((K - K0).abs().max())
            assert dj <= 1e-13 and dk <= 1e-13, (prec, dj, dk)
            assert plan.stats().nquartets_fp32 == n0
        plan.close()


def test_noalloc_rejects_oversized_build(env):
    torch, jk, L = env
    wl = synth.small_workload(2, "A", seed=303, nset=1)
    plan = jk.Plan(wl.mol, wl.cutoff)
    # enough densities that the Cartesian J' and K' alone exceed the array
    nset = (128 << 20) // (8 * plan.nao_cart * plan.nao_cart * 2) + 1
    D = torch.zeros((nset, plan.nao, plan.nao), dtype=torch.float64, device="cuda")
    rc, _, _ = noalloc(env, plan, D)
    assert rc == jk.JK_EINVAL and "scratch" in jk.lib().jk_last_error().decode()
