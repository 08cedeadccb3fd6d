"""ctypes binding of libjk.so (include/jk.h).

Argument marshalling only: every step of the J/K build runs in the HIP
library.  Torch supplies device memory and the current stream.  Importing
this module fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjk.so")

JK_OK, JK_EINVAL, JK_EUNSUPPORTED, JK_ENOMEM, JK_EDEVICE = 0, -1, -2, -3, -4
JK_FP64, JK_MIXED, JK_FP32 = 0, 1, 2
JK_DO_J, JK_DO_K, JK_ACCUMULATE, JK_CHECK_SYMMETRY, JK_DETERMINISTIC = 1, 2, 4, 8, 16
PRECISION = {"fp64": JK_FP64, "mixed": JK_MIXED, "fp32": JK_FP32}


class JKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jk error {code}: {msg}")
        self.code = code


class _Basis(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int32), ("natom", ctypes.c_int32), ("spherical", ctypes.c_int32),
                ("l", ctypes.c_void_p), ("nprim", ctypes.c_void_p), ("atom", ctypes.c_void_p),
                ("exps", ctypes.c_void_p), ("coefs", ctypes.c_void_p), ("coords", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("nquartets", ctypes.c_int64), ("nprim_quartets", ctypes.c_int64),
                ("nquartets_fp32", ctypes.c_int64), ("nclasses", ctypes.c_int32),
                ("npairs", ctypes.c_int32), ("setup_ms", ctypes.c_double), ("model_flops", ctypes.c_double),
                ("nquartets_evaluated", ctypes.c_int64)]


class ClassTiming(ctypes.Structure):
    _fields_ = [("li", ctypes.c_int32), ("lj", ctypes.c_int32), ("lk", ctypes.c_int32), ("ll", ctypes.c_int32),
                ("npb", ctypes.c_int32), ("npk", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("family", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("nquartets", ctypes.c_int64), ("model_flops", ctypes.c_double), ("ms", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.jk_plan_create.argtypes = [ctypes.POINTER(_Basis), f64, ctypes.POINTER(vp)]
        L.jk_plan_destroy.argtypes = [vp]
        L.jk_plan_destroy.restype = None
        L.jk_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.jk_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.jk_plan_schwarz.argtypes = [vp, vp]
        L.jk_execute.argtypes = [vp, vp, i32, i32, i32, f64, f64, vp, vp, vp]
        L.jk_build.argtypes = [ctypes.POINTER(_Basis), vp, i32, f64, i32, vp, vp, vp]
        L.jk_eri_block.argtypes = [vp, i32, i32, i32, i32, i32, vp]
        L.jk_rys_eval.argtypes = [i32, vp, i32, i32, vp, vp]
        L.jk_boys_eval.argtypes = [i32, vp, i32, i32, vp]
        L.jk_batch_create.argtypes = [vp, i32, i32, i32, f64, ctypes.POINTER(vp)]
        L.jk_batch_execute.argtypes = [vp, vp, vp, vp, vp]
        L.jk_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.jk_batch_destroy.argtypes = [vp]
        L.jk_batch_destroy.restype = None
        L.jk_plan_profile.argtypes = [vp, i32]
        L.jk_plan_set_density_screening.argtypes = [vp, f64]
        L.jk_plan_timings.argtypes = [vp, ctypes.POINTER(ClassTiming), i32, ctypes.POINTER(i32)]
        L.jk_tune_set.argtypes = [i32, i32, i32, i32, i32, i32]
        L.jk_tune_get.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.jk_tune_load.argtypes = [ctypes.c_char_p]
        L.jk_tune_set_row.argtypes = [i32, i32, i32, i32, i32, i32]
        L.jk_tune_set_shape.argtypes = [i32, i32, i32, i32, i32, i32]
        L.jk_tune_set_split.argtypes = [i32, i32, i32, i32, i32]
        L.jk_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise JKError(rc, lib().jk_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class BasisArrays:
    """Contiguous copies of a molecule's basis arrays and the jk_basis view."""

    def __init__(self, mol):
        self.l = np.ascontiguousarray(mol.l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(mol.nprim, dtype=np.int32)
        self.atom = np.ascontiguousarray(mol.atom, dtype=np.int32)
        self.exps = np.ascontiguousarray(mol.exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(mol.coefs, dtype=np.float64)
        self.coords = np.ascontiguousarray(mol.coords, dtype=np.float64)
        self.c = _Basis(self.l.size, self.coords.shape[0], int(bool(mol.spherical)), _ptr(self.l).value,
                        _ptr(self.nprim).value, _ptr(self.atom).value, _ptr(self.exps).value,
                        _ptr(self.coefs).value, _ptr(self.coords).value)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """jk_plan for one geometry."""

    def __init__(self, mol, cutoff: float = 1e-13):
        self._b = BasisArrays(mol)
        h = ctypes.c_void_p()
        _check(lib().jk_plan_create(ctypes.byref(self._b.c), cutoff, ctypes.byref(h)))
        self.h = h
        nao, naoc = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().jk_plan_info(self.h, ctypes.byref(nao), ctypes.byref(naoc)))
        self.nao, self.nao_cart = nao.value, naoc.value
        self.nshell = self._b.l.size

    def close(self):
        if getattr(self, "h", None):
            lib().jk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> Stats:
        s = Stats()
        _check(lib().jk_plan_stats(self.h, ctypes.byref(s)))
        return s

    def schwarz(self) -> np.ndarray:
        Q = np.zeros((self.nshell, self.nshell))
        _check(lib().jk_plan_schwarz(self.h, _ptr(Q)))
        return Q

    def execute(self, D, J=None, K=None, precision="fp64", mix_threshold=1e-4, flags=JK_DO_J | JK_DO_K,
                omega=0.0, stream=None):
        """D: torch float64 CUDA tensor [nset, nao, nao] (or [nao, nao]).
        Returns (J, K) tensors of the same shape (allocated when not given)."""
        import torch
        squeeze = D.dim() == 2
        Dv = D.unsqueeze(0) if squeeze else D
        if Dv.dtype != torch.float64 or not Dv.is_cuda or not Dv.is_contiguous():
            raise ValueError("D must be a contiguous float64 CUDA tensor")
        if Dv.shape[1] != self.nao or Dv.shape[2] != self.nao:
            raise ValueError(f"D must be [nset, {self.nao}, {self.nao}]")
        if J is None and flags & JK_DO_J:
            J = torch.empty_like(Dv)
        if K is None and flags & JK_DO_K:
            K = torch.empty_like(Dv)
        for M in (J, K):
            if M is not None and (M.shape != Dv.shape or M.dtype != torch.float64 or not M.is_contiguous()):
                raise ValueError("J/K must match D")
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        _check(lib().jk_execute(self.h, ctypes.c_void_p(Dv.data_ptr()), Dv.shape[0], flags, prec, mix_threshold,
                                omega, ctypes.c_void_p(J.data_ptr() if J is not None else 0),
                                ctypes.c_void_p(K.data_ptr() if K is not None else 0), _stream_handle(stream)))
        if squeeze:
            return (J[0] if J is not None else None), (K[0] if K is not None else None)
        return J, K

    def set_density_screening(self, threshold: float):
        """Drop quartets with Q_IJ Q_KL max|D_block| below threshold in later
        builds (0 turns it off)."""
        _check(lib().jk_plan_set_density_screening(self.h, threshold))

    def profile(self, enable: bool = True):
        """Per-kernel HIP-event timing of later executes (resets totals)."""
        _check(lib().jk_plan_profile(self.h, int(enable)))

    def timings(self) -> list:
        n = ctypes.c_int32()
        _check(lib().jk_plan_timings(self.h, None, 0, ctypes.byref(n)))
        arr = (ClassTiming * max(1, n.value))()
        _check(lib().jk_plan_timings(self.h, arr, n.value, ctypes.byref(n)))
        return [arr[i] for i in range(n.value)]

    def eri_block(self, I, J, K, L, precision="fp64") -> np.ndarray:
        n = [(int(self._b.l[x]) + 1) * (int(self._b.l[x]) + 2) // 2 for x in (I, J, K, L)]
        out = np.zeros(n)
        _check(lib().jk_eri_block(self.h, I, J, K, L, PRECISION[precision], _ptr(out)))
        return out


class Batch:
    """jk_batch: one build over many molecules (one plan each), recorded
    into a hipGraph at the first call and replayed afterwards."""

    def __init__(self, plans, nset: int, precision="fp64", mix_threshold: float = 1e-4):
        self.plans = list(plans)  # keeps the plans alive as long as the batch
        self.nset = int(nset)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.h.value for p in self.plans])
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _check(lib().jk_batch_create(arr, len(self.plans), self.nset, prec, mix_threshold, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().jk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def execute(self, Ds, Js, Ks, stream=None):
        """Ds, Js, Ks: lists of contiguous float64 CUDA tensors
        [nset, nao_m, nao_m], one per molecule (outputs overwritten)."""
        import torch
        n = len(self.plans)
        if not (len(Ds) == len(Js) == len(Ks) == n):
            raise ValueError(f"need {n} D, J and K tensors")
        for P, *Ms in zip(self.plans, Ds, Js, Ks):
            for M in Ms:
                if (M.dtype != torch.float64 or not M.is_cuda or not M.is_contiguous()
                        or tuple(M.shape) != (self.nset, P.nao, P.nao)):
                    raise ValueError(f"tensors must be contiguous float64 CUDA [{self.nset}, {P.nao}, {P.nao}]")
        ptrs = [(ctypes.c_void_p * n)(*[M.data_ptr() for M in Ms]) for Ms in (Ds, Js, Ks)]
        _check(lib().jk_batch_execute(self.h, ptrs[0], ptrs[1], ptrs[2], _stream_handle(stream)))

    def stats(self):
        """(quartets the last execute evaluated, how many of them in FP32)."""
        n, n32 = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().jk_batch_stats(self.h, ctypes.byref(n), ctypes.byref(n32)))
        return n.value, n32.value


def build(mol, D, cutoff=1e-13, precision="fp64", stream=None):
    """One-shot jk_build.  D: torch float64 CUDA [nset, nao, nao]."""
    import torch
    Dv = D.unsqueeze(0) if D.dim() == 2 else D
    J = torch.empty_like(Dv)
    K = torch.empty_like(Dv)
    b = BasisArrays(mol)
    _check(lib().jk_build(ctypes.byref(b.c), ctypes.c_void_p(Dv.data_ptr()), Dv.shape[0], cutoff,
                          PRECISION[precision], ctypes.c_void_p(J.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                          _stream_handle(stream)))
    return J, K


def tune_set(li, lj, lk, ll, precision, family):
    """Kernel family (1, 2, 3; 0 = default) for one canonical class."""
    _check(lib().jk_tune_set(li, lj, lk, ll, PRECISION[precision], family))


def tune_set_row(li, lj, lk, ll, precision, row):
    """Row mode for one canonical class: 0 default (= 1), 1 bras with long ket
    prefixes, 2 off, 3 every bra (short ones in 64-lane workgroups); batched
    builds run the class as row tasks unless it is 2."""
    _check(lib().jk_tune_set_row(li, lj, lk, ll, PRECISION[precision], row))


def tune_set_shape(li, lj, lk, ll, min_kets=0, chunk=0):
    """Task shape of one canonical class: long-bra threshold and kets per row
    task (0 = default)."""
    _check(lib().jk_tune_set_shape(li, lj, lk, ll, min_kets, chunk))


def tune_set_split(li, lj, lk, ll, split=1):
    """Mixed-precision split of one canonical class: 1 (default) splits its
    quartets by the bound, 0 runs the class in double precision in mixed
    builds."""
    _check(lib().jk_tune_set_split(li, lj, lk, ll, split))


def tune_get(li, lj, lk, ll, precision):
    """(family a new plan would use, bit mask of built families: 1, 2, 4 for
    families 1, 2, 3)."""
    f, m = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().jk_tune_get(li, lj, lk, ll, PRECISION[precision], ctypes.byref(f), ctypes.byref(m)))
    return f.value, m.value


def tune_load(path):
    _check(lib().jk_tune_load(os.fsencode(path)))


def canonical_classes(lmax=4):
    return [(i, j, k, l) for i in range(lmax + 1) for j in range(i + 1) for k in range(i + 1)
            for l in range(k + 1) if k < i or (k == i and l <= j)]


def rys_eval(n: int, T, precision="fp64"):
    T = np.ascontiguousarray(T, dtype=np.float64)
    u = np.zeros((T.size, n))
    w = np.zeros((T.size, n))
    _check(lib().jk_rys_eval(n, _ptr(T), T.size, PRECISION[precision], _ptr(u), _ptr(w)))
    return u, w


def boys_eval(T, precision="fp64"):
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = np.zeros((T.size, 2))
    _check(lib().jk_boys_eval(1, _ptr(T), T.size, PRECISION[precision], _ptr(out)))
    return out
