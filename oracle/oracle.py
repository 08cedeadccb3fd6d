"""Python access to the CPU reference J/K build (oracle.c).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only tests/, the smoke check and the
benchmark's CPU-baseline leg import this module.  It imports nothing from
the GPU package; callers hand it plain numpy arrays.

Parity status of each function (pins in tests/test_oracle_*.py):
  boys        pinned: mpmath 1F1 form, F_m(0), large-T closed form, recursion
  eri_block   pinned: (ss|ss) closed forms, brute-force quadrature of s/p
              primitive integrals, 8-fold symmetry, Schwarz bound, scaling
  schwarz     pinned through eri_block
  jk          pinned: brute == 8-fold, symmetry, Tr(DJ) >= 0,
              0 <= Tr(DK) <= Tr(DJ), rotation / translation invariance,
              linearity in D
  jk_blocks   pinned: equals the corresponding blocks of jk
  mixed_count pinned: its significant count equals jk's; its FP32 count
              equals a brute-force count over every ordered quartet in numpy
  c2s         pinned: orthonormality, harmonicity, agreement with an
              independent least-squares projection of spherical harmonics
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP, -O2, strict IEEE arithmetic)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_oracle(force=True)
        _lib = ctypes.CDLL(_SO)
    return _lib


_i32p = ctypes.POINTER(ctypes.c_int)
_f64p = ctypes.POINTER(ctypes.c_double)


def _ip(a):
    return a.ctypes.data_as(_i32p)


def _dp(a):
    return a.ctypes.data_as(_f64p)


class _Basis:
    """Keeps contiguous copies of the basis arrays alive during a call."""

    def __init__(self, mol):
        self.l = np.ascontiguousarray(mol.l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(mol.nprim, dtype=np.int32)
        self.atom = np.ascontiguousarray(mol.atom, dtype=np.int32)
        self.exps = np.ascontiguousarray(mol.exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(mol.coefs, dtype=np.float64)
        self.coords = np.ascontiguousarray(mol.coords, dtype=np.float64)
        self.spherical = int(bool(mol.spherical))
        self.ns = int(self.l.size)
        self.natom = int(self.coords.shape[0])

    def args(self):
        return (ctypes.c_int(self.ns), ctypes.c_int(self.natom), ctypes.c_int(self.spherical),
                _ip(self.l), _ip(self.nprim), _ip(self.atom), _dp(self.exps), _dp(self.coefs),
                _dp(self.coords))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    _load().oracle_boys(ctypes.c_int(mmax), ctypes.c_double(T), _dp(F))
    return F


def nao(mol) -> tuple[int, int]:
    b = _Basis(mol)
    ne, nc = ctypes.c_int(), ctypes.c_int()
    rc = _load().oracle_nao(*b.args(), ctypes.byref(ne), ctypes.byref(nc))
    if rc:
        raise ValueError("invalid basis")
    return ne.value, nc.value


def eri_block(mol, I: int, J: int, K: int, L: int, omega: float = 0.0) -> np.ndarray:
    """Contracted Cartesian block (IJ|KL), shape [nI, nJ, nK, nL], over the
    operator 1/r (omega = 0), erf(omega r)/r (omega > 0) or
    erfc(|omega| r)/r (omega < 0)."""
    b = _Basis(mol)
    nc = [(int(mol.l[x]) + 1) * (int(mol.l[x]) + 2) // 2 for x in (I, J, K, L)]
    out = np.zeros(nc)
    rc = _load().oracle_eri_block_op(*b.args(), ctypes.c_double(omega), ctypes.c_int(I), ctypes.c_int(J),
                                     ctypes.c_int(K), ctypes.c_int(L), _dp(out))
    if rc:
        raise ValueError("invalid basis")
    return out


def schwarz(mol) -> np.ndarray:
    """Q[I, J] = sqrt(max_{a in I, b in J} |(ab|ab)|)."""
    b = _Basis(mol)
    Q = np.zeros((b.ns, b.ns))
    if _load().oracle_schwarz(*b.args(), _dp(Q)):
        raise ValueError("invalid basis")
    return Q


def jk(mol, D: np.ndarray, cutoff: float = 1e-13, mode: int = 1, Q: np.ndarray | None = None,
       omega: float = 0.0, dscreen: float = 0.0):
    """Full J, K ([nset, nao, nao] each) and the number of significant unique
    shell quartets.  mode 0: every ordered quartet; mode 1: eight-fold.
    omega selects the operator as in eri_block; the Schwarz screening always
    uses the full-range factors.  dscreen > 0 adds the density screening
    Q_IJ Q_KL max|D over the six blocks| >= dscreen."""
    b = _Basis(mol)
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    nset, n = D.shape[0], D.shape[1]
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    cnt = ctypes.c_longlong()
    qp = _dp(np.ascontiguousarray(Q, dtype=np.float64)) if Q is not None else None
    if Q is not None:
        Qc = np.ascontiguousarray(Q, dtype=np.float64)
        qp = _dp(Qc)
    rc = _load().oracle_jk_screen(*b.args(), ctypes.c_double(omega), ctypes.c_double(dscreen), _dp(D),
                                  ctypes.c_int(nset), ctypes.c_double(cutoff), qp, ctypes.c_int(mode), _dp(J), _dp(K),
                                  ctypes.byref(cnt))
    if rc:
        raise ValueError("invalid basis")
    return J, K, int(cnt.value)


def mixed_count(mol, D: np.ndarray, cutoff: float = 1e-13, thr: float = 1e-4, Q: np.ndarray | None = None):
    """(significant unique quartets, those whose bound Q_IJ Q_KL max|D_block|
    over the six blocks is below thr): the mixed-precision split's count."""
    b = _Basis(mol)
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    qp = None
    if Q is not None:
        Qc = np.ascontiguousarray(Q, dtype=np.float64)
        qp = _dp(Qc)
    ns, nl = ctypes.c_longlong(), ctypes.c_longlong()
    rc = _load().oracle_mixed_count(*b.args(), _dp(D), ctypes.c_int(D.shape[0]), ctypes.c_double(cutoff),
                                    ctypes.c_double(thr), qp, ctypes.byref(ns), ctypes.byref(nl))
    if rc:
        raise ValueError("invalid basis")
    return int(ns.value), int(nl.value)


def jk_blocks(mol, D: np.ndarray, Q: np.ndarray, jpairs, kpairs, cutoff: float = 1e-13):
    """Sampled J blocks (I, J) and K blocks (I, K) in the external basis.

    Returns (list of J blocks [nset, nI, nJ], list of K blocks [nset, nI, nK]).
    """
    b = _Basis(mol)
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    nset = D.shape[0]
    sph = bool(mol.spherical)
    size = (lambda l: 2 * l + 1) if sph else (lambda l: (l + 1) * (l + 2) // 2)
    jp = np.ascontiguousarray(np.asarray(jpairs, dtype=np.int32).reshape(-1, 2))
    kp = np.ascontiguousarray(np.asarray(kpairs, dtype=np.int32).reshape(-1, 2))
    js = [(size(int(mol.l[i])), size(int(mol.l[j]))) for i, j in jp]
    ks = [(size(int(mol.l[i])), size(int(mol.l[j]))) for i, j in kp]
    Jo = np.zeros(sum(nset * a * c for a, c in js) + 1)
    Ko = np.zeros(sum(nset * a * c for a, c in ks) + 1)
    Qc = np.ascontiguousarray(Q, dtype=np.float64)
    rc = _load().oracle_jk_blocks(*b.args(), _dp(D), ctypes.c_int(nset), ctypes.c_double(cutoff), _dp(Qc),
                                  ctypes.c_int(len(jp)), _ip(jp), ctypes.c_int(len(kp)), _ip(kp),
                                  _dp(Jo), _dp(Ko))
    if rc:
        raise ValueError("invalid basis")
    outJ, outK, o = [], [], 0
    for a, c in js:
        outJ.append(Jo[o:o + nset * a * c].reshape(nset, a, c))
        o += nset * a * c
    o = 0
    for a, c in ks:
        outK.append(Ko[o:o + nset * a * c].reshape(nset, a, c))
        o += nset * a * c
    return outJ, outK


def jk_subset(mol, D: np.ndarray, Q: np.ndarray, sel, cutoff: float = 1e-13):
    """Eight-fold digestion over the bra pair indices in ``sel`` only
    (unsymmetrised Cartesian partial J', K').  Returns (J', K', nsig)."""
    b = _Basis(mol)
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    nset = D.shape[0]
    nc = int(sum((int(x) + 1) * (int(x) + 2) // 2 for x in mol.l))
    Jp = np.zeros((nset, nc, nc))
    Kp = np.zeros((nset, nc, nc))
    s = np.ascontiguousarray(sel, dtype=np.int32)
    Qc = np.ascontiguousarray(Q, dtype=np.float64)
    cnt = ctypes.c_longlong()
    rc = _load().oracle_jk_subset(*b.args(), _dp(D), ctypes.c_int(nset), ctypes.c_double(cutoff), _dp(Qc),
                                  ctypes.c_int(s.size), _ip(s), _dp(Jp), _dp(Kp), ctypes.byref(cnt))
    if rc:
        raise ValueError("invalid basis")
    return Jp, Kp, int(cnt.value)


def c2s(l: int) -> np.ndarray:
    """[(2l+1), ncart] real-solid-harmonic coefficients (rows m = -l..l;
    l = 1 stays x, y, z)."""
    T = np.zeros((2 * l + 1, (l + 1) * (l + 2) // 2))
    if _load().oracle_c2s(ctypes.c_int(l), _dp(T)):
        raise ValueError("l out of range")
    return T


def energies(D: np.ndarray, J: np.ndarray, K: np.ndarray):
    """Closed-shell reading: E_J = 2 Tr(D J), E_K = Tr(D K), per density."""
    D = D.reshape(-1, *D.shape[-2:])
    J = J.reshape(D.shape)
    K = K.reshape(D.shape)
    EJ = 2.0 * np.einsum("sij,sij->s", D, J)
    EK = np.einsum("sij,sij->s", D, K)
    return EJ, EK


def timed_jk(mol, D, cutoff=1e-13, mode=1):
    t0 = time.perf_counter()
    r = jk(mol, D, cutoff, mode)
    return r, time.perf_counter() - t0
