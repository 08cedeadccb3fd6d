"""Pins of the oracle's density screening (direct-SCF screening by the
density matrix at shell-pair level, Section 2): a quartet is kept when
Q_IJ Q_KL max(Dm_IJ, Dm_KL, Dm_IK, Dm_IL, Dm_JK, Dm_JL) >= dscreen, with Dm
the block maxima of |D| over the Cartesian density (double precision).

The reference here is a separate brute-force J/K in numpy over every ordered
shell quartet (blocks from the pinned oracle ERI), with the screening rule
applied independently, plus the bound that every dropped contribution obeys."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2507_09772_amd import synth


def brute_jk_screened(mol, D, cutoff, dscreen):
    ns = mol.nshell
    off = mol.ao_offsets()
    Q = o.schwarz(mol)
    D = D[0]
    dm = np.zeros((ns, ns))
    for I in range(ns):
        for J in range(ns):
            dm[I, J] = float(np.abs(D[off[I]:off[I + 1], off[J]:off[J + 1]]).max())
    J_ = np.zeros_like(D)
    K_ = np.zeros_like(D)
    kept = dropped = 0
    for I in range(ns):
        for Jx in range(ns):
            for K in range(ns):
                for L in range(ns):
                    if Q[I, Jx] * Q[K, L] < cutoff:
                        continue
                    m = max(dm[I, Jx], dm[K, L], dm[I, K], dm[I, L], dm[Jx, K], dm[Jx, L])
                    if Q[I, Jx] * Q[K, L] * m < dscreen:
                        dropped += 1
                        continue
                    kept += 1
                    blk = o.eri_block(mol, I, Jx, K, L)
                    si, sj, sk, sl = (slice(off[x], off[x + 1]) for x in (I, Jx, K, L))
                    J_[si, sj] += np.einsum("abcd,cd->ab", blk, D[sk, sl])
                    K_[si, sk] += np.einsum("abcd,bd->ac", blk, D[sj, sl])
    return J_, K_, kept, dropped


@pytest.fixture(scope="module")
def water():
    wl = synth.small_workload(1, "A", seed=8)
    wl.mol.spherical = False
    return wl


@pytest.mark.parametrize("dscreen", [1e-9, 1e-6, 1e-4])
def test_screened_jk_matches_brute_force(water, dscreen):
    mol, D = water.mol, water.D
    Jb, Kb, kept, dropped = brute_jk_screened(mol, D, 1e-13, dscreen)
    assert kept > 0 and dropped > 0
    for mode in (0, 1):
        J, K, _ = o.jk(mol, D, 1e-13, mode=mode, dscreen=dscreen)
        assert np.abs(J[0] - Jb).max() <= 1e-13 * max(1.0, np.abs(Jb).max())
        assert np.abs(K[0] - Kb).max() <= 1e-13 * max(1.0, np.abs(Kb).max())


def test_zero_threshold_and_bound():
    wl = synth.workload("c0")
    J0, K0, n0 = o.jk(wl.mol, wl.D, wl.cutoff)
    Jz, Kz, nz = o.jk(wl.mol, wl.D, wl.cutoff, dscreen=0.0)
    assert nz == n0 and np.abs(Jz - J0).max() <= 1e-13 and np.abs(Kz - K0).max() <= 1e-13
    for thr in (1e-8, 1e-5):
        J, K, n = o.jk(wl.mol, wl.D, wl.cutoff, dscreen=thr)
        assert n < n0
        # each dropped unique quartet feeds at most 2 J and 4 K element updates per
        # Cartesian element, each below thr; J' and K' are then symmetrised
        bound = 2 * 8 * (n0 - n) * thr
        assert np.abs(J - J0).max() <= bound and np.abs(K - K0).max() <= bound


@pytest.mark.parametrize("basis,nw,thr", [("A", 3, 1e-4), ("B", 2, 1e-4), ("A", 2, 1e-6)])
def test_mixed_count_brute_force(basis, nw, thr):
    """The mixed-precision split count: significant unique quartets as in jk,
    and those with Q_IJ Q_KL max|D| over the six blocks below thr, counted
    here by a plain loop over the canonical quartets in numpy."""
    wl = synth.small_workload(nw, basis, seed=17 + nw)
    mol, D = wl.mol, wl.D
    ns = mol.nshell
    Q = o.schwarz(mol)
    # Cartesian density blocks (spherical bases: D_cart = T^T D T per shell)
    if mol.spherical:
        T = [o.c2s(l) for l in range(4)]
        offe = mol.ao_offsets()
        nc = [(int(l) + 1) * (int(l) + 2) // 2 for l in mol.l]
        offc = np.concatenate([[0], np.cumsum(nc)])
        Dc = np.zeros((D.shape[0], offc[-1], offc[-1]))
        for I in range(ns):
            for J in range(ns):
                Dc[:, offc[I]:offc[I + 1], offc[J]:offc[J + 1]] = np.einsum(
                    "ma,smn,nb->sab", T[mol.l[I]], D[:, offe[I]:offe[I + 1], offe[J]:offe[J + 1]], T[mol.l[J]])
    else:
        Dc, offc = D, mol.ao_offsets()
    dm = np.array([[np.abs(Dc[:, offc[I]:offc[I + 1], offc[J]:offc[J + 1]]).max() for J in range(ns)]
                   for I in range(ns)])
    pairs = [(I, J) for I in range(ns) for J in range(I + 1)]
    nsig = nlow = 0
    for a, (I, J) in enumerate(pairs):
        for (K, L) in pairs[:a + 1]:
            qq = Q[I, J] * Q[K, L]
            if qq < 1e-13:
                continue
            nsig += 1
            if qq * max(dm[I, J], dm[K, L], dm[I, K], dm[I, L], dm[J, K], dm[J, L]) < thr:
                nlow += 1
    got = o.mixed_count(mol, D, 1e-13, thr)
    assert got == (nsig, nlow)
    assert got[0] == o.jk(mol, D, 1e-13)[2]
    assert 0 < nlow < nsig
