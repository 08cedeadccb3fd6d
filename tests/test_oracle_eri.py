"""Pins of the oracle's contracted ERI blocks (Section 2, eq. rys0) against
closed forms, brute-force numerical quadrature, the permutational symmetry
and the Schwarz bound (Section 2, eq. schwartz) and exact scaling laws."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as o
from paper_2507_09772_amd import synth


def prim_molecule(centers, shells):
    """shells: list of (l, alpha, coef, atom)."""
    return synth.Molecule(
        l=np.array([s[0] for s in shells], np.int32),
        nprim=np.ones(len(shells), np.int32),
        atom=np.array([s[3] for s in shells], np.int32),
        exps=np.array([s[1] for s in shells], float),
        coefs=np.array([s[2] for s in shells], float),
        coords=np.asarray(centers, float), spherical=False)


def cart_list(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def ssss_closed(a, A, b, B, c, C, d, D):
    """(ss|ss) over raw s primitives: 2 pi^(5/2)/(p q sqrt(p+q)) K_AB K_CD F_0(T),
    with F_0 from math.erf."""
    A, B, C, D = map(np.asarray, (A, B, C, D))
    p, q = a + b, c + d
    P, Q = (a * A + b * B) / p, (c * C + d * D) / q
    kab = math.exp(-a * b / p * np.sum((A - B) ** 2))
    kcd = math.exp(-c * d / q * np.sum((C - D) ** 2))
    T = p * q / (p + q) * np.sum((P - Q) ** 2)
    F0 = 1.0 if T < 1e-300 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    return 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * kab * kcd * F0


def test_ssss_same_centre_normalised():
    # four identical normalised s Gaussians on one centre: 2 sqrt(alpha/pi)
    for alpha in (1.0, 0.37, 12.5):
        n = (2 * alpha / math.pi) ** 0.75
        mol = prim_molecule([[0.3, -0.2, 0.1]], [(0, alpha, n, 0)])
        v = o.eri_block(mol, 0, 0, 0, 0)[0, 0, 0, 0]
        assert v == pytest.approx(2 * math.sqrt(alpha / math.pi), rel=1e-14)
    mol = prim_molecule([[0, 0, 0]], [(0, 1.0, (2 / math.pi) ** 0.75, 0)])
    assert o.eri_block(mol, 0, 0, 0, 0)[0, 0, 0, 0] == pytest.approx(1.1283791670955126, rel=1e-15)


def test_ssss_separated_charge_distributions():
    # normalised s densities |phi_a|^2 and |phi_b|^2 interact as erf(sqrt(rho) R)/R
    a, b = 0.8, 1.7
    R = 2.3
    na, nb = (2 * a / math.pi) ** 0.75, (2 * b / math.pi) ** 0.75
    mol = prim_molecule([[0, 0, 0], [0, 0, R]], [(0, a, na, 0), (0, b, nb, 1)])
    v = o.eri_block(mol, 0, 0, 1, 1)[0, 0, 0, 0]
    rho = (2 * a) * (2 * b) / (2 * a + 2 * b)
    assert v == pytest.approx(math.erf(math.sqrt(rho) * R) / R, rel=1e-14)


def test_ssss_general_closed_form():
    rng = np.random.default_rng(5)
    for _ in range(20):
        C = rng.uniform(-2, 2, size=(4, 3))
        ex = np.exp(rng.uniform(math.log(0.1), math.log(20), size=4))
        mol = prim_molecule(C, [(0, ex[i], 1.0, i) for i in range(4)])
        v = o.eri_block(mol, 0, 1, 2, 3)[0, 0, 0, 0]
        ref = ssss_closed(ex[0], C[0], ex[1], C[1], ex[2], C[2], ex[3], C[3])
        assert v == pytest.approx(ref, rel=1e-13)


# ---------------------------------------------------------------------------
# brute-force quadrature: 1/r12 = 2/sqrt(pi) int_0^inf exp(-t^2 r12^2) dt.
# For fixed t the six-dimensional integral factorises into three
# two-dimensional Gaussian x polynomial integrals, done exactly by
# tensor Gauss-Hermite quadrature on the principal axes; the t integral is
# done numerically.  No Boys function and no recurrence is involved.
# ---------------------------------------------------------------------------
# 10 nodes per axis integrate polynomials up to degree 19 exactly: enough
# for every Cartesian product up to (gg|gg) (degree 16 along one axis).
_GH_X, _GH_W = np.polynomial.hermite.hermgauss(10)


def _direction_integral(t, al, ce, pw):
    """al: 4 exponents, ce: 4 centre coordinates (this axis), pw: 4 powers."""
    t2 = t * t
    M = np.array([[al[0] + al[1] + t2, -t2], [-t2, al[2] + al[3] + t2]])
    bvec = np.array([al[0] * ce[0] + al[1] * ce[1], al[2] * ce[2] + al[3] * ce[3]])
    c0 = sum(al[i] * ce[i] ** 2 for i in range(4))
    x0 = np.linalg.solve(M, bvec)
    e0 = c0 - bvec @ x0
    lam, V = np.linalg.eigh(M)
    Z1, Z2 = np.meshgrid(_GH_X, _GH_X, indexing="ij")
    W = np.outer(_GH_W, _GH_W)
    Y = V @ np.stack([Z1.ravel() / math.sqrt(lam[0]), Z2.ravel() / math.sqrt(lam[1])])
    X1 = x0[0] + Y[0]
    X2 = x0[1] + Y[1]
    f = (X1 - ce[0]) ** pw[0] * (X1 - ce[1]) ** pw[1] * (X2 - ce[2]) ** pw[2] * (X2 - ce[3]) ** pw[3]
    return math.exp(-e0) * float(W.ravel() @ f) / math.sqrt(np.linalg.det(M))


def eri_quadrature(al, centers, powers):
    def g(t):
        v = 1.0
        for ax in range(3):
            v *= _direction_integral(t, al, [c[ax] for c in centers], [p[ax] for p in powers])
        return v
    val, err = integrate.quad(g, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
    return 2.0 / math.sqrt(math.pi) * val


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1), (2, 1, 0, 1),
                                (3, 0, 0, 0), (0, 0, 0, 3), (3, 1, 2, 0), (2, 2, 2, 2), (3, 3, 1, 1), (1, 3, 3, 2),
                                (3, 3, 3, 3), (4, 0, 0, 0), (0, 1, 4, 2), (4, 4, 2, 1), (3, 4, 4, 3), (4, 4, 4, 4)])
def test_primitive_eri_vs_quadrature(ls):
    """Every (li lj|lk ll) pattern the workloads reach up to (gg|gg), with
    the f and g shells in every position, against brute-force quadrature."""
    rng = np.random.default_rng(100 + sum(ls) + 7 * ls[0] + 3 * ls[3])
    C = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.2), math.log(5), size=4))
    mol = prim_molecule(C, [(ls[i], ex[i], 1.0, i) for i in range(4)])
    blk = o.eri_block(mol, 0, 1, 2, 3)
    carts = [cart_list(l) for l in ls]
    idx = list(np.ndindex(*blk.shape))
    sel = [idx[i] for i in rng.choice(len(idx), size=min(6, len(idx)), replace=False)]
    for (a, b, c, d) in sel:
        pw = [carts[0][a], carts[1][b], carts[2][c], carts[3][d]]
        ref = eri_quadrature(ex, C, pw)
        assert blk[a, b, c, d] == pytest.approx(ref, rel=1e-9, abs=1e-12), (ls, (a, b, c, d))


# ---------------------------------------------------------------------------
# symmetry, bounds, scaling on the config-0 molecule
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c0():
    return synth.workload("c0")


def _quartets_by_l(mol, want):
    out = {}
    ls = [int(x) for x in mol.l]
    for I in range(len(ls)):
        for J in range(len(ls)):
            for K in range(len(ls)):
                for L in range(len(ls)):
                    key = (ls[I], ls[J], ls[K], ls[L])
                    if key in want and key not in out and len({mol.atom[I], mol.atom[J], mol.atom[K], mol.atom[L]}) > 2:
                        out[key] = (I, J, K, L)
    return out


def test_eightfold_symmetry(c0):
    mol = c0.mol
    qs = _quartets_by_l(mol, {(2, 1, 0, 1), (1, 1, 2, 0), (2, 2, 1, 0), (0, 1, 1, 2)})
    assert len(qs) == 4
    for (I, J, K, L) in qs.values():
        v = o.eri_block(mol, I, J, K, L)
        np.testing.assert_allclose(o.eri_block(mol, J, I, K, L), v.transpose(1, 0, 2, 3), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(o.eri_block(mol, I, J, L, K), v.transpose(0, 1, 3, 2), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(o.eri_block(mol, K, L, I, J), v.transpose(2, 3, 0, 1), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(o.eri_block(mol, L, K, J, I), v.transpose(3, 2, 1, 0), rtol=1e-12, atol=1e-15)


def test_schwarz_bound_and_positivity(c0):
    mol = c0.mol
    Q = o.schwarz(mol)
    rng = np.random.default_rng(3)
    ns = mol.nshell
    for I in range(ns):
        for J in range(I + 1):
            d = o.eri_block(mol, I, J, I, J)
            nab = d.shape[0] * d.shape[1]
            diag = np.diag(d.reshape(nab, nab))
            assert np.all(diag >= 0)
            assert math.sqrt(diag.max()) == pytest.approx(Q[I, J], rel=1e-14)
    for _ in range(150):
        I, J, K, L = rng.integers(0, ns, size=4)
        v = o.eri_block(mol, I, J, K, L)
        assert np.abs(v).max() <= Q[I, J] * Q[K, L] * (1 + 1e-12)


def test_scaling_law(c0):
    # coords x lam, exps / lam^2, coefs x lam^-(l+3/2): every ERI scales by 1/lam
    mol = c0.mol
    lam = 1.7
    lpp = np.repeat(mol.l, mol.nprim)
    mol2 = synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps / lam ** 2,
                          coefs=mol.coefs * lam ** (-(lpp + 1.5)), coords=mol.coords * lam, spherical=False)
    qs = _quartets_by_l(mol, {(2, 1, 0, 1), (1, 0, 0, 0), (2, 2, 1, 1)})
    for (I, J, K, L) in qs.values():
        np.testing.assert_allclose(o.eri_block(mol2, I, J, K, L) * lam, o.eri_block(mol, I, J, K, L),
                                   rtol=1e-12, atol=1e-16)


# ---------------------------------------------------------------------------
# the same pins on a molecule of the spherical triple-zeta-shaped basis,
# whose quartets reach f shells in every position
# ---------------------------------------------------------------------------
def _quartets_by_l_sampled(mol, want, seed=0):
    """One shell quartet per wanted (li, lj, lk, ll) pattern, on at least
    three distinct atoms, by random draws over the shells of each l."""
    rng = np.random.default_rng(seed)
    by_l = {}
    for i, l in enumerate(int(x) for x in mol.l):
        by_l.setdefault(l, []).append(i)
    out = {}
    for key in sorted(want):
        for _ in range(2000):
            q = tuple(int(rng.choice(by_l[l])) for l in key)
            if len({int(mol.atom[x]) for x in q}) > 2:
                out[key] = q
                break
    return out


@pytest.fixture(scope="module")
def wat_b():
    wl = synth.small_workload(3, "B", seed=31)
    mol = wl.mol
    # Cartesian blocks: the ERI pins concern the Cartesian integrals
    return synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps, coefs=mol.coefs,
                          coords=mol.coords, spherical=False)


_F_KEYS = {(3, 0, 0, 0), (3, 2, 1, 0), (3, 3, 1, 1), (1, 3, 3, 2), (3, 3, 3, 3), (2, 3, 0, 3), (3, 1, 3, 1)}


def test_eightfold_symmetry_f_shells(wat_b):
    mol = wat_b
    qs = _quartets_by_l_sampled(mol, _F_KEYS)
    assert len(qs) == len(_F_KEYS)
    for (I, J, K, L) in qs.values():
        v = o.eri_block(mol, I, J, K, L)
        tol = dict(rtol=1e-12, atol=1e-14 * max(1.0, np.abs(v).max()))
        np.testing.assert_allclose(o.eri_block(mol, J, I, K, L), v.transpose(1, 0, 2, 3), **tol)
        np.testing.assert_allclose(o.eri_block(mol, I, J, L, K), v.transpose(0, 1, 3, 2), **tol)
        np.testing.assert_allclose(o.eri_block(mol, K, L, I, J), v.transpose(2, 3, 0, 1), **tol)
        np.testing.assert_allclose(o.eri_block(mol, L, K, J, I), v.transpose(3, 2, 1, 0), **tol)


def test_schwarz_bound_f_shells(wat_b):
    mol = wat_b
    Q = o.schwarz(mol)
    ls = [int(x) for x in mol.l]
    f = [i for i, l in enumerate(ls) if l == 3]
    assert f
    for I in f:
        for J in range(mol.nshell):
            d = o.eri_block(mol, I, J, I, J)
            nab = d.shape[0] * d.shape[1]
            diag = np.diag(d.reshape(nab, nab))
            assert np.all(diag >= 0)
            assert math.sqrt(diag.max()) == pytest.approx(Q[I, J], rel=1e-14)
    rng = np.random.default_rng(11)
    for _ in range(60):
        I, J, K = (int(x) for x in rng.integers(0, mol.nshell, size=3))
        L = f[int(rng.integers(len(f)))]
        v = o.eri_block(mol, I, J, K, L)
        assert np.abs(v).max() <= Q[I, J] * Q[K, L] * (1 + 1e-12)


def test_scaling_law_f_shells(wat_b):
    mol = wat_b
    lam = 0.83
    lpp = np.repeat(mol.l, mol.nprim)
    mol2 = synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps / lam ** 2,
                          coefs=mol.coefs * lam ** (-(lpp + 1.5)), coords=mol.coords * lam, spherical=False)
    for (I, J, K, L) in _quartets_by_l_sampled(mol, _F_KEYS).values():
        ref = o.eri_block(mol, I, J, K, L)
        np.testing.assert_allclose(o.eri_block(mol2, I, J, K, L) * lam, ref, rtol=1e-12,
                                   atol=1e-14 * max(1.0, np.abs(ref).max()))


# ---------------------------------------------------------------------------
# g shells: the same pins on a molecule of the quadruple-zeta-shaped basis
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def wat_c():
    wl = synth.small_workload(3, "C", seed=33)
    mol = wl.mol
    return synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps, coefs=mol.coefs,
                          coords=mol.coords, spherical=False)


_G_KEYS = {(4, 0, 0, 0), (4, 3, 2, 1), (4, 4, 1, 0), (2, 4, 4, 1), (4, 4, 4, 4), (3, 4, 0, 4)}


def test_eightfold_symmetry_g_shells(wat_c):
    mol = wat_c
    qs = _quartets_by_l_sampled(mol, _G_KEYS)
    assert len(qs) == len(_G_KEYS)
    for (I, J, K, L) in qs.values():
        v = o.eri_block(mol, I, J, K, L)
        tol = dict(rtol=1e-12, atol=1e-14 * max(1.0, np.abs(v).max()))
        np.testing.assert_allclose(o.eri_block(mol, J, I, K, L), v.transpose(1, 0, 2, 3), **tol)
        np.testing.assert_allclose(o.eri_block(mol, K, L, I, J), v.transpose(2, 3, 0, 1), **tol)
        np.testing.assert_allclose(o.eri_block(mol, L, K, J, I), v.transpose(3, 2, 1, 0), **tol)


def test_schwarz_bound_and_scaling_g_shells(wat_c):
    mol = wat_c
    Q = o.schwarz(mol)
    g = [i for i, l in enumerate(int(x) for x in mol.l) if l == 4]
    assert g
    for I in g:
        for J in range(0, mol.nshell, 3):
            d = o.eri_block(mol, I, J, I, J)
            nab = d.shape[0] * d.shape[1]
            diag = np.diag(d.reshape(nab, nab))
            assert np.all(diag >= 0)
            assert math.sqrt(diag.max()) == pytest.approx(Q[I, J], rel=1e-14)
    rng = np.random.default_rng(12)
    for _ in range(30):
        I, J, K = (int(x) for x in rng.integers(0, mol.nshell, size=3))
        L = g[int(rng.integers(len(g)))]
        assert np.abs(o.eri_block(mol, I, J, K, L)).max() <= Q[I, J] * Q[K, L] * (1 + 1e-12)
    lam = 1.3
    lpp = np.repeat(mol.l, mol.nprim)
    mol2 = synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps / lam ** 2,
                          coefs=mol.coefs * lam ** (-(lpp + 1.5)), coords=mol.coords * lam, spherical=False)
    for (I, J, K, L) in _quartets_by_l_sampled(mol, {(4, 4, 2, 1), (4, 0, 3, 4)}, seed=5).values():
        ref = o.eri_block(mol, I, J, K, L)
        np.testing.assert_allclose(o.eri_block(mol2, I, J, K, L) * lam, ref, rtol=1e-12,
                                   atol=1e-14 * max(1.0, np.abs(ref).max()))
