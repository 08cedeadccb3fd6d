"""Pins of the oracle's J/K (Section 2, eq. jk) and of its real-solid-harmonic
transform (Section 2: spherical functions are fixed combinations of
Cartesian ones)."""
import itertools
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as o
from paper_2507_09772_amd import synth


@pytest.fixture(scope="module")
def c0():
    return synth.workload("c0")


@pytest.fixture(scope="module")
def c0_jk(c0):
    return o.jk(c0.mol, c0.D, 1e-13, mode=1)


@pytest.fixture(scope="module")
def sph2():
    return synth.small_workload(2, "B", seed=11, nset=2)


def test_brute_equals_eightfold(c0, c0_jk):
    J1, K1, n1 = c0_jk
    J0, K0, n0 = o.jk(c0.mol, c0.D, 1e-13, mode=0)
    assert n0 == n1
    assert np.abs(J1 - J0).max() <= 1e-13 * max(1.0, np.abs(J0).max())
    assert np.abs(K1 - K0).max() <= 1e-13 * max(1.0, np.abs(K0).max())


def test_brute_equals_eightfold_spherical_multi_density(sph2):
    J1, K1, n1 = o.jk(sph2.mol, sph2.D, 1e-13, mode=1)
    J0, K0, n0 = o.jk(sph2.mol, sph2.D, 1e-13, mode=0)
    assert n0 == n1
    np.testing.assert_allclose(J1, J0, atol=1e-12)
    np.testing.assert_allclose(K1, K0, atol=1e-12)


def test_symmetry_and_traces(c0, c0_jk):
    J, K, _ = c0_jk
    D = c0.D[0]
    np.testing.assert_allclose(J[0], J[0].T, atol=1e-13)
    np.testing.assert_allclose(K[0], K[0].T, atol=1e-13)
    tj, tk = np.trace(D @ J[0]), np.trace(D @ K[0])
    # positive Coulomb kernel; |gamma(1,2)|^2 <= rho(1) rho(2) for D = C C^T
    assert tj > 0
    assert 0 <= tk <= tj


def test_linear_in_density(c0):
    mol = c0.mol
    D2 = synth.random_density(mol.nao, 7, 999)[0]
    Ja, Ka, _ = o.jk(mol, c0.D[0], mode=1)
    Jb, Kb, _ = o.jk(mol, D2, mode=1)
    Jc, Kc, _ = o.jk(mol, c0.D[0] - 2.5 * D2, mode=1)
    np.testing.assert_allclose(Jc, Ja - 2.5 * Jb, atol=1e-12)
    np.testing.assert_allclose(Kc, Ka - 2.5 * Kb, atol=1e-12)


def test_translation_invariance(c0, c0_jk):
    mol = c0.mol
    m2 = synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps, coefs=mol.coefs,
                        coords=mol.coords + np.array([3.1, -7.7, 0.45]), spherical=False)
    J, K, n = o.jk(m2, c0.D, mode=1)
    J0, K0, n0 = c0_jk
    assert n == n0
    np.testing.assert_allclose(J, J0, atol=1e-12)
    np.testing.assert_allclose(K, K0, atol=1e-12)


def _cart_rotation(l, R):
    """M[new, old] for raw monomials: (R^-1 u)^e_old = sum_new M[new, old] u^e_new."""
    carts = [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]
    Rinv = R.T
    M = np.zeros((len(carts), len(carts)))
    index = {c: i for i, c in enumerate(carts)}
    for j, e in enumerate(carts):
        # expand prod_k (sum_m Rinv[k, m] u_m)^e_k
        poly = {(0, 0, 0): 1.0}
        for k in range(3):
            for _ in range(e[k]):
                new = {}
                for mono, c in poly.items():
                    for m in range(3):
                        if Rinv[k, m] == 0.0:
                            continue
                        mm = list(mono)
                        mm[m] += 1
                        new[tuple(mm)] = new.get(tuple(mm), 0.0) + c * Rinv[k, m]
                poly = new
        for mono, c in poly.items():
            M[index[mono], j] += c
    return M


def _rotate(mol, R):
    blocks = [_cart_rotation(int(l), R) for l in mol.l]
    n = sum(b.shape[0] for b in blocks)
    M = np.zeros((n, n))
    o_ = 0
    for b in blocks:
        k = b.shape[0]
        M[o_:o_ + k, o_:o_ + k] = b.T  # rows old AO, cols new AO
        o_ += k
    m2 = synth.Molecule(l=mol.l, nprim=mol.nprim, atom=mol.atom, exps=mol.exps, coefs=mol.coefs,
                        coords=mol.coords @ R.T, spherical=False)
    return m2, M


@pytest.mark.parametrize("kind", ["quarter_turn", "random"])
def test_rotation_covariance(c0, c0_jk, kind):
    """Rotated system: D' = M^T D M gives J = M J' M^T (and so E_J, E_K
    unchanged), M the Cartesian AO map of the rotation."""
    if kind == "quarter_turn":
        R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    else:
        q, r = np.linalg.qr(np.random.default_rng(8).standard_normal((3, 3)))
        R = q * np.sign(np.diag(r))
        if np.linalg.det(R) < 0:
            R[:, 0] *= -1
    m2, M = _rotate(c0.mol, R)
    D = c0.D[0]
    Dp = M.T @ D @ M
    J, K, n = c0_jk
    J2, K2, n2 = o.jk(m2, Dp, mode=1)
    if kind == "quarter_turn":
        # signed permutation: exact, including the screened set
        assert n2 == n
        np.testing.assert_allclose(M @ J2[0] @ M.T, J[0], atol=1e-12)
        np.testing.assert_allclose(M @ K2[0] @ M.T, K[0], atol=1e-12)
    # energies are invariant (screening may differ at the 1e-13 level)
    ej, ek = o.energies(D[None], J, K)
    ej2, ek2 = o.energies(Dp[None], J2, K2)
    assert ej2[0] == pytest.approx(ej[0], rel=1e-11)
    assert ek2[0] == pytest.approx(ek[0], rel=1e-11)


def test_blocks_match_full(c0, c0_jk):
    mol = c0.mol
    Q = o.schwarz(mol)
    J, K, _ = c0_jk
    off = mol.ao_offsets()
    jp = [(5, 0), (8, 3), (29, 29), (0, 13)]
    kp = [(5, 11), (2, 2), (17, 0)]
    Jb, Kb = o.jk_blocks(mol, c0.D, Q, jp, kp)
    for (I, Jx), blk in zip(jp, Jb):
        np.testing.assert_allclose(blk[0], J[0, off[I]:off[I + 1], off[Jx]:off[Jx + 1]], atol=1e-12)
    for (I, Kx), blk in zip(kp, Kb):
        np.testing.assert_allclose(blk[0], K[0, off[I]:off[I + 1], off[Kx]:off[Kx + 1]], atol=1e-12)


def test_blocks_match_full_spherical(sph2):
    mol = sph2.mol
    Q = o.schwarz(mol)
    J, K, _ = o.jk(mol, sph2.D, mode=1, Q=Q)
    off = mol.ao_offsets()
    d_or_f = [i for i, l in enumerate(mol.l) if l >= 2]
    jp = [(d_or_f[0], d_or_f[-1]), (3, 1)]
    kp = [(d_or_f[-1], 0), (d_or_f[1], d_or_f[0])]
    Jb, Kb = o.jk_blocks(mol, sph2.D, Q, jp, kp)
    for (I, Jx), blk in zip(jp, Jb):
        np.testing.assert_allclose(blk, J[:, off[I]:off[I + 1], off[Jx]:off[Jx + 1]], atol=1e-12)
    for (I, Kx), blk in zip(kp, Kb):
        np.testing.assert_allclose(blk, K[:, off[I]:off[I + 1], off[Kx]:off[Kx + 1]], atol=1e-12)


# ---------------------------------------------------------------------------
# real solid harmonics
# ---------------------------------------------------------------------------
def _carts(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def _cart_overlap(l):
    """Angular overlap of raw monomials with a common radial factor, in units
    of the x^l norm: prod (e1+e2-1)!! / (2l-1)!!."""
    def df(n):
        r = 1
        while n > 1:
            r *= n
            n -= 2
        return r
    cs = _carts(l)
    S = np.zeros((len(cs), len(cs)))
    for i, a in enumerate(cs):
        for j, b in enumerate(cs):
            s = [a[k] + b[k] for k in range(3)]
            if any(x % 2 for x in s):
                continue
            S[i, j] = df(s[0] - 1) * df(s[1] - 1) * df(s[2] - 1) / df(2 * l - 1)
    return S


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_c2s_orthonormal(l):
    T = o.c2s(l)
    np.testing.assert_allclose(T @ _cart_overlap(l) @ T.T, np.eye(2 * l + 1), atol=1e-14)


@pytest.mark.parametrize("l", [2, 3, 4])
def test_c2s_harmonic(l):
    # Laplacian of each solid harmonic polynomial vanishes
    T = o.c2s(l)
    cs = _carts(l)
    lower = {c: i for i, c in enumerate(_carts(l - 2))}
    for row in T:
        lap = np.zeros(len(lower))
        for c, coef in zip(cs, row):
            for k in range(3):
                if c[k] >= 2:
                    e = list(c)
                    e[k] -= 2
                    lap[lower[tuple(e)]] += coef * c[k] * (c[k] - 1)
        np.testing.assert_allclose(lap, 0.0, atol=1e-13)


@pytest.mark.parametrize("l", [2, 3, 4])
def test_c2s_matches_projection_of_spherical_harmonics(l):
    """Independent derivation: least-squares fit of r^l * real Y_lm (scipy)
    on random points, normalised with the same monomial overlap; sign fixed
    by the coefficient of x^|m| z^(l-|m|) (m >= 0) or x^(|m|-1) y z^(l-|m|)
    (m < 0) being positive."""
    rng = np.random.default_rng(l)
    pts = rng.standard_normal((400, 3))
    r = np.linalg.norm(pts, axis=1)
    theta = np.arccos(pts[:, 2] / r)
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    cs = _carts(l)
    A = np.stack([pts[:, 0] ** c[0] * pts[:, 1] ** c[1] * pts[:, 2] ** c[2] for c in cs], axis=1)
    S = _cart_overlap(l)
    T = o.c2s(l)
    for m in range(-l, l + 1):
        Y = special.sph_harm_y(l, abs(m), theta, phi)
        y = (Y.real if m >= 0 else Y.imag) * r ** l
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        coef /= math.sqrt(coef @ S @ coef)
        lead = (abs(m), 0, l - abs(m)) if m >= 0 else (abs(m) - 1, 1, l - abs(m))
        if coef[cs.index(lead)] < 0:
            coef = -coef
        np.testing.assert_allclose(coef, T[m + l], atol=1e-12)


def test_spherical_one_centre_overlap_is_identity():
    """Normalised contracted spherical shell: one-centre overlap matrix = I
    (Gaussian moments from the textbook formula, not from the oracle)."""
    for (l, e, c) in synth.make_basis("B").shells["O"] + synth.make_basis("C").shells["O"]:
        if l < 2:
            continue
        T = o.c2s(l)
        cs = _carts(l)

        def df(n):
            r = 1
            while n > 1:
                r *= n
                n -= 2
            return r
        S = np.zeros((len(cs), len(cs)))
        for i, a in enumerate(cs):
            for j, bb in enumerate(cs):
                s = [a[k] + bb[k] for k in range(3)]
                if any(x % 2 for x in s):
                    continue
                for p in range(e.size):
                    for q in range(e.size):
                        g = e[p] + e[q]
                        S[i, j] += c[p] * c[q] * math.pi ** 1.5 / g ** 1.5 * \
                            df(s[0] - 1) * df(s[1] - 1) * df(s[2] - 1) / (2 * g) ** l
        np.testing.assert_allclose(T @ S @ T.T, np.eye(2 * l + 1), atol=1e-13)
