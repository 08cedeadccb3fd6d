"""Pins of the oracle's range-separated integrals (the range-separation
parameter omega of Tables 1 and 2: long range erf(omega r)/r for omega > 0,
short range erfc(|omega| r)/r for omega < 0).

Independent of the oracle's Hermite/Boys machinery: the Gaussian transform
erf(w r)/r = (2/sqrt(pi)) int_0^w exp(-t^2 r^2) dt (and the remaining range
[w, inf) for erfc) integrated numerically over Gaussian-product quadrature,
and the closed-form attenuated interaction of two normalised s charge
distributions."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as o
from paper_2507_09772_amd import synth

from test_oracle_eri import _direction_integral, cart_list, prim_molecule


def eri_quadrature_range(al, centers, powers, lo, hi):
    def g(t):
        v = 1.0
        for ax in range(3):
            v *= _direction_integral(t, al, [c[ax] for c in centers], [p[ax] for p in powers])
        return v
    val, _ = integrate.quad(g, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)
    return 2.0 / math.sqrt(math.pi) * val


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (2, 0, 1, 0), (2, 1, 1, 1)])
@pytest.mark.parametrize("omega", [0.35, 1.3])
def test_range_separated_vs_quadrature(ls, omega):
    rng = np.random.default_rng(300 + 7 * sum(ls) + int(10 * omega))
    C = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.2), math.log(5), size=4))
    mol = prim_molecule(C, [(ls[i], ex[i], 1.0, i) for i in range(4)])
    lr = o.eri_block(mol, 0, 1, 2, 3, omega=omega)
    sr = o.eri_block(mol, 0, 1, 2, 3, omega=-omega)
    carts = [cart_list(l) for l in ls]
    idx = list(np.ndindex(*lr.shape))
    sel = [idx[i] for i in rng.choice(len(idx), size=min(5, len(idx)), replace=False)]
    for (a, b, c, d) in sel:
        pw = [carts[0][a], carts[1][b], carts[2][c], carts[3][d]]
        ref_lr = eri_quadrature_range(ex, C, pw, 0.0, omega)
        ref_sr = eri_quadrature_range(ex, C, pw, omega, np.inf)
        assert lr[a, b, c, d] == pytest.approx(ref_lr, rel=1e-9, abs=1e-13), (ls, omega, (a, b, c, d))
        assert sr[a, b, c, d] == pytest.approx(ref_sr, rel=1e-9, abs=1e-13), (ls, omega, (a, b, c, d))


def test_long_range_charge_distributions():
    # normalised s densities (exponents 2a, 2b) through erf(w r)/r interact as
    # erf(mu R)/R with 1/mu^2 = 1/(2a) + 1/(2b) + 1/w^2
    a, b, R = 0.8, 1.7, 2.3
    na, nb = (2 * a / math.pi) ** 0.75, (2 * b / math.pi) ** 0.75
    mol = prim_molecule([[0, 0, 0], [0, 0, R]], [(0, a, na, 0), (0, b, nb, 1)])
    for w in (0.1, 0.5, 2.0, 9.0):
        mu = 1.0 / math.sqrt(1 / (2 * a) + 1 / (2 * b) + 1 / w ** 2)
        v = o.eri_block(mol, 0, 0, 1, 1, omega=w)[0, 0, 0, 0]
        assert v == pytest.approx(math.erf(mu * R) / R, rel=1e-13)
        full = o.eri_block(mol, 0, 0, 1, 1)[0, 0, 0, 0]
        assert o.eri_block(mol, 0, 0, 1, 1, omega=-w)[0, 0, 0, 0] == pytest.approx(full - math.erf(mu * R) / R,
                                                                                    rel=1e-12, abs=1e-15)


def test_range_separation_limits():
    wl = synth.small_workload(1, "A", seed=3)
    for q in [(3, 0, 3, 0), (5, 3, 1, 0), (5, 5, 5, 5)]:
        full = o.eri_block(wl.mol, *q)
        # w -> inf: long range -> full, short range -> 0
        assert np.abs(o.eri_block(wl.mol, *q, omega=1e7) - full).max() <= 1e-12 * np.abs(full).max()
        assert np.abs(o.eri_block(wl.mol, *q, omega=-1e7)).max() <= 1e-12 * np.abs(full).max()
    # w -> 0 on s shells: erf(w r)/r -> 2w/sqrt(pi), so (ab|cd) -> 2w/sqrt(pi) S_ab S_cd,
    # linear in w (the next term is O(w^3))
    s_sh = [i for i in range(wl.mol.nshell) if wl.mol.l[i] == 0][:3]
    for q in [(s_sh[0], s_sh[1], s_sh[2], s_sh[2]), (s_sh[1], s_sh[1], s_sh[0], s_sh[2])]:
        l1 = o.eri_block(wl.mol, *q, omega=1e-4)[0, 0, 0, 0]
        l2 = o.eri_block(wl.mol, *q, omega=2e-4)[0, 0, 0, 0]
        assert l1 > 0 and abs(l2 - 2 * l1) <= 1e-6 * l1


def test_jk_long_plus_short_is_full():
    wl = synth.workload("c0")
    Q = o.schwarz(wl.mol)
    J0, K0, n0 = o.jk(wl.mol, wl.D, wl.cutoff, Q=Q)
    Jl, Kl, nl = o.jk(wl.mol, wl.D, wl.cutoff, Q=Q, omega=0.4)
    Js, Ks, ns = o.jk(wl.mol, wl.D, wl.cutoff, Q=Q, omega=-0.4)
    assert n0 == nl == ns
    assert np.abs(Jl + Js - J0).max() <= 1e-12 and np.abs(Kl + Ks - K0).max() <= 1e-12
    assert np.abs(Jl).max() > 1e-3 and np.abs(Js).max() > 1e-3
