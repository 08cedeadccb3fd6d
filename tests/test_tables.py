"""CPU checks of the generated constant tables the kernels read: the Rys
fits reproduce the Boys moments (Gauss quadrature exactness), the large-T
limit is the Gauss-Hermite rule, the Boys grid and the two-root moment grid
match the oracle's pinned Boys function, the two-root rule built from the
moment grid the way the kernels build it is exact on F_0..F_3, and the
spherical coefficients match the oracle's independently derived ones."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TAB = os.path.join(ROOT, "paper_2507_09772_amd", "csrc", "tables")


def _arrays():
    meta = open(os.path.join(TAB, "jk_tables_meta.h")).read() + open(os.path.join(TAB, "jk_tables_mom_meta.h")).read()
    data = open(os.path.join(TAB, "jk_tables.h")).read() + open(os.path.join(TAB, "jk_tables_mom.h")).read()
    out = {}
    for m in re.finditer(r"(?:constexpr|const)\s+(?:int32_t|double)\s+(\w+)\[[^\]]*\]\s*=\s*\{([^}]*)\}", meta + data):
        out[m.group(1)] = np.array([float(x) for x in m.group(2).replace("\n", " ").split(",") if x.strip()])
    defs = dict(re.findall(r"#define\s+(\w+)\s+([\d.]+)", meta))
    return out, {k: float(v) for k, v in defs.items()}


@pytest.fixture(scope="module")
def tabs():
    return _arrays()


def rys_cpu(tabs, n, T):
    a, d = tabs
    deg = int(d["JKT_RYS_DEG"])
    nf = 2 * n
    if T < a["jkt_rys_tmax"][n]:
        it = int(T)
        x = 2.0 * (T - it) - 1.0
        base = int(a["jkt_rys_offset"][n]) + it * (deg + 1) * nf
        c = a["jkt_rys_coef"][base: base + (deg + 1) * nf].reshape(deg + 1, nf)
        acc = c[deg].copy()
        for k in range(deg - 1, -1, -1):
            acc = acc * x + c[k]
        return acc[:n], acc[n:]
    off = int(a["jkt_herm_offset"][n])
    return a["jkt_herm_x2"][off:off + n] / T, a["jkt_herm_w"][off:off + n] / np.sqrt(T)


@pytest.mark.parametrize("n", range(1, 10))
def test_rys_fit_moments(tabs, n):
    rng = np.random.default_rng(n)
    Ts = np.concatenate([[0.0, 1e-10, 0.5, 1.0, 7.25, tabs[0]["jkt_rys_tmax"][n] - 1e-9,
                          tabs[0]["jkt_rys_tmax"][n], 200.0], rng.uniform(0, 85, 60)])
    for T in Ts:
        u, w = rys_cpu(tabs, n, float(T))
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0)
        F = o.boys(2 * n - 1, float(T))
        for k in range(2 * n):
            assert abs(np.sum(w * u ** k) - F[k]) <= 3e-14 * F[k], (n, T, k)


@pytest.mark.parametrize("n", [1, 4, 9])
def test_large_T_is_gauss_hermite(tabs, n):
    a, _ = tabs
    off = int(a["jkt_herm_offset"][n])
    x, w = np.polynomial.hermite.hermgauss(2 * n)
    np.testing.assert_allclose(a["jkt_herm_x2"][off:off + n], np.sort(x[x > 0] ** 2), rtol=1e-13)
    np.testing.assert_allclose(np.sort(a["jkt_herm_w"][off:off + n]), np.sort(w[x > 0]), rtol=1e-12)


def test_boys_grid(tabs):
    a, d = tabs
    mmax = int(d["JKT_BOYS_MMAX"])
    dens = d["JKT_BOYS_DENSITY"]
    tab = a["jkt_boys"].reshape(-1, mmax + 1)
    for j in list(range(0, tab.shape[0], 37)) + [tab.shape[0] - 1]:
        F = o.boys(mmax, j / dens)
        np.testing.assert_allclose(tab[j], F, rtol=2e-15)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_c2s_matches_oracle(tabs, l):
    a, _ = tabs
    off = int(a["jkt_c2s_offset"][l])
    nc = (l + 1) * (l + 2) // 2
    T = a["jkt_c2s"][off: off + (2 * l + 1) * nc].reshape(2 * l + 1, nc)
    np.testing.assert_allclose(T, o.c2s(l), atol=1e-12)


def test_moment_grid(tabs):
    """Rows [e^-T_j, F_3(T_j), ..., F_9(T_j)] at T_j = j / density."""
    a, d = tabs
    cols = int(d["JKT_MOM_COLS"])
    m0 = int(d["JKT_MOM_M0"])
    dens = d["JKT_MOM_DENSITY"]
    tab = a["jkt_mom"].reshape(-1, cols)
    assert tab.shape[0] == int(d["JKT_MOM_NT"]) and (tab.shape[0] - 1) / dens == d["JKT_MOM_TMAX"]
    for j in list(range(0, tab.shape[0], 29)) + [tab.shape[0] - 1]:
        T = j / dens
        F = o.boys(m0 + cols - 2, T)
        assert abs(tab[j, 0] - np.exp(-T)) <= 2e-15 * np.exp(-T)
        np.testing.assert_allclose(tab[j, 1:], F[m0:], rtol=2e-15)


def _two_root_rule(tabs, T):
    """The two-point rule as the kernels form it from the moment grid:
    Taylor expansions of F_3 and exp about the nearest grid point, downward
    recursion to F_0, closed-form nodes and weights; the Gauss-Hermite
    limit beyond the grid."""
    a, d = tabs
    cols = int(d["JKT_MOM_COLS"])
    if T >= d["JKT_MOM_TMAX"]:
        rt = 1.0 / np.sqrt(T)
        return a["jkt_mom_hx2"] * rt * rt, a["jkt_mom_hw"] * rt
    j = int(T * d["JKT_MOM_DENSITY"] + 0.5)
    row = a["jkt_mom"].reshape(-1, cols)[j]
    dd = j / d["JKT_MOM_DENSITY"] - T
    f3, ed = row[cols - 1], 1.0
    for k in range(cols - 2, 0, -1):
        f3 = row[k] + f3 * dd / k
        ed = 1.0 + ed * dd / k
    ex = row[0] * ed
    f2 = (2 * T * f3 + ex) / 5
    f1 = (2 * T * f2 + ex) / 3
    f0 = 2 * T * f1 + ex
    det = f1 * f1 - f0 * f2
    aa = (f0 * f3 - f1 * f2) / det
    bb = (f2 * f2 - f1 * f3) / det
    up = 0.5 * (np.sqrt(aa * aa - 4 * bb) - aa)
    um = bb / up
    wp = (f1 - um * f0) / (up - um)
    return np.array([um, up]), np.array([f0 - wp, wp])


def test_two_root_rule_from_moments(tabs):
    rng = np.random.default_rng(7)
    Ts = [0.0, 1e-12, 1e-6, 0.015625, 0.5, 1.0, 7.3, 20.0, 39.99, 40.0, 45.98, 46.0, 60.0, 1e3]
    for T in Ts + list(rng.uniform(0, 50, 300)):
        u, w = _two_root_rule(tabs, float(T))
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0), T
        F = o.boys(3, float(T))
        for k in range(4):
            assert abs(np.sum(w * u ** k) - F[k]) <= 3e-14 * F[k], (T, k)
