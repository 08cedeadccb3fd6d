"""Offline generator of the constant tables the HIP kernels read.

Run ``python -m paper_2507_09772_amd.tablegen`` to rewrite
``csrc/tables/jk_tables.h``.  It needs mpmath and takes a few minutes.

Tables (all derived here from their mathematical definitions):

* Rys roots and weights (Section 2, eq. rys1).  For n roots and a given T the
  quadrature nodes u_i = t_i^2 in (0, 1) and weights w_i satisfy
  sum_i w_i u_i^k = F_k(T) for k = 0..2n-1, F_k the Boys function.  They are
  computed at 50 significant digits from the moments (Chebyshev algorithm
  to the Jacobi matrix, then its eigen-decomposition) and fitted by
  polynomials of degree ``DEG`` on intervals of width ``H[n]`` covering
  [0, TMAX[n]).  Each interval stores, per function (u_1..u_n, w_1..w_n),
  power-series coefficients in x = 2 (T - T_lo) / H - 1, stored
  degree-major ([degree][u_1..u_n, w_1..w_n]) so one Horner step reads
  all 2n functions of the interval contiguously.
  Beyond TMAX[n] the kernels use the large-T limit u_i = x_i^2 / T,
  w_i = W_i / sqrt(T), with x_i > 0 the nodes and W_i the weights of the
  2n-point Gauss-Hermite rule; TMAX[n] is where that limit reproduces every
  moment to 1e-16 relative.
* Boys function grid: F_m(T_j) on T_j = j / BOYS_DENSITY for the Taylor
  expansion F_m(T_j + d) = sum_k F_(m+k)(T_j) (-d)^k / k!.
* Moment grid for the two-root rule: e^(-T_j) and F_3..F_9 at the same
  T_j, up to the point where the Gauss-Hermite limit of n = 2 takes over.
  The kernels expand F_3 and e^(-T) about the nearest T_j, recover
  F_2, F_1, F_0 by downward recursion and solve the two-point Gauss rule of
  the moments F_0..F_3 in closed form.
* Real solid harmonic coefficients (spherical <-> Cartesian), obtained by a
  least-squares projection of scipy's spherical harmonics onto monomials and
  normalised with the monomial overlap in units of the x^l norm.
"""
from __future__ import annotations

import math
import os
import sys
from multiprocessing import Pool

import numpy as np

NMAX = 9            # roots: (gg|gg) needs 9
DEG = 13            # polynomial degree per interval
BOYS_DENSITY = 32   # grid points per unit T
BOYS_TMAX = 40.0    # beyond: F_0 = sqrt(pi/T)/2 and upward recursion
BOYS_MMAX = 8       # highest tabulated order (F_1 with 7 Taylor terms)
DPS = 50
LMAX = 4

MOM_M0 = 3          # first tabulated order of the moment grid
MOM_TERMS = 7       # Taylor terms of F_3 and of exp
MOM_TMAX = 46.0     # = the n = 2 Gauss-Hermite switch point (tmax_for(2))

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tables", "jk_tables.h")


def _mp():
    import mpmath
    mpmath.mp.dps = DPS
    return mpmath


def boys_mp(kmax, T):
    """F_0..F_kmax at T in mpmath precision (1F1 at kmax, downward recursion)."""
    mp = _mp()
    T = mp.mpf(T)
    F = [None] * (kmax + 1)
    F[kmax] = mp.hyp1f1(kmax + mp.mpf(1) / 2, kmax + mp.mpf(3) / 2, -T) / (2 * kmax + 1)
    e = mp.exp(-T)
    for k in range(kmax - 1, -1, -1):
        F[k] = (2 * T * F[k + 1] + e) / (2 * k + 1)
    return F


def rys_mp(n, T):
    """n-point Rys nodes (t^2) and weights at T, as mpmath numbers."""
    mp = _mp()
    mu = boys_mp(2 * n - 1, T)
    # Chebyshev algorithm: moments -> three-term recurrence (a_k, b_k)
    a = [mp.mpf(0)] * n
    b = [mp.mpf(0)] * n
    sig_prev = [mp.mpf(0)] * (2 * n)
    sig = list(mu)
    a[0] = mu[1] / mu[0]
    b[0] = mu[0]
    for k in range(1, n):
        new = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            new[l] = sig[l + 1] - a[k - 1] * sig[l] - b[k - 1] * sig_prev[l]
        a[k] = new[k + 1] / new[k] - sig[k] / sig[k - 1]
        b[k] = new[k] / sig[k - 1]
        sig_prev, sig = sig, new
    Jm = mp.matrix(n, n)
    for i in range(n):
        Jm[i, i] = a[i]
        if i + 1 < n:
            Jm[i, i + 1] = Jm[i + 1, i] = mp.sqrt(b[i + 1])
    E, Q = mp.eigsy(Jm)
    nodes = [E[i] for i in range(n)]
    wts = [b[0] * Q[0, i] ** 2 for i in range(n)]
    order = sorted(range(n), key=lambda i: nodes[i])
    return [nodes[i] for i in order], [wts[i] for i in order]


def hermite_half(n):
    """Positive nodes x_i and weights W_i of the 2n-point Gauss-Hermite rule,
    ascending, at mpmath precision (Newton-polished from numpy's)."""
    mp = _mp()
    x0, w0 = np.polynomial.hermite.hermgauss(2 * n)
    out_x, out_w = [], []
    for x in x0[x0 > 0]:
        x = mp.mpf(float(x))
        for _ in range(60):
            # H_2n(x) and derivative by recurrence
            h0, h1 = mp.mpf(1), 2 * x
            for k in range(1, 2 * n):
                h0, h1 = h1, 2 * x * h1 - 2 * k * h0
            d = 2 * (2 * n) * h0
            step = h1 / d
            x -= step
            if abs(step) < mp.mpf(10) ** (-DPS + 5):
                break
        h0, h1 = mp.mpf(1), 2 * x
        for k in range(1, 2 * n - 1):
            h0, h1 = h1, 2 * x * h1 - 2 * k * h0
        # W = 2^(N-1) N! sqrt(pi) / (N^2 H_(N-1)(x)^2), N = 2n
        N = 2 * n
        W = mp.mpf(2) ** (N - 1) * mp.factorial(N) * mp.sqrt(mp.pi) / (N * N * h1 ** 2)
        out_x.append(x)
        out_w.append(W)
    order = sorted(range(n), key=lambda i: out_x[i])
    return [out_x[i] for i in order], [out_w[i] for i in order]


def tmax_for(n, tol=1e-16):
    """Smallest integer T beyond which the Gauss-Hermite limit reproduces
    F_0..F_(2n-1) to relative ``tol``."""
    mp = _mp()
    xs, ws = hermite_half(n)
    T = 5
    while True:
        F = boys_mp(2 * n - 1, T)
        ok = True
        for k in range(2 * n):
            approx = sum(ws[i] * xs[i] ** (2 * k) for i in range(n)) / mp.mpf(T) ** (k + mp.mpf(1) / 2)
            if abs(approx - F[k]) > tol * F[k]:
                ok = False
                break
        if ok:
            return T
        T += 1


def _cheb_nodes(deg):
    k = np.arange(deg + 1)
    return np.cos(np.pi * (k + 0.5) / (deg + 1))


def _fit_interval(args):
    """Power-series coefficients (in x in [-1, 1]) of u_i and w_i on
    [lo, lo+h], from values at Chebyshev nodes (interpolation)."""
    n, lo, h = args
    mp = _mp()
    xs = _cheb_nodes(DEG)
    vals = []
    for x in xs:
        T = mp.mpf(lo) + (mp.mpf(float(x)) + 1) * mp.mpf(h) / 2
        u, w = rys_mp(n, T)
        vals.append(u + w)
    # solve the Vandermonde system in mpmath (well posed at Chebyshev nodes, deg 13)
    V = mp.matrix(DEG + 1, DEG + 1)
    for r, x in enumerate(xs):
        for c in range(DEG + 1):
            V[r, c] = mp.mpf(float(x)) ** c
    coefs = []
    for f in range(2 * n):
        rhs = mp.matrix([vals[r][f] for r in range(DEG + 1)])
        sol = mp.lu_solve(V, rhs)
        coefs.append([float(sol[c]) for c in range(DEG + 1)])
    # check at off-node points, evaluating the stored doubles like the kernel does
    err = 0.0
    for x in (-0.97, -0.5, -0.11, 0.31, 0.77, 0.999):
        T = mp.mpf(lo) + (mp.mpf(x) + 1) * mp.mpf(h) / 2
        u, w = rys_mp(n, T)
        ref = u + w
        for f in range(2 * n):
            acc = 0.0
            for c in reversed(coefs[f]):
                acc = acc * x + c
            err = max(err, abs(acc - float(ref[f])) / abs(float(ref[f])))
    return coefs, err


# interval widths per root count (chosen so that the fits reach ~1e-15)
H = {1: 1.0, 2: 1.0, 3: 1.0, 4: 1.0, 5: 1.0, 6: 1.0, 7: 1.0, 8: 1.0, 9: 1.0}


def rys_tables(procs=8, nmax=NMAX):
    out = {}
    with Pool(procs) as pool:
        tm = pool.map(tmax_for, range(1, nmax + 1))
        for n in range(1, nmax + 1):
            tmax = tm[n - 1]
            h = H[n]
            nint = int(math.ceil(tmax / h))
            res = pool.map(_fit_interval, [(n, i * h, h) for i in range(nint)])
            coefs = [r[0] for r in res]
            err = max(r[1] for r in res)
            xs, ws = hermite_half(n)
            out[n] = dict(tmax=nint * h, h=h, nint=nint, coefs=coefs, err=err,
                          hx=[float(x) ** 2 for x in xs], hw=[float(w) for w in ws])
            print(f"rys n={n}: T<{nint * h}, {nint} intervals, max rel err {err:.2e}", file=sys.stderr)
    return out


def boys_table():
    nt = int(BOYS_TMAX * BOYS_DENSITY) + 1
    tab = np.zeros((nt, BOYS_MMAX + 1))
    for j in range(nt):
        F = boys_mp(BOYS_MMAX, mp_frac(j, BOYS_DENSITY))
        tab[j] = [float(f) for f in F]
    return tab


def moment_table():
    """Rows [e^(-T_j), F_3(T_j), ..., F_9(T_j)], T_j = j / BOYS_DENSITY."""
    mp = _mp()
    nt = int(MOM_TMAX * BOYS_DENSITY) + 1
    tab = np.zeros((nt, 1 + MOM_TERMS))
    for j in range(nt):
        T = mp_frac(j, BOYS_DENSITY)
        F = boys_mp(MOM_M0 + MOM_TERMS - 1, T)
        tab[j] = [float(mp.exp(-T))] + [float(f) for f in F[MOM_M0:]]
    return tab


def write_moment_header(mom, path=None):
    """jk_tables_mom_meta.h (sizes, for device code) and jk_tables_mom.h
    (the grid, for the host copy)."""
    d = os.path.dirname(path or OUT)
    meta = ["/* Generated by paper_2507_09772_amd/tablegen.py -- do not edit. */", "#pragma once", "",
            f"#define JKT_MOM_M0 {MOM_M0}", f"#define JKT_MOM_TERMS {MOM_TERMS}",
            f"#define JKT_MOM_COLS {mom.shape[1]}", f"#define JKT_MOM_NT {mom.shape[0]}",
            f"#define JKT_MOM_DENSITY {BOYS_DENSITY}", f"#define JKT_MOM_TMAX {MOM_TMAX!r}", ""]
    # the n = 2 large-T limit as constants (no table load on that branch)
    xs, ws = hermite_half(2)
    meta.append("static constexpr double jkt_mom_hx2[2] = {" + ", ".join(repr(float(x) ** 2) for x in xs) + "};")
    meta.append("static constexpr double jkt_mom_hw[2] = {" + ", ".join(repr(float(w)) for w in ws) + "};")
    data = ["/* Generated by paper_2507_09772_amd/tablegen.py -- do not edit. */", "#pragma once",
            '#include "jk_tables_mom_meta.h"', "",
            "static const double jkt_mom[JKT_MOM_NT * JKT_MOM_COLS] = {", _fmt(mom.ravel()), "};"]
    with open(os.path.join(d, "jk_tables_mom_meta.h"), "w") as f:
        f.write("\n".join(meta) + "\n")
    with open(os.path.join(d, "jk_tables_mom.h"), "w") as f:
        f.write("\n".join(data) + "\n")


def mp_frac(a, b):
    mp = _mp()
    return mp.mpf(a) / b


def c2s_tables(lmax=LMAX):
    """Rows m = -l..l (l = 1: x, y, z) over Cartesian monomials."""
    from scipy import special
    out = {}
    for l in range(lmax + 1):
        carts = [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]
        if l == 1:
            out[l] = np.eye(3)
            continue
        rng = np.random.default_rng(1234 + l)
        pts = rng.standard_normal((60 * len(carts), 3))
        r = np.linalg.norm(pts, axis=1)
        theta = np.arccos(np.clip(pts[:, 2] / r, -1, 1))
        phi = np.arctan2(pts[:, 1], pts[:, 0])
        A = np.stack([pts[:, 0] ** c[0] * pts[:, 1] ** c[1] * pts[:, 2] ** c[2] for c in carts], axis=1)

        def df(k):
            v = 1
            while k > 1:
                v *= k
                k -= 2
            return v
        S = np.zeros((len(carts), len(carts)))
        for i, a in enumerate(carts):
            for j, b in enumerate(carts):
                s = [a[k] + b[k] for k in range(3)]
                if all(x % 2 == 0 for x in s):
                    S[i, j] = df(s[0] - 1) * df(s[1] - 1) * df(s[2] - 1) / df(2 * l - 1)
        T = np.zeros((2 * l + 1, len(carts)))
        for m in range(-l, l + 1):
            Y = special.sph_harm_y(l, abs(m), theta, phi)
            y = (Y.real if m >= 0 else Y.imag) * r ** l
            c, *_ = np.linalg.lstsq(A, y, rcond=None)
            c[np.abs(c) < 1e-12 * np.abs(c).max()] = 0.0
            c /= math.sqrt(c @ S @ c)
            lead = (abs(m), 0, l - abs(m)) if m >= 0 else (abs(m) - 1, 1, l - abs(m))
            if c[carts.index(lead)] < 0:
                c = -c
            T[m + l] = c
        out[l] = T
    return out


def _fmt(vals, per_line=4):
    s = []
    for i in range(0, len(vals), per_line):
        s.append("    " + ", ".join(repr(float(v)) for v in vals[i:i + per_line]) + ",")
    return "\n".join(s)


def write_header(rys, boys, c2s, path=OUT):
    """Two headers: jk_tables_meta.h (sizes and per-n metadata as constexpr,
    for device code) and jk_tables.h (the bulk arrays, for the host copy)."""
    meta = ["/* Generated by paper_2507_09772_amd/tablegen.py -- do not edit. */",
            "#pragma once", "#include <stdint.h>", "",
            f"#define JKT_RYS_NMAX {max(rys)}", f"#define JKT_RYS_DEG {DEG}",
            f"#define JKT_BOYS_DENSITY {BOYS_DENSITY}", f"#define JKT_BOYS_MMAX {BOYS_MMAX}",
            f"#define JKT_BOYS_NT {boys.shape[0]}", f"#define JKT_BOYS_TMAX {BOYS_TMAX!r}",
            f"#define JKT_C2S_LMAX {max(c2s)}", ""]
    data = ["/* Generated by paper_2507_09772_amd/tablegen.py -- do not edit. */",
            "#pragma once", '#include "jk_tables_meta.h"', ""]
    flat, offs = [], []
    for n in sorted(rys):
        offs.append(len(flat))
        for iv in rys[n]["coefs"]:
            # degree-major inside an interval: [deg][u_1..u_n, w_1..w_n]
            for c in range(DEG + 1):
                flat.extend(iv[f][c] for f in range(2 * n))
    meta.append("static constexpr int32_t jkt_rys_offset[JKT_RYS_NMAX + 1] = {0, " + ", ".join(map(str, offs)) + "};")
    meta.append("static constexpr int32_t jkt_rys_nint[JKT_RYS_NMAX + 1] = {0, " + ", ".join(str(rys[n]["nint"]) for n in sorted(rys)) + "};")
    meta.append("static constexpr double jkt_rys_h[JKT_RYS_NMAX + 1] = {0.0, " + ", ".join(repr(rys[n]["h"]) for n in sorted(rys)) + "};")
    meta.append("static constexpr double jkt_rys_tmax[JKT_RYS_NMAX + 1] = {0.0, " + ", ".join(repr(rys[n]["tmax"]) for n in sorted(rys)) + "};")
    meta.append(f"#define JKT_RYS_NCOEF {len(flat)}")
    data.append("static const double jkt_rys_coef[JKT_RYS_NCOEF] = {")
    data.append(_fmt(flat))
    data.append("};")
    hx, hw, hoff = [], [], []
    for n in sorted(rys):
        hoff.append(len(hx))
        hx.extend(rys[n]["hx"])
        hw.extend(rys[n]["hw"])
    meta.append("static constexpr int32_t jkt_herm_offset[JKT_RYS_NMAX + 1] = {0, " + ", ".join(map(str, hoff)) + "};")
    meta.append(f"#define JKT_HERM_N {len(hx)}")
    data.append("static const double jkt_herm_x2[JKT_HERM_N] = {")
    data.append(_fmt(hx))
    data.append("};")
    data.append("static const double jkt_herm_w[JKT_HERM_N] = {")
    data.append(_fmt(hw))
    data.append("};")
    data.append(f"static const double jkt_boys[{boys.size}] = {{")
    data.append(_fmt(boys.ravel()))
    data.append("};")
    flat, offs = [], []
    for l in sorted(c2s):
        offs.append(len(flat))
        flat.extend(c2s[l].ravel())
    meta.append("static constexpr int32_t jkt_c2s_offset[JKT_C2S_LMAX + 1] = {" + ", ".join(map(str, offs)) + "};")
    meta.append(f"#define JKT_C2S_N {len(flat)}")
    data.append("static const double jkt_c2s[JKT_C2S_N] = {")
    data.append(_fmt(flat))
    data.append("};")
    errs = {n: rys[n]["err"] for n in rys}
    meta.append("/* max relative fit error per n (off-node checks): " +
                ", ".join(f"{n}:{e:.1e}" for n, e in sorted(errs.items())) + " */")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(os.path.join(os.path.dirname(path), "jk_tables_meta.h"), "w") as f:
        f.write("\n".join(meta) + "\n")
    with open(path, "w") as f:
        f.write("\n".join(data) + "\n")


def main():
    if "--moments" in sys.argv[1:]:
        # the moment grid alone (seconds)
        write_moment_header(moment_table())
        print("wrote moment grid", file=sys.stderr)
        return
    write_moment_header(moment_table())
    nmax = int(sys.argv[1]) if len(sys.argv) > 1 else NMAX
    rys = rys_tables(nmax=nmax)
    boys = boys_table()
    c2s = c2s_tables()
    write_header(rys, boys, c2s)
    print("wrote", OUT, file=sys.stderr)


if __name__ == "__main__":
    main()
