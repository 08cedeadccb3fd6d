"""Seeded synthetic workloads for the J/K build: water lattices, contracted
Gaussian basis sets and density matrices.

This module defines inputs only.  It holds no integral, screening or
contraction arithmetic, imports nothing from the rest of the package and is
shared by the GPU path, the CPU reference and the benchmark.

Conventions (the interface contract of the library):

* A shell is (l, nprim, atom) with primitive exponents ``exps`` and
  coefficients ``coefs``.  ``coefs`` multiply the *raw* primitive
  ``x^ax y^ay z^az exp(-a r^2)`` (centred on the atom), so all primitive
  normalisation is already folded in: every Cartesian component of a shell
  carries the factor that normalises its x^l component, and the contraction
  is rescaled so that x^l has unit norm.
* Cartesian components follow reversed lexicographic order (xx, xy, xz, yy,
  yz, zz for d), as stated with the definition of the index function in
  Section 2 of the paper.
* Spherical shells are real solid harmonics ordered m = -l..l, except l = 1,
  which stays (x, y, z).
* Coordinates are in bohr.

Workloads (the shapes and value distributions of the paper's benchmarks,
Section 4, with synthetic water lattices standing in for its molecules):

* basis A: split-valence + polarisation, Cartesian (6-31G*-shaped);
* basis B: triple-zeta + double polarisation, spherical (def2-TZVPP-shaped);
* basis C: quadruple-zeta with g shells, spherical (cc-pVQZ-shaped:
  O [5s4p3d2f1g], H [4s3p2d1f]).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903  # CODATA 2018 Bohr radius in angstrom

# (l, nprim, is_core) per shell, per element.
BASIS_A_SHELLS = {
    "O": [(0, 6, True), (0, 3, False), (0, 1, False), (1, 3, False), (1, 1, False), (2, 1, False)],
    "H": [(0, 3, False), (0, 1, False)],
}
BASIS_B_SHELLS = {
    "O": [(0, 6, True), (0, 2, False), (0, 1, False), (0, 1, False), (0, 1, False),
          (1, 4, False), (1, 1, False), (1, 1, False), (2, 1, False), (2, 1, False), (3, 1, False)],
    "H": [(0, 3, False), (0, 1, False), (0, 1, False), (1, 1, False)],
}
BASIS_C_SHELLS = {
    "O": [(0, 6, True), (0, 2, False), (0, 1, False), (0, 1, False), (0, 1, False),
          (1, 4, False), (1, 1, False), (1, 1, False), (1, 1, False),
          (2, 1, False), (2, 1, False), (2, 1, False), (3, 1, False), (3, 1, False), (4, 1, False)],
    "H": [(0, 3, False), (0, 1, False), (0, 1, False), (0, 1, False),
          (1, 1, False), (1, 1, False), (1, 1, False), (2, 1, False), (2, 1, False), (3, 1, False)],
}
BASIS_SEED = {"A": 101, "B": 102, "C": 103}
CORE_RANGE = (0.1, 5.0e3)
VALENCE_RANGE = (0.1, 10.0)

OH_ANGSTROM = 0.96
HOH_DEGREES = 104.5
LATTICE_ANGSTROM = 3.0
JITTER_ANGSTROM = 0.3
OCC_PER_WATER = 5


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nsph(l: int) -> int:
    return 2 * l + 1


def _dfact(n: int) -> float:
    """Double factorial with (-1)!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return float(r)


def _prim_norm(alpha: np.ndarray, l: int) -> np.ndarray:
    """Factor normalising x^l exp(-alpha r^2)."""
    return (2.0 * alpha / math.pi) ** 0.75 * (4.0 * alpha) ** (l / 2.0) / math.sqrt(_dfact(2 * l - 1))


def _contract_norm(alpha: np.ndarray, d: np.ndarray, l: int) -> np.ndarray:
    """Coefficients for raw primitives such that the contracted x^l function
    has unit norm.  Uses the textbook Gaussian moment
    int x^(2l) exp(-s r^2) d^3r = (2l-1)!! / (2s)^l * (pi/s)^(3/2)."""
    c = d * _prim_norm(alpha, l)
    s = alpha[:, None] + alpha[None, :]
    ovl = _dfact(2 * l - 1) / (2.0 * s) ** l * (math.pi / s) ** 1.5
    nrm2 = float(c @ ovl @ c)
    return c / math.sqrt(nrm2)


@dataclasses.dataclass
class BasisTemplate:
    """Exponents and coefficients per element, drawn once per basis name."""
    name: str
    spherical: bool
    shells: dict  # element -> list of (l, exps ndarray, coefs ndarray)


def make_basis(name: str) -> BasisTemplate:
    """Draw basis A, B or C from its fixed seed.

    Exponents: log-uniform on [0.1, 5e3] for the core shell and on [0.1, 10]
    for every other shell, sorted descending.  Raw contraction weights
    U(0.2, 1) (1 for single-primitive shells), then normalised as described
    in the module docstring.
    """
    spec = {"A": BASIS_A_SHELLS, "B": BASIS_B_SHELLS, "C": BASIS_C_SHELLS}[name]
    rng = np.random.default_rng(BASIS_SEED[name])
    shells = {}
    for elem in ("O", "H"):
        out = []
        for (l, npr, core) in spec[elem]:
            lo, hi = CORE_RANGE if core else VALENCE_RANGE
            e = np.exp(rng.uniform(math.log(lo), math.log(hi), size=npr))
            e = np.sort(e)[::-1].copy()
            d = rng.uniform(0.2, 1.0, size=npr) if npr > 1 else np.ones(1)
            out.append((l, e, _contract_norm(e, d, l)))
        shells[elem] = out
    return BasisTemplate(name=name, spherical=(name != "A"), shells=shells)


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def water_lattice(nwater: int, seed) -> tuple[list, np.ndarray]:
    """Atoms (O, H, H per water) of ``nwater`` waters on a cubic lattice.

    Sites are the first ``nwater`` points, x fastest, of the smallest k^3
    cube with k^3 >= nwater, spaced 3.0 A; each O is jittered by
    U(-0.3, 0.3) A per axis and each molecule is given a Haar-random
    rotation about its O.  Returns (elements, coords in bohr [natom, 3]).
    """
    rng = np.random.default_rng(seed)
    k = 1
    while k ** 3 < nwater:
        k += 1
    half = math.radians(HOH_DEGREES) / 2.0
    h_local = OH_ANGSTROM * np.array([[math.sin(half), 0.0, math.cos(half)],
                                      [-math.sin(half), 0.0, math.cos(half)]])
    elems, xyz = [], []
    for s in range(nwater):
        site = np.array([s % k, (s // k) % k, s // (k * k)], dtype=float) * LATTICE_ANGSTROM
        o = site + rng.uniform(-JITTER_ANGSTROM, JITTER_ANGSTROM, size=3)
        rot = _haar_rotation(rng)
        elems += ["O", "H", "H"]
        xyz += [o, o + rot @ h_local[0], o + rot @ h_local[1]]
    return elems, np.asarray(xyz) * ANGSTROM_TO_BOHR


@dataclasses.dataclass
class Molecule:
    """Flat shell arrays in the layout the library's C ABI takes."""
    l: np.ndarray        # int32 [nshell]
    nprim: np.ndarray    # int32 [nshell]
    atom: np.ndarray     # int32 [nshell]
    exps: np.ndarray     # float64 [sum nprim]
    coefs: np.ndarray    # float64 [sum nprim]
    coords: np.ndarray   # float64 [natom, 3] bohr
    spherical: bool
    nwater: int = 0

    @property
    def nshell(self) -> int:
        return int(self.l.size)

    @property
    def natom(self) -> int:
        return int(self.coords.shape[0])

    @property
    def nao(self) -> int:
        f = nsph if self.spherical else ncart
        return int(sum(f(int(x)) for x in self.l))

    @property
    def nao_cart(self) -> int:
        return int(sum(ncart(int(x)) for x in self.l))

    def ao_offsets(self) -> np.ndarray:
        f = nsph if self.spherical else ncart
        sizes = np.array([f(int(x)) for x in self.l], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(sizes)])


def build_molecule(basis: BasisTemplate, elems, coords) -> Molecule:
    l, npr, atom, ex, co = [], [], [], [], []
    for ia, el in enumerate(elems):
        for (ll, e, c) in basis.shells[el]:
            l.append(ll)
            npr.append(e.size)
            atom.append(ia)
            ex.append(e)
            co.append(c)
    return Molecule(l=np.asarray(l, np.int32), nprim=np.asarray(npr, np.int32),
                    atom=np.asarray(atom, np.int32), exps=np.concatenate(ex),
                    coefs=np.concatenate(co), coords=np.ascontiguousarray(coords, dtype=np.float64),
                    spherical=basis.spherical, nwater=sum(1 for e in elems if e == "O"))


def random_density(nao: int, nocc: int, seed, nset: int = 1) -> np.ndarray:
    """[nset, nao, nao] densities D = C C^T, C an orthonormalised Gaussian
    nao x nocc matrix (QR)."""
    rng = np.random.default_rng(seed)
    out = np.empty((nset, nao, nao))
    for s in range(nset):
        c, _ = np.linalg.qr(rng.standard_normal((nao, nocc)))
        out[s] = c @ c.T
    return out


@dataclasses.dataclass
class Workload:
    name: str
    mol: Molecule
    D: np.ndarray  # [nset, nao, nao]
    cutoff: float = 1e-13


# Water counts and basis per workload.  "c3" is mixed precision run on the
# molecules of c1 and c2; "c4" is a list of molecules (see batch_workload).
WORKLOADS = {
    "c0": dict(nwater=3, basis="A", geom_seed=200, dens_seed=300),
    "c1": dict(nwater=64, basis="A", geom_seed=201, dens_seed=301),
    "c2": dict(nwater=32, basis="B", geom_seed=202, dens_seed=302),
    # g shells: 8 waters in the quadruple-zeta-shaped basis C (920 AOs)
    "qz8": dict(nwater=8, basis="C", geom_seed=205, dens_seed=305),
}


def workload(name: str) -> Workload:
    """Single-molecule workloads c0 (3 waters, basis A), c1 (64 waters,
    basis A), c2 (32 waters, basis B) and qz8 (8 waters, basis C, up to g)."""
    spec = WORKLOADS[name]
    basis = make_basis(spec["basis"])
    elems, xyz = water_lattice(spec["nwater"], spec["geom_seed"])
    mol = build_molecule(basis, elems, xyz)
    D = random_density(mol.nao, OCC_PER_WATER * spec["nwater"], spec["dens_seed"])
    return Workload(name=name, mol=mol, D=D)


def small_workload(nwater: int, basis: str, seed: int, nset: int = 1) -> Workload:
    """A water cluster of any size for tests (same recipe, free seed)."""
    b = make_basis(basis)
    elems, xyz = water_lattice(nwater, seed)
    mol = build_molecule(b, elems, xyz)
    D = random_density(mol.nao, OCC_PER_WATER * nwater, seed + 1, nset)
    return Workload(name=f"w{nwater}{basis}s{seed}", mol=mol, D=D)


BATCH_SEED = 400
BATCH_DENS_SEED = 304


def batch_workload(nmol: int = 256, nset: int = 4, seed: int = BATCH_SEED) -> list:
    """Many independent molecules of 1..8 waters (sizes uniform from the
    seed); after a seeded shuffle the first half use basis A and the rest
    basis B.  Each carries ``nset`` densities with 5 occupied orbitals per
    water."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 9, size=nmol)
    order = rng.permutation(nmol)
    which = np.empty(nmol, dtype=object)
    which[order[: nmol // 2]] = "A"
    which[order[nmol // 2:]] = "B"
    bases = {"A": make_basis("A"), "B": make_basis("B")}
    out = []
    for m in range(nmol):
        elems, xyz = water_lattice(int(sizes[m]), [seed, m])
        mol = build_molecule(bases[which[m]], elems, xyz)
        D = random_density(mol.nao, OCC_PER_WATER * int(sizes[m]), [BATCH_DENS_SEED, m], nset)
        out.append(Workload(name=f"b{m}", mol=mol, D=D))
    return out


def uniform_shell_workload(name: str, l: int, nprim: int, exponent: float, nset: int = 1,
                           spherical: bool = False) -> Workload:
    """Every atom of a single-molecule workload's geometry (c1 or c2) gets
    the same one shell: angular momentum ``l`` with ``nprim`` copies of one
    exponent, each weighted 1/nprim, so the contracted function (and hence
    every integral and the screening) is the same for every ``nprim`` while
    the primitive work grows as nprim^4 -- the profiling basis of the
    paper's appendix B micro-benchmarks.  Densities: seeded independently of
    nprim, nset of them, half as many occupied orbitals as atoms."""
    spec = WORKLOADS[name]
    elems, xyz = water_lattice(spec["nwater"], spec["geom_seed"])
    e = np.full(nprim, float(exponent))
    c = _contract_norm(e, np.full(nprim, 1.0 / nprim), l)
    shell = (l, e, c)
    tmpl = BasisTemplate(name=f"uniform-l{l}", spherical=spherical, shells={"O": [shell], "H": [shell]})
    mol = build_molecule(tmpl, elems, xyz)
    D = random_density(mol.nao, max(1, len(elems) // 2), [spec["dens_seed"], l], nset)
    return Workload(name=f"{name}-l{l}-p{nprim}", mol=mol, D=D)
