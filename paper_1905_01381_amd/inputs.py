"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and lays out arrays; it holds none of the
method's arithmetic (no integrals, no normalization, no density contraction).
Each consumer turns the raw orbitals into an S-orthonormal density with its
own overlap matrix.

Recipe (fixed draw order per molecule: geometry, then coefficients, then
orbitals; ``numpy.random.default_rng(seed)``):

* Geometry: cubic lattice of constant 1.8 bohr; the first N sites of the
  smallest m**3 >= N cube in ``itertools.product`` order; every coordinate is
  jittered uniformly by +-0.2 bohr and the whole jitter is redrawn until the
  minimum interatomic distance is >= 1.4 bohr.
* Shells: every atom carries the same list of angular momenta.  For each l the
  exponents are 3*n_l values spaced geometrically from ``hi`` down to ``lo``
  and handed out as consecutive triples, tightest triple first.  Contraction
  coefficients are U(0.1, 1), one triple per shell in atom-major order.
* Orbitals: Q from the QR factorization of a standard-normal matrix (complex
  normal for two-component spinors); callers form C = S^{-1/2} Q.
* Spherical variant (``spherical=True``): the same draws, with every d shell
  taken as spherical (5 functions instead of 6): 3s2p1d gives 14 functions
  per atom.
* General-contraction variant (``general_molecule``): per atom, the n_l
  shells of one l become one generally contracted shell with n_l
  contractions over m = min(3 n_l, 8) geometric exponents from ``hi`` down
  to ``lo``.  Contraction k weights its own window of primitives
  [k m / n_l, (k+1) m / n_l) with U(0.1, 1) and every other primitive with
  U(0, 0.05), so that the contractions share every exponent yet stay far
  from linearly dependent.  Draw order per atom and shell: geometry first,
  then the n_l x m coefficients row by row, then the orbitals.

The contracted Gaussian basis itself follows the paper's LCAO setting
(Introduction: contracted Gaussian-type orbital expansions, segmented
contraction).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

LATTICE = 1.8
JITTER = 0.2
MIN_DIST = 1.4
NPRIM = 3


@dataclass
class Molecule:
    """Raw synthetic molecule: atoms, shells (center, l, exponents, raw
    coefficients) in atom-major order."""

    atoms: np.ndarray                 # [natom, 3] bohr
    charges: np.ndarray               # [natom]
    shell_atom: np.ndarray            # [nshell] int
    shell_l: np.ndarray               # [nshell] int
    shell_xyz: np.ndarray             # [nshell, 3]
    nprim: np.ndarray                 # [nshell] int
    alpha: np.ndarray                 # [sum nprim]
    coef: np.ndarray                  # [sum nprim * ncontr] raw (unnormalized), contraction-major per shell
    rng_state: dict = field(default_factory=dict, repr=False)
    ncontr: np.ndarray | None = None  # [nshell] contractions per shell (None: all 1)
    pure: np.ndarray | None = None    # [nshell] 1 = spherical shell (None: all Cartesian)

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        n = 0
        for s, l in enumerate(self.shell_l):
            nf = 2 * l + 1 if (self.pure is not None and self.pure[s] and l >= 2) else (l + 1) * (l + 2) // 2
            n += nf * (1 if self.ncontr is None else int(self.ncontr[s]))
        return int(n)

    def as_spherical(self) -> "Molecule":
        """The same shells with every d and f shell spherical."""
        pure = (np.asarray(self.shell_l) >= 2).astype(np.int32)
        nco = self.ncontr if self.ncontr is not None else np.ones(self.nshell, np.int32)
        return Molecule(self.atoms, self.charges, self.shell_atom, self.shell_l, self.shell_xyz, self.nprim,
                        self.alpha, self.coef, self.rng_state, nco, pure)


def lattice_geometry(natom: int, rng: np.random.Generator) -> np.ndarray:
    m = 1
    while m ** 3 < natom:
        m += 1
    sites = np.array(list(itertools.product(range(m), repeat=3))[:natom], dtype=np.float64) * LATTICE
    while True:
        xyz = sites + rng.uniform(-JITTER, JITTER, size=sites.shape)
        if natom < 2:
            return xyz
        d = np.sqrt(((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(-1))
        d[np.diag_indices(natom)] = np.inf
        if d.min() >= MIN_DIST:
            return xyz


def shell_exponents(ls: list[int], lo: float, hi: float) -> list[np.ndarray]:
    """Per-shell exponent triples for one atom (same for every atom)."""
    out: list[np.ndarray | None] = [None] * len(ls)
    for l in sorted(set(ls)):
        idx = [i for i, x in enumerate(ls) if x == l]
        vals = np.geomspace(hi, lo, NPRIM * len(idx))
        for k, i in enumerate(idx):
            out[i] = vals[NPRIM * k: NPRIM * (k + 1)].copy()
    return out  # type: ignore[return-value]


def make_molecule(natom: int, ls: list[int], lo: float, hi: float,
                  rng: np.random.Generator, charge: float = 1.0) -> Molecule:
    atoms = lattice_geometry(natom, rng)
    exps = shell_exponents(ls, lo, hi)
    nsh = natom * len(ls)
    coef = rng.uniform(0.1, 1.0, size=(nsh, NPRIM))
    shell_atom = np.repeat(np.arange(natom), len(ls))
    shell_l = np.tile(np.array(ls, dtype=np.int32), natom)
    alpha = np.concatenate([exps[i % len(ls)] for i in range(nsh)])
    return Molecule(
        atoms=atoms,
        charges=np.full(natom, charge),
        shell_atom=shell_atom.astype(np.int32),
        shell_l=shell_l.astype(np.int32),
        shell_xyz=atoms[shell_atom].copy(),
        nprim=np.full(nsh, NPRIM, dtype=np.int32),
        alpha=alpha.astype(np.float64),
        coef=coef.reshape(-1).astype(np.float64),
    )


def general_molecule(natom: int, ls: list[int], lo: float, hi: float, rng: np.random.Generator,
                     spherical: bool = True, charge: float = 1.0) -> Molecule:
    """The recipe's atoms with the n_l shells of each l merged into one
    generally contracted shell (n_l contractions over min(3 n_l, 8)
    exponents); d and f shells spherical if ``spherical``."""
    atoms = lattice_geometry(natom, rng)
    counts = {l: ls.count(l) for l in sorted(set(ls))}
    per_atom = []
    for l, n in counts.items():
        per_atom.append((l, min(NPRIM * n, 8), n, np.geomspace(hi, lo, min(NPRIM * n, 8))))
    sh_atom, sh_l, npr, nco, alpha, coef = [], [], [], [], [], []
    for a in range(natom):
        for l, npl, nc, ex in per_atom:
            sh_atom.append(a)
            sh_l.append(l)
            npr.append(npl)
            nco.append(nc)
            alpha.append(ex)
            for k in range(nc):
                own = np.zeros(npl, bool)
                own[k * npl // nc:(k + 1) * npl // nc] = True
                coef.append(np.where(own, rng.uniform(0.1, 1.0, npl), rng.uniform(0.0, 0.05, npl)))
    sh_atom = np.array(sh_atom, np.int32)
    sh_l = np.array(sh_l, np.int32)
    return Molecule(atoms=atoms, charges=np.full(natom, charge), shell_atom=sh_atom, shell_l=sh_l,
                    shell_xyz=atoms[sh_atom].copy(), nprim=np.array(npr, np.int32),
                    alpha=np.concatenate(alpha), coef=np.concatenate(coef), ncontr=np.array(nco, np.int32),
                    pure=((sh_l >= 2) & spherical).astype(np.int32))


def random_orbitals(nbf: int, nocc: int, rng: np.random.Generator, complex_: bool = False) -> np.ndarray:
    """Orthonormal columns Q (nbf x nocc) from QR of a (complex) normal matrix."""
    if complex_:
        z = rng.standard_normal((nbf, nocc)) + 1j * rng.standard_normal((nbf, nocc))
    else:
        z = rng.standard_normal((nbf, nocc))
    q, _ = np.linalg.qr(z)
    return q


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
SHELLS_2S1P = [0, 0, 1]
SHELLS_3S2P1D = [0, 0, 0, 1, 1, 2]
# a triple-zeta-like polarized atom with one f shell (35 Cartesian / 30
# spherical functions per atom), for the classes above d
SHELLS_4S3P2D1F = [0, 0, 0, 0, 1, 1, 1, 2, 2, 3]


@dataclass
class Workload:
    name: str
    mol: Molecule
    orbitals: np.ndarray     # Q, orthonormal columns
    two_component: bool
    nocc: int


def c1(seed: int = 0) -> Workload:
    """6 atoms, 2s1p per atom (exponents 0.15..30), nbf = 30, 5 real orbitals."""
    rng = np.random.default_rng(seed)
    mol = make_molecule(6, SHELLS_2S1P, 0.15, 30.0, rng)
    q = random_orbitals(mol.nbf, 5, rng)
    return Workload("C1", mol, q, False, 5)


def c2(seed: int = 0, natom: int = 40, nocc: int = 60, spherical: bool = False) -> Workload:
    """40 atoms, 3s2p1d per atom (exponents 0.1..1e3), nbf = 600 Cartesian
    (560 with spherical d); 60 complex spinors in the 2*nbf spin-blocked
    space."""
    rng = np.random.default_rng(seed)
    mol = make_molecule(natom, SHELLS_3S2P1D, 0.1, 1.0e3, rng)
    if spherical:
        mol = mol.as_spherical()
    q = random_orbitals(2 * mol.nbf, nocc, rng, complex_=True)
    return Workload("C2", mol, q, True, nocc)


def c3(seed: int = 0, natom: int = 200, nocc: int = 400) -> Workload:
    """200 atoms, 3s2p1d, nbf = 3000, 400 real orbitals."""
    rng = np.random.default_rng(seed)
    mol = make_molecule(natom, SHELLS_3S2P1D, 0.1, 1.0e3, rng)
    q = random_orbitals(mol.nbf, nocc, rng)
    return Workload("C3", mol, q, False, nocc)


def c4_sizes(seed: int = 0, nmol: int = 64) -> np.ndarray:
    return np.random.default_rng(seed).integers(10, 121, size=nmol)


def c4_molecule(i: int, seed: int = 0, nmol: int = 64) -> Workload:
    """Molecule i of the batch: c4_sizes()[i] atoms drawn from
    default_rng([seed, i]); nocc_i = 2 N_i."""
    n = int(c4_sizes(seed, nmol)[i])
    rng = np.random.default_rng([seed, i])
    mol = make_molecule(n, SHELLS_3S2P1D, 0.1, 1.0e3, rng)
    q = random_orbitals(mol.nbf, 2 * n, rng)
    return Workload(f"C4[{i}]", mol, q, False, 2 * n)


def c4(seed: int = 0, nmol: int = 64) -> list[Workload]:
    """64 molecules of U{10..120} atoms (see c4_molecule)."""
    return [c4_molecule(i, seed, nmol) for i in range(nmol)]


def c5(seed: int = 0, natom: int = 60) -> Workload:
    """60 atoms of nuclear charge 1, 3s2p1d, nbf = 900, 30 doubly occupied
    orbitals (the orbitals here only seed the ground-state search)."""
    rng = np.random.default_rng(seed)
    mol = make_molecule(natom, SHELLS_3S2P1D, 0.1, 1.0e3, rng)
    q = random_orbitals(mol.nbf, natom // 2, rng)
    return Workload("C5", mol, q, False, natom // 2)


def small(natom: int, ls: list[int], seed: int = 0, nocc: int | None = None,
          lo: float = 0.1, hi: float = 1.0e3, complex_: bool = False, spherical: bool = False,
          general: bool = False) -> Workload:
    """A reduced molecule with the same recipe (for parity at oracle-sized
    inputs); ``spherical``: d and f shells spherical; ``general``: the
    general contraction variant."""
    rng = np.random.default_rng(seed)
    if general:
        mol = general_molecule(natom, ls, lo, hi, rng, spherical=spherical)
    else:
        mol = make_molecule(natom, ls, lo, hi, rng)
        if spherical:
            mol = mol.as_spherical()
    n = mol.nbf
    if nocc is None:
        nocc = max(1, n // 4)
    q = random_orbitals(2 * n if complex_ else n, nocc, rng, complex_=complex_)
    return Workload(f"small{natom}", mol, q, complex_, nocc)


def random_symmetric(n: int, rng: np.random.Generator, sign: int = 1) -> np.ndarray:
    """Dense random (anti)symmetric matrix, used for the antisymmetric and
    multi-density parity cases."""
    a = rng.standard_normal((n, n))
    return 0.5 * (a + sign * a.T)
