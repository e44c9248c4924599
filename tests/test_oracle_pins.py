"""Pins of the CPU oracle against facts other than itself (no GPU).

Boys function: F_m(0) = 1/(2m+1); F_0(T) = sqrt(pi/T) erf(sqrt T)/2; the
large-T asymptote; the recursion identity; mpmath 40-digit quadrature.
ERIs: the analytic (ss|ss) formula; brute-force Gauss-Hermite x adaptive-t
quadrature of 1/r12 for primitives up to (dd|dd) components; 8-fold
permutational symmetry; the Schwarz inequality.
Basis: unit self-overlap of every contracted Cartesian function by quadrature;
the overlap matrix by quadrature.
J/K: the canonical-quartet build equals the plain definition; the plain
definition equals an einsum over the full ERI tensor; single-orbital
Tr(PJ) = Tr(PK); translation and 90-degree rotation invariance; signs.
"""
import itertools

import mpmath
import numpy as np
import pytest
from scipy.special import erf

import oracle
from paper_1905_01381_amd import inputs
from tests import quad

mpmath.mp.dps = 40


# ---------------------------------------------------------------- Boys
@pytest.mark.parametrize("m", range(0, 13))
def test_boys_at_zero(m):
    assert oracle.boys(m, 0.0) == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)


@pytest.mark.parametrize("T", [1e-8, 1e-3, 0.3, 1.0, 5.0, 17.5, 35.9, 49.9, 50.1, 80.0, 300.0])
def test_boys_f0_erf(T):
    ref = 0.5 * np.sqrt(np.pi / T) * erf(np.sqrt(T))
    assert oracle.boys(0, T) == pytest.approx(ref, rel=2e-15)


def _boys_mp(m, T):
    f = lambda t: t ** (2 * m) * mpmath.exp(-T * t * t)
    return mpmath.quad(f, [0, 0.25, 0.5, 0.75, 1])


@pytest.mark.parametrize("m,T", list(itertools.product([0, 1, 3, 5, 8, 11], [0.05, 0.7, 2.5, 9.0, 21.0, 36.0, 45.0, 60.0])))
def test_boys_mpmath_quadrature(m, T):
    ref = float(_boys_mp(m, mpmath.mpf(T)))
    assert oracle.boys(m, T) == pytest.approx(ref, rel=5e-15)


@pytest.mark.parametrize("T", [0.01, 1.0, 12.0, 40.0, 70.0])
def test_boys_recursion_identity(T):
    for m in range(0, 10):
        lhs = oracle.boys(m, T)
        rhs = (2 * T * oracle.boys(m + 1, T) + np.exp(-T)) / (2 * m + 1)
        assert lhs == pytest.approx(rhs, rel=1e-14)


def test_boys_large_T_asymptote():
    # F_m(T) -> (2m-1)!!/2^{m+1} sqrt(pi/T^{2m+1}); exact up to ~exp(-T) terms
    for m in range(0, 4):
        T = 200.0
        df = np.prod(np.arange(2 * m - 1, 0, -2)) if m > 0 else 1.0
        asym = df / 2 ** (m + 1) * np.sqrt(np.pi / T ** (2 * m + 1))
        assert oracle.boys(m, T) == pytest.approx(asym, rel=1e-14)


# ---------------------------------------------------------------- primitive ERIs
def test_ss_ss_closed_form():
    rng = np.random.default_rng(3)
    z = (0, 0, 0)
    for _ in range(20):
        a, b, c, d = rng.uniform(0.1, 20.0, 4)
        A, B, C, D = rng.uniform(-1.5, 1.5, (4, 3))
        p, q = a + b, c + d
        P = (a * A + b * B) / p
        Q = (c * C + d * D) / q
        rho = p * q / (p + q)
        T = rho * np.sum((P - Q) ** 2)
        F0 = 1.0 if T < 1e-14 else 0.5 * np.sqrt(np.pi / T) * erf(np.sqrt(T))
        ref = (2 * np.pi ** 2.5 / (p * q * np.sqrt(p + q)) * np.exp(-a * b / p * np.sum((A - B) ** 2))
               * np.exp(-c * d / q * np.sum((C - D) ** 2)) * F0)
        got = oracle.eri_prim(z, a, A, z, b, B, z, c, C, z, d, D)
        assert got == pytest.approx(ref, rel=1e-13)


def _random_quartet_case(rng, ls):
    exps = rng.uniform(0.2, 4.0, 4)
    cen = rng.uniform(-0.8, 0.8, (4, 3))
    comps = [quad.cart_components(l)[rng.integers(0, (l + 1) * (l + 2) // 2)] for l in ls]
    return comps, exps, cen


@pytest.mark.parametrize("ls", [(1, 0, 0, 0), (0, 0, 1, 0), (1, 1, 0, 0), (1, 0, 1, 0), (2, 0, 0, 0),
                                (2, 1, 1, 0), (1, 1, 1, 1), (2, 0, 2, 0), (2, 2, 1, 1), (2, 2, 2, 2),
                                (3, 0, 0, 0), (3, 1, 2, 0), (3, 2, 3, 1), (3, 3, 3, 3)])
def test_eri_prim_brute_quadrature(ls):
    rng = np.random.default_rng(sum(ls) * 7 + ls[0])
    for _ in range(2):
        comps, e, c = _random_quartet_case(rng, ls)
        got = oracle.eri_prim(comps[0], e[0], c[0], comps[1], e[1], c[1], comps[2], e[2], c[2], comps[3], e[3], c[3])
        ref = quad.eri_prim(comps[0], e[0], c[0], comps[1], e[1], c[1], comps[2], e[2], c[2], comps[3], e[3], c[3])
        assert abs(got - ref) <= 1e-10 * max(abs(ref), 1e-3 * _scale(e)), (comps, got, ref)


def _scale(e):
    return 2 * np.pi ** 2.5 / ((e[0] + e[1]) * (e[2] + e[3]) * np.sqrt(e.sum()))


# ---------------------------------------------------------------- contracted basis
def _tiny(ls=(0, 1, 2), natom=2, seed=1):
    rng = np.random.default_rng(seed)
    return inputs.make_molecule(natom, list(ls), 0.3, 20.0, rng)


@pytest.mark.parametrize("ls", [(0, 1, 2), (0, 1, 2, 3)])
def test_contracted_functions_unit_norm_by_quadrature(ls):
    mol = _tiny(ls=ls)
    B = oracle.Basis.from_molecule(mol)
    coef, cnorm = B.normalized_coefs()
    po = np.concatenate([[0], np.cumsum(mol.nprim)])
    mu = 0
    for s in range(mol.nshell):
        l = int(mol.shell_l[s])
        A = mol.shell_xyz[s]
        for comp in quad.cart_components(l):
            tot = 0.0
            for i in range(po[s], po[s + 1]):
                for j in range(po[s], po[s + 1]):
                    tot += coef[i] * coef[j] * quad.overlap_prim(comp, mol.alpha[i], A, comp, mol.alpha[j], A)
            assert tot * cnorm[mu] ** 2 == pytest.approx(1.0, rel=1e-13)
            mu += 1


def test_overlap_matrix_by_quadrature():
    mol = _tiny()
    B = oracle.Basis.from_molecule(mol)
    S = B.overlap()
    coef, cnorm = B.normalized_coefs()
    po = np.concatenate([[0], np.cumsum(mol.nprim)])
    funcs = []
    for s in range(mol.nshell):
        for comp in quad.cart_components(int(mol.shell_l[s])):
            funcs.append((s, comp))
    for mu, (sa, ca) in enumerate(funcs):
        for nu, (sb, cb) in enumerate(funcs):
            tot = 0.0
            for i in range(po[sa], po[sa + 1]):
                for j in range(po[sb], po[sb + 1]):
                    tot += coef[i] * coef[j] * quad.overlap_prim(ca, mol.alpha[i], mol.shell_xyz[sa],
                                                                 cb, mol.alpha[j], mol.shell_xyz[sb])
            assert S[mu, nu] == pytest.approx(tot * cnorm[mu] * cnorm[nu], abs=1e-13)
    assert np.allclose(np.diag(S), 1.0, rtol=0, atol=1e-13)


def test_eri_eightfold_symmetry_and_schwarz():
    mol = _tiny(ls=(0, 1, 2), natom=2)
    B = oracle.Basis.from_molecule(mol)
    g = B.eri_full()
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.allclose(g, g.transpose(perm), rtol=0, atol=1e-14 * np.abs(g).max())
    n = g.shape[0]
    diag = np.einsum("ijij->ij", g)
    assert diag.min() > 0
    bound = np.sqrt(np.outer(diag.reshape(-1), diag.reshape(-1))).reshape(n, n, n, n)
    assert np.all(np.abs(g) <= bound * (1 + 1e-12) + 1e-15)


def test_contracted_shell_block_by_quadrature():
    """One contracted (pd|sp) block by brute-force quadrature over primitives."""
    mol = _tiny(ls=(0, 1, 2), natom=2, seed=5)
    B = oracle.Basis.from_molecule(mol)
    coef, cnorm = B.normalized_coefs()
    po = np.concatenate([[0], np.cumsum(mol.nprim)])
    sh = [1, 5, 3, 4]  # p(atom0) d(atom1) s(atom1) p(atom1)
    blk = B.eri_shell(*sh)
    comps = [quad.cart_components(int(mol.shell_l[s])) for s in sh]
    rng = np.random.default_rng(0)
    for _ in range(3):
        idx = [rng.integers(0, len(c)) for c in comps]
        tot = 0.0
        for ps in itertools.product(*[range(po[s], po[s + 1]) for s in sh]):
            cc = np.prod([coef[i] for i in ps])
            tot += cc * quad.eri_prim(*sum(([comps[k][idx[k]], mol.alpha[ps[k]], mol.shell_xyz[sh[k]]] for k in range(4)), []))
        fn = [B.offsets[s] + i for s, i in zip(sh, idx)]
        tot *= np.prod([cnorm[f] for f in fn])
        assert blk[tuple(idx)] == pytest.approx(tot, rel=1e-9, abs=1e-12)


def test_contracted_f_shell_blocks_by_quadrature():
    """Sampled elements of contracted blocks with f shells ((fd|ps), (ff|fp))
    by brute-force quadrature over primitives."""
    mol = _tiny(ls=(0, 1, 2, 3), natom=2, seed=9)
    B = oracle.Basis.from_molecule(mol)
    coef, cnorm = B.normalized_coefs()
    po = np.concatenate([[0], np.cumsum(mol.nprim)])
    rng = np.random.default_rng(2)
    for sh in ([3, 6, 5, 0], [3, 7, 7, 1]):  # f(0) d(1) p(1) s(0); f(0) f(1) f(1) p(0)
        blk = B.eri_shell(*sh)
        comps = [quad.cart_components(int(mol.shell_l[s])) for s in sh]
        for _ in range(2):
            idx = [rng.integers(0, len(c)) for c in comps]
            tot = 0.0
            for ps in itertools.product(*[range(po[s], po[s + 1]) for s in sh]):
                cc = np.prod([coef[i] for i in ps])
                tot += cc * quad.eri_prim(*sum(([comps[k][idx[k]], mol.alpha[ps[k]], mol.shell_xyz[sh[k]]]
                                                for k in range(4)), []))
            fn = [B.offsets[s] + i for s, i in zip(sh, idx)]
            tot *= np.prod([cnorm[f] for f in fn])
            assert blk[tuple(idx)] == pytest.approx(tot, rel=1e-9, abs=1e-12 * np.abs(blk).max()), (sh, idx)


# ---------------------------------------------------------------- J / K
def _small_case(seed=0, ls=(0, 1, 2), natom=2):
    mol = _tiny(ls=ls, natom=natom, seed=seed)
    B = oracle.Basis.from_molecule(mol)
    S = B.overlap()
    rng = np.random.default_rng(seed + 100)
    Q = inputs.random_orbitals(B.nbf, 3, rng)
    P = oracle.density_real(S, Q)
    return mol, B, P


def test_jk_definition_einsum_and_symmetric_build():
    mol, B, P = _small_case()
    g = B.eri_full()
    rng = np.random.default_rng(9)
    A = inputs.random_symmetric(B.nbf, rng, -1)
    X = np.stack([P, A, rng.standard_normal((B.nbf, B.nbf))])
    Jf, Kf = B.jk_full(X)
    Jref = np.einsum("ijkl,mkl->mij", g, X)
    Kref = np.einsum("ikjl,mkl->mij", g, X)
    assert np.allclose(Jf, Jref, rtol=0, atol=1e-13 * np.abs(Jref).max())
    assert np.allclose(Kf, Kref, rtol=0, atol=1e-13 * np.abs(Kref).max())
    Js, Ks = B.jk(X)
    assert np.allclose(Js, Jf, rtol=0, atol=1e-13 * np.abs(Jf).max())
    assert np.allclose(Ks, Kf, rtol=0, atol=1e-13 * np.abs(Kf).max())


def test_jk_symmetry_signs_and_positivity():
    mol, B, P = _small_case(seed=2)
    rng = np.random.default_rng(4)
    A = inputs.random_symmetric(B.nbf, rng, -1)
    J, K = B.jk(np.stack([P, A]))
    assert np.allclose(J[0], J[0].T, atol=1e-14)
    assert np.allclose(K[0], K[0].T, atol=1e-14)
    assert np.abs(J[1]).max() < 1e-13
    assert np.allclose(K[1], -K[1].T, atol=1e-14)
    assert np.sum(P * J[0]) > 0 and np.sum(P * K[0]) > 0


def test_single_orbital_coulomb_equals_exchange():
    mol = _tiny(natom=3, seed=4)
    B = oracle.Basis.from_molecule(mol)
    c = np.random.default_rng(1).standard_normal(B.nbf)
    P = np.outer(c, c)
    J, K = B.jk(P)
    assert np.sum(P * J) == pytest.approx(np.sum(P * K), rel=1e-13)


def test_translation_invariance():
    mol, B, P = _small_case(seed=3)
    shift = np.array([0.37, -1.2, 2.5])
    B2 = oracle.Basis(mol.shell_xyz + shift, mol.shell_l, mol.nprim, mol.alpha, mol.coef)
    J1, K1 = B.jk(P)
    J2, K2 = B2.jk(P)
    assert np.allclose(J1, J2, rtol=0, atol=1e-12 * np.abs(J1).max())
    assert np.allclose(K1, K2, rtol=0, atol=1e-12 * np.abs(K1).max())


def _rotz90_matrix(mol, B):
    """Signed permutation D with phi_mu(R^-1 r) = sum_nu D_{nu mu} phi'_nu(r)
    for the rotation (x, y, z) -> (-y, x, z)."""
    n = B.nbf
    D = np.zeros((n, n))
    for s in range(mol.nshell):
        comps = quad.cart_components(int(mol.shell_l[s]))
        o = B.offsets[s]
        for i, (a, b, c) in enumerate(comps):
            # x^a y^b z^c evaluated at R^-1 r = (y, -x, z) -> (-1)^b x^b y^a z^c
            j = comps.index((b, a, c))
            D[o + j, o + i] = (-1) ** b
    return D


def test_rotation_invariance_exact():
    mol, B, P = _small_case(seed=6, natom=3)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    B2 = oracle.Basis(mol.shell_xyz @ R.T, mol.shell_l, mol.nprim, mol.alpha, mol.coef)
    D = _rotz90_matrix(mol, B)
    J1, K1 = B.jk(P)
    P2 = D @ P @ D.T
    J2, K2 = B2.jk(P2)
    assert np.allclose(J2, D @ J1 @ D.T, rtol=0, atol=1e-12 * np.abs(J1).max())
    assert np.allclose(K2, D @ K1 @ D.T, rtol=0, atol=1e-12 * np.abs(K1).max())
    assert np.sum(P2 * J2) == pytest.approx(np.sum(P * J1), rel=1e-13)


def test_rotation_general_traces():
    """A generic rotation leaves Tr(PJ) and Tr(PK) unchanged when P rotates
    with the basis (d functions through the symmetric-tensor representation)."""
    mol, B, P = _small_case(seed=8, natom=2)
    th = 0.7
    ax = np.array([1.0, 2.0, -0.5]); ax /= np.linalg.norm(ax)
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    B2 = oracle.Basis(mol.shell_xyz @ R.T, mol.shell_l, mol.nprim, mol.alpha, mol.coef)
    # transformation of unnormalized monomials under r -> R^T r, then the
    # component normalization factors
    coef, cn = B.normalized_coefs()
    n = B.nbf
    D = np.zeros((n, n))
    for s in range(mol.nshell):
        l = int(mol.shell_l[s]); comps = quad.cart_components(l); o = B.offsets[s]
        # monomial m(R^T r) expanded in monomials of r, by sampling points
        pts = np.random.default_rng(0).standard_normal((len(comps) + 5, 3))
        M = np.array([[np.prod(p ** np.array(c)) for c in comps] for p in pts])
        Mr = np.array([[np.prod((R.T @ p) ** np.array(c)) for c in comps] for p in pts])
        T = np.linalg.lstsq(M, Mr, rcond=None)[0]  # Mr = M T
        for i in range(len(comps)):
            for j in range(len(comps)):
                D[o + j, o + i] = T[j, i] * cn[o + i] / cn[o + j]
    J1, K1 = B.jk(P)
    P2 = D @ P @ D.T
    J2, K2 = B2.jk(P2)
    assert np.sum(P2 * J2) == pytest.approx(np.sum(P * J1), rel=1e-12)
    assert np.sum(P2 * K2) == pytest.approx(np.sum(P * K1), rel=1e-12)


def test_blocks_match_full_build():
    mol, B, P = _small_case(seed=7, natom=2)
    J, K = B.jk(P)
    o = B.offsets
    for a, b in [(0, 1), (2, 5), (4, 4)]:
        jb = B.j_block(a, b, P)[0]
        kb = B.k_block(a, b, P)[0]
        assert np.allclose(jb, J[o[a]:o[a + 1], o[b]:o[b + 1]], rtol=0, atol=1e-13)
        assert np.allclose(kb, K[o[a]:o[a + 1], o[b]:o[b + 1]], rtol=0, atol=1e-13)


def test_schwarz_matches_diagonal():
    mol, B, P = _small_case(seed=1)
    g = B.eri_full()
    Q = B.schwarz()
    o = B.offsets
    for a in range(mol.nshell):
        for b in range(mol.nshell):
            blk = g[o[a]:o[a + 1], o[b]:o[b + 1], o[a]:o[a + 1], o[b]:o[b + 1]]
            d = np.einsum("ijij->ij", blk)
            assert Q[a, b] == pytest.approx(np.sqrt(d.max()), rel=1e-14)
