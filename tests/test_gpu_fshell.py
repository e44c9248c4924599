"""Shells up to f (l = 3; paper: Introduction, contracted Gaussian basis
functions) against the oracle on the same seeded inputs: every class with
an f shell goes through the workgroup-per-quartet kernel, the rest through
the generated kernels, in one build.

* Shell blocks of every f class and orientation (cq_eri_quartet) within
  1e-10 of the largest element of the block.
* Schwarz factors and one-electron integrals with f shells.
* J/K of symmetric, antisymmetric and general densities within 1e-10
  relative per matrix; the two-component build; a batch handle mixing
  f and d molecules.
* Spherical f shells with general contraction.
* Screening: nothing skipped at a negligible threshold gives bitwise the
  unscreened result; at 1e-6 the counters add up to the unique quartets and
  the change stays within the skipped quartets' bounds.
* Builds repeat bitwise; the allocation-free entry point matches.
* Routed mode, the autotuner, per-class timing, the RS driver and real-time
  EM2 steps on bases with f shells.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import spherical as osph
from oracle import twocomp
from paper_1905_01381_amd import inputs
from tests.gpu_common import rel_err

pytestmark = pytest.mark.gpu

TOL_JK = 1e-10
SHELLS = [0, 1, 2, 3]


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.name}", flush=True)
    sys.stdout.flush()
    yield


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1905_01381_amd import cq
    cq.lib()
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def fcase(torch_cuda):
    """3 atoms, s p d f per atom (exponents 0.3..50), nbf 60."""
    from paper_1905_01381_amd import cq
    w = inputs.small(3, SHELLS, seed=3, lo=0.3, hi=50.0)
    ob = oracle.Basis.from_molecule(w.mol)
    P = oracle.density_real(ob.overlap(), w.orbitals)
    gb = cq.Basis.from_molecule(w.mol)
    return w, ob, gb, P


def test_f_class_blocks_every_orientation(fcase):
    w, ob, gb, _ = fcase
    ls = w.mol.shell_l
    by_l = {l: [int(s) for s in np.where(ls == l)[0]] for l in range(4)}
    rng = np.random.default_rng(2)
    worst, count = (0.0, None), 0
    for q in itertools.product(range(4), repeat=4):
        if 3 not in q:
            continue
        sh = [by_l[x][rng.integers(len(by_l[x]))] for x in q]
        e = rel_err(gb.eri_quartet(*sh), ob.eri_shell(*sh))
        worst = max(worst, (e, tuple(sh)), key=lambda t: t[0])
        count += 1
    # same-shell and same-pair quartets (degenerate cases)
    f0, f1 = by_l[3][0], by_l[3][1]
    for sh in [(f0, f0, f0, f0), (f0, f1, f0, f1), (f1, f0, f0, f1), (f0, f0, by_l[0][0], by_l[0][0])]:
        e = rel_err(gb.eri_quartet(*sh), ob.eri_shell(*sh))
        worst = max(worst, (e, tuple(sh)), key=lambda t: t[0])
        count += 1
    print(f"worst f block relative error {worst[0]:.3e} at shells {worst[1]} over {count} blocks", flush=True)
    assert worst[0] < TOL_JK, worst
    assert count == 4 ** 4 - 3 ** 4 + 4


def test_f_schwarz_and_one_electron(fcase, torch_cuda):
    w, ob, gb, _ = fcase
    Q = gb.schwarz().cpu().numpy()
    Qr = ob.schwarz()
    # diagonal blocks from two FP64 algorithms (product-centred recurrence
    # summed over primitives here, Hermite expansion in the oracle): within
    # 2e-12 of the largest factor; 1e-11 is kept, the block bar of the s-d
    # classes
    assert rel_err(Q, Qr) < 1e-11
    for kind in ("overlap", "kinetic"):
        assert rel_err(gb.one_electron(kind).cpu().numpy(), ob.one_electron(kind)) < 1e-12, kind
    got = gb.one_electron("dipole", direction=0, origin=(0.1, 0.2, -0.3)).cpu().numpy()
    assert rel_err(got, ob.one_electron("dipole", direction=0, origin=(0.1, 0.2, -0.3))) < 1e-12
    mol = w.mol
    got = gb.one_electron("nuclear", charges=mol.charges, centers=mol.atoms).cpu().numpy()
    assert rel_err(got, ob.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)) < 1e-12


def test_f_jk_mixed_symmetry_full_parity(fcase, torch_cuda):
    torch = torch_cuda
    w, ob, gb, P = fcase
    rng = np.random.default_rng(7)
    A = inputs.random_symmetric(gb.nbf, rng, sign=-1)
    G = rng.standard_normal((gb.nbf, gb.nbf))
    r = gb.jk([_dev(torch, P), _dev(torch, A), _dev(torch, G)], sym=[1, -1, 0], want_j=[True, False, True])
    torch.cuda.synchronize()
    Jr, Kr = ob.jk_full(np.array([P, A, G]))
    assert rel_err(r.J[0].cpu().numpy(), Jr[0]) < TOL_JK
    assert rel_err(r.K[0].cpu().numpy(), Kr[0]) < TOL_JK
    assert rel_err(r.K[1].cpu().numpy(), Kr[1]) < TOL_JK
    assert rel_err(r.J[2].cpu().numpy(), Jr[2]) < TOL_JK
    assert rel_err(r.K[2].cpu().numpy(), Kr[2]) < TOL_JK


def test_f_only_basis_and_eight_densities(torch_cuda):
    """Every shell an f shell (all classes (ff|ff)), 8 densities, and a
    one-shell basis."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.small(3, [3, 3], seed=5, lo=0.4, hi=20.0)
    ob = oracle.Basis.from_molecule(w.mol)
    gb = cq.Basis.from_molecule(w.mol)
    rng = np.random.default_rng(3)
    mats = [inputs.random_symmetric(gb.nbf, rng) for _ in range(8)]
    r = gb.jk([_dev(torch, m) for m in mats])
    torch.cuda.synchronize()
    Jr, Kr = ob.jk(np.array(mats))
    for m in range(8):
        assert rel_err(r.J[m].cpu().numpy(), Jr[m]) < TOL_JK, m
        assert rel_err(r.K[m].cpu().numpy(), Kr[m]) < TOL_JK, m
    w1 = inputs.small(1, [3], seed=6, lo=0.4, hi=20.0)
    ob1 = oracle.Basis.from_molecule(w1.mol)
    gb1 = cq.Basis.from_molecule(w1.mol)
    P1 = inputs.random_symmetric(10, rng)
    r1 = gb1.jk([_dev(torch, P1)])
    torch.cuda.synchronize()
    J1, K1 = ob1.jk(P1)
    assert rel_err(r1.J[0].cpu().numpy(), J1) < TOL_JK
    assert rel_err(r1.K[0].cpu().numpy(), K1) < TOL_JK


def test_f_two_component(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.small(2, SHELLS, seed=8, lo=0.3, hi=50.0, complex_=True)
    ob = oracle.Basis.from_molecule(w.mol)
    P2 = oracle.density_2c(ob.overlap(), w.orbitals)
    gb = cq.Basis.from_molecule(w.mol)
    G = gb.fock2e_2c(_dev(torch, P2))
    torch.cuda.synchronize()
    Gr, _ = twocomp.fock2e(ob, P2)
    assert rel_err(G.cpu().numpy(), Gr) < TOL_JK


def test_f_spherical_general(torch_cuda):
    """Spherical d and f, generally contracted shells (2 atoms of the
    4s3p2d1f recipe as general contractions: nbf 2 * (4 + 9 + 10 + 7) = 60)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.small(2, inputs.SHELLS_4S3P2D1F, seed=9, lo=0.3, hi=50.0, spherical=True, general=True)
    ob = osph.SphericalBasis.from_molecule(w.mol)
    gb = cq.Basis.from_molecule(w.mol)
    assert gb.nbf == ob.nbf == w.mol.nbf == 60
    S = ob.overlap()
    assert rel_err(gb.one_electron("overlap").cpu().numpy(), S) < 1e-12
    P = oracle.density_real(S, w.orbitals)
    G = np.random.default_rng(4).standard_normal((gb.nbf, gb.nbf))
    r = gb.jk([_dev(torch, P), _dev(torch, G)], sym=[1, 0])
    torch.cuda.synchronize()
    Jr, Kr = ob.jk(np.array([P, G]))
    for m in range(2):
        assert rel_err(r.J[m].cpu().numpy(), Jr[m]) < TOL_JK, m
        assert rel_err(r.K[m].cpu().numpy(), Kr[m]) < TOL_JK, m


def test_f_batch_with_d_molecules(torch_cuda):
    """A batch handle over an f molecule, a d-only molecule and a spherical
    f molecule, against the oracle molecule by molecule."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws = [inputs.small(2, SHELLS, seed=11, lo=0.3, hi=50.0),
          inputs.small(3, inputs.SHELLS_3S2P1D, seed=12, lo=0.3, hi=50.0),
          inputs.small(2, SHELLS, seed=13, lo=0.3, hi=50.0, spherical=True)]
    mols = [w.mol for w in ws]
    gb = cq.Basis.from_molecules(mols)
    obs = [osph.SphericalBasis.from_molecule(m) for m in mols]
    assert gb.mol_nbf == [ob.nbf for ob in obs] == [40, 45, 32]
    Ps = [oracle.density_real(ob.overlap(), w.orbitals) for ob, w in zip(obs, ws)]
    r = gb.jk([gb.pack([_dev(torch, P) for P in Ps])])
    torch.cuda.synchronize()
    Js, Ks = gb.unpack(r.J[0]), gb.unpack(r.K[0])
    for i, (ob, P) in enumerate(zip(obs, Ps)):
        Jr, Kr = ob.jk(P)
        assert rel_err(Js[i].cpu().numpy(), Jr) < TOL_JK, i
        assert rel_err(Ks[i].cpu().numpy(), Kr) < TOL_JK, i


def test_f_screening_and_counts(fcase, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, P = fcase
    total = sum(gb.quartet_counts().values())
    assert any(3 in k for k in gb.quartet_counts())
    ns = gb.nshell
    npair = ns * (ns + 1) // 2
    assert total == npair * (npair + 1) // 2
    r0 = gb.jk([_dev(torch, P)])
    J0, K0 = r0.J[0].cpu().numpy(), r0.K[0].cpu().numpy()
    r1 = gb.jk([_dev(torch, P)], th=cq.thresholds(skip=1e-300))
    assert np.array_equal(r1.J[0].cpu().numpy(), J0) and np.array_equal(r1.K[0].cpu().numpy(), K0)
    st = gb.build_stats()
    assert st["skipped"] == 0 and st["fp64"] == total
    # the same molecule stretched 4x, so that distant tight pairs fall below
    w4 = inputs.small(3, SHELLS, seed=3, lo=0.3, hi=50.0)
    w4.mol.atoms *= 4.0
    w4.mol.shell_xyz *= 4.0
    ob4 = oracle.Basis.from_molecule(w4.mol)
    P4 = oracle.density_real(ob4.overlap(), w4.orbitals)
    g4 = cq.Basis.from_molecule(w4.mol)
    r0 = g4.jk([_dev(torch, P4)])
    J0, K0 = r0.J[0].cpu().numpy(), r0.K[0].cpu().numpy()
    tau = 1e-6
    r2 = g4.jk([_dev(torch, P4)], th=cq.thresholds(skip=tau))
    st = g4.build_stats()
    dJ = np.abs(r2.J[0].cpu().numpy() - J0).max()
    dK = np.abs(r2.K[0].cpu().numpy() - K0).max()
    print(f"skip {tau}: {st}, max|dJ| {dJ:.2e}, max|dK| {dK:.2e}", flush=True)
    assert st["fp64"] + st["skipped"] == total and st["skipped"] > 0
    # a skipped quartet changes an element by at most its bound per pair of
    # summed functions (at most 10 x 10) on each of its (at most 8) routes
    assert dJ <= 8 * 100 * tau * st["skipped"]
    assert dK <= 8 * 100 * tau * st["skipped"]


def test_f_bitwise_repeat_and_noalloc(fcase, torch_cuda):
    torch = torch_cuda
    w, ob, gb, P = fcase
    rng = np.random.default_rng(17)
    mats = [P, inputs.random_symmetric(gb.nbf, rng)]
    out = []
    for noalloc in (False, False, True):
        r = gb.jk([_dev(torch, m) for m in mats], noalloc=noalloc)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in r.J + r.K])
    for k in range(4):
        assert np.array_equal(out[0][k], out[1][k]), k
        assert np.array_equal(out[0][k], out[2][k]), k


def test_f_classes_profiled(fcase, torch_cuda):
    """Per-class timing lists the f classes next to the generated ones, one
    launch each per build."""
    torch = torch_cuda
    w, ob, gb, P = fcase
    gb.profile(True, reset=True)
    gb.jk([_dev(torch, P)])
    torch.cuda.synchronize()
    prof = gb.profile_read()
    gb.profile(False)
    fcls = {k: v for k, v in prof.items() if 3 in k}
    print(f"f classes timed: {len(fcls)}, total {sum(v[0] for v in fcls.values()):.3f} ms", flush=True)
    assert set(fcls) == {k for k, n in gb.quartet_counts().items() if 3 in k and n > 0}
    assert all(v[1] == 1 and v[0] > 0 for v in fcls.values())


def test_f_routed_mode(fcase, torch_cuda):
    """Routed mode on a basis with f shells: the f classes stay FP64, the
    counters add up to the unique quartets, and the energy stays within
    1e-6 Eh of the oracle at FP32 below 1e-5."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, P = fcase
    total = sum(gb.quartet_counts().values())
    nq_f = sum(v for k, v in gb.quartet_counts().items() if 3 in k)
    r = gb.jk([_dev(torch, P)], th=cq.thresholds(mode=1, fp32_below=1e-5))
    st = gb.build_stats()
    assert st["fp64"] + st["fp32"] + st["skipped"] == total
    assert st["fp64"] >= nq_f
    Jr, Kr = ob.jk(P)
    J, K = r.J[0].cpu().numpy(), r.K[0].cpu().numpy()
    dE = abs((2 * np.sum(P * J) - np.sum(P * K)) - (2 * np.sum(P * Jr) - np.sum(P * Kr)))
    print(f"routed: {st}, dE {dE:.2e}", flush=True)
    assert dE < 1e-6


def test_f_autotune_keeps_results(torch_cuda):
    """cq_autotune on a basis with f shells tunes the generated classes and
    leaves the build's results unchanged (the f classes have no plan)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.small(2, SHELLS, seed=19, lo=0.3, hi=50.0)
    ob = oracle.Basis.from_molecule(w.mol)
    P = oracle.density_real(ob.overlap(), w.orbitals)
    gb = cq.Basis.from_molecule(w.mol)
    r0 = gb.jk([_dev(torch, P)])
    J0, K0 = r0.J[0].cpu().numpy(), r0.K[0].cpu().numpy()
    plan = gb.autotune(nmat=1, reps=1)
    assert plan and all(3 not in p["cls"] for p in plan)
    r1 = gb.jk([_dev(torch, P)])
    assert rel_err(r1.J[0].cpu().numpy(), J0) < 1e-13 and rel_err(r1.K[0].cpu().numpy(), K0) < 1e-13
    Jr, Kr = ob.jk(P)
    assert rel_err(r1.J[0].cpu().numpy(), Jr) < TOL_JK and rel_err(r1.K[0].cpu().numpy(), Kr) < TOL_JK


def test_f_rhf_and_em2_against_oracle(torch_cuda):
    """The RS driver and real-time EM2 steps on a basis with f shells (2
    atoms of charge 1, s p d f each, nbf 40) against the oracle's RHF and
    EM2."""
    torch = torch_cuda
    from oracle import rt
    from oracle import scf as oscf
    from paper_1905_01381_amd import cq, scf
    w = inputs.small(2, SHELLS, seed=23, lo=0.3, hi=50.0)
    ob = oracle.Basis.from_molecule(w.mol)
    gb = cq.Basis.from_molecule(w.mol)
    P, h, S, X, E = oscf.rhf(ob, w.mol, 1)
    res = scf.scf(gb, w.mol, "RS", 1, conv=1e-11)
    assert res.converged
    assert abs((res.energy - res.e_nuc) - E) < 1e-8
    Sh = S @ X
    Po = (Sh @ P @ Sh).astype(complex)
    Dz = ob.one_electron("dipole", direction=2)
    U = rt.expm_herm(X @ Dz @ X, 1e-2)
    P0 = U @ Po @ U.conj().T
    r = cq.RT(gb, _dev(torch, h), _dev(torch, X), _dev(torch, Dz), _dev(torch, P0), 0.05, cq.RT_EM2)
    _, mu, nb = r.step(3)
    Pg = r.density().cpu().numpy()
    Pr = P0
    for _ in range(3):
        Pr = rt.em2_step(ob, h, X, Pr, 0.05)
    assert np.abs(Pg - Pr).max() < 1e-10 * np.abs(Pr).max()
    _, mu_ref = rt.energy_dipole(ob, h, X, Dz, Pr)
    assert abs(mu[-1] - mu_ref) < 1e-10
