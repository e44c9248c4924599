"""The library's Hartree-Fock driver (RS / US / GS Roothaan-Hall with damping
and DIIS; every J/K on the GPU) against the oracle's RHF / UHF / GHF on the
6-atom 2s1p workload (6 electrons): electronic energies within 1e-8 Eh."""
import sys

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle import scf as oscf
from oracle import twocomp
from paper_1905_01381_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.name}", flush=True)
    sys.stdout.flush()
    yield


@pytest.fixture(scope="module")
def c1():
    import torch
    assert torch.cuda.is_available()
    from paper_1905_01381_amd import cq
    w = inputs.c1()
    return w.mol, oracle.Basis.from_molecule(w.mol), cq.Basis.from_molecule(w.mol)


def test_rs_scf_against_oracle_rhf(c1):
    from paper_1905_01381_amd import scf
    mol, ob, gb = c1
    ref = oscf.rhf(ob, mol, 3)[4]
    res = scf.scf(gb, mol, "RS", 3, conv=1e-11)
    assert res.converged
    assert abs((res.energy - res.e_nuc) - ref) < 1e-8
    damped = scf.scf(gb, mol, "RS", 3, conv=1e-11, damping=0.4, damp_until=1e-1)
    assert damped.converged and abs(damped.energy - res.energy) < 1e-9


def test_us_scf_against_oracle_uhf(c1):
    from paper_1905_01381_amd import scf
    mol, ob, gb = c1
    Pa, Pb, ref = oscf.uhf(ob, mol, 4, 2)
    res = scf.scf(gb, mol, "US", 4, 2, conv=1e-11)
    assert res.converged
    assert abs((res.energy - res.e_nuc) - ref) < 1e-8
    S = ob.overlap()
    assert abs(np.sum(res.P[0] * S) - 4) < 1e-10 and abs(np.sum(res.P[1] * S) - 2) < 1e-10


def test_gs_scf_against_oracle(c1):
    """GS from a globally spin-rotated UHF density: the GPU driver reaches
    the oracle's GHF energy from the same start, which equals the UHF
    energy (spin-rotation invariance); the density keeps 6 electrons."""
    from paper_1905_01381_amd import scf
    mol, ob, gb = c1
    Pa, Pb, Eu = oscf.uhf(ob, mol, 4, 2)
    n = Pa.shape[0]
    Z = np.zeros((n, n))
    axis = np.array([0.6, 0.2, -0.7]); axis /= np.linalg.norm(axis)
    R = np.kron(expm(-0.5j * 0.9 * sum(a * s for a, s in zip(axis, twocomp.PAULI[1:]))), np.eye(n))
    P2 = R @ np.block([[Pa, Z], [Z, Pb]]).astype(complex) @ R.conj().T
    P2o, Eg = oscf.ghf(ob, mol, 6, P2)
    res = scf.scf(gb, mol, "GS", 4, 2, guess=P2, conv=1e-11)
    assert res.converged
    assert abs((res.energy - res.e_nuc) - Eg) < 1e-8
    assert abs(Eg - Eu) < 1e-8
    S = ob.overlap()
    S2 = np.block([[S, Z], [Z, S]])
    assert abs(np.trace(res.P @ S2).real - 6) < 1e-10
