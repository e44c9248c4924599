"""Shared helpers for the GPU parity tests (inputs come from the seeded
generator; expected values only from the oracle)."""
import numpy as np

import oracle
from paper_1905_01381_amd import inputs


def rel_err(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def case_real(natom, ls, seed=0, nocc=None, lo=0.1, hi=1.0e3):
    w = inputs.small(natom, ls, seed=seed, nocc=nocc, lo=lo, hi=hi)
    ob = oracle.Basis.from_molecule(w.mol)
    S = ob.overlap()
    P = oracle.density_real(S, w.orbitals)
    return w, ob, P


def case_2c(natom, ls, seed=0, nocc=None, lo=0.1, hi=1.0e3):
    w = inputs.small(natom, ls, seed=seed, nocc=nocc, lo=lo, hi=hi, complex_=True)
    ob = oracle.Basis.from_molecule(w.mol)
    S = ob.overlap()
    P2 = oracle.density_2c(S, w.orbitals)
    return w, ob, P2
