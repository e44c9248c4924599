"""Write the oracle regression fixtures of this folder (calls only oracle/
and the seeded input generator).

The paper prints no worked numerical example (no integral, energy or matrix
element of a named system), so no fixture here is a value from the paper.
These files pin the oracle to itself over time: a later change of its
arithmetic that moves any of these numbers fails tests/test_golden.py and
has to say why.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import twocomp  # noqa: E402
from paper_1905_01381_amd import inputs  # noqa: E402


def c1_fixture():
    """6 atoms, 2s1p (nbf 30): energies Tr(P J), Tr(P K) and the first row
    of J and K for the seeded 5-orbital density."""
    w = inputs.c1()
    ob = oracle.Basis.from_molecule(w.mol)
    P = oracle.density_real(ob.overlap(), w.orbitals)
    J, K = ob.jk_full(P)
    return {"workload": "6 atoms, 2s1p, exponents 0.15..30, seed 0; P from 5 S-orthonormal orbitals",
            "tr_PJ": float(np.sum(P * J)), "tr_PK": float(np.sum(P * K)),
            "J_row0": [float(x) for x in J[0]], "K_row0": [float(x) for x in K[0]]}


def twocomp_fixture():
    """2 atoms, 3s2p1d (exponents 0.3..50): the two-electron energy of the
    two-component Fock matrix, 1/2 Tr[P G]."""
    w = inputs.small(2, inputs.SHELLS_3S2P1D, seed=7, lo=0.3, hi=50.0, complex_=True)
    ob = oracle.Basis.from_molecule(w.mol)
    P2 = oracle.density_2c(ob.overlap(), w.orbitals)
    G, _ = twocomp.fock2e(ob, P2, full=True)
    return {"workload": "2 atoms, 3s2p1d, exponents 0.3..50, seed 7; 2C density",
            "E2_2c": twocomp.energy_2e_2c(P2, G)}


def boys_fixture():
    T = [0.0, 0.3, 2.5, 17.0, 40.0]
    return {"T": T, "F": [[oracle.boys(m, t) for m in range(9)] for t in T]}


if __name__ == "__main__":
    out = {"c1": c1_fixture(), "twocomp": twocomp_fixture(), "boys": boys_fixture()}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1)
