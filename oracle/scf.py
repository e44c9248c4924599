"""Closed-shell Hartree-Fock ground state with the oracle's J/K (TEST
INFRASTRUCTURE): builds initial states for the real-time checks entirely on
the oracle side.  Plain Roothaan-Hall iterations (Eq. rh_1c) with DIIS."""
from __future__ import annotations

import numpy as np


def rhf(basis, mol, nocc, maxiter=200, conv=1e-11):
    S = basis.overlap()
    h = basis.one_electron("kinetic") + basis.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)
    w, U = np.linalg.eigh(S)
    X = (U / np.sqrt(w)) @ U.T

    def dens(F):
        _, Cp = np.linalg.eigh(X @ F @ X)
        C = X @ Cp[:, :nocc]
        return C @ C.T

    P = dens(h)
    Fs, Es = [], []
    Eold = 0.0
    for it in range(maxiter):
        J, K = basis.jk(P)
        F = h + 2 * J - K
        E = float(np.sum(P * (h + F)))
        err = X @ (F @ P @ S - S @ P @ F) @ X
        Fs, Es = (Fs + [F])[-8:], (Es + [err])[-8:]
        m = len(Fs)
        if m > 1:
            B = -np.ones((m + 1, m + 1)); B[m, m] = 0
            for i in range(m):
                for j in range(m):
                    B[i, j] = np.sum(Es[i] * Es[j])
            c = np.linalg.solve(B, np.r_[np.zeros(m), -1.0])[:m]
            F = sum(ci * fi for ci, fi in zip(c, Fs))
        P = dens(F)
        if abs(E - Eold) < conv and np.abs(err).max() < 1e-8:
            break
        Eold = E
    return P, h, S, X, E
