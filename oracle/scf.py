"""Hartree-Fock with the oracle's J/K (TEST INFRASTRUCTURE): ground states
for the real-time checks, and the reference for the library's SCF driver.
Plain Roothaan-Hall iterations with DIIS (paper: "Self-Consistent Field
Optimization"): closed shell (rhf, Eq. rh_1c, RS), spin unrestricted (uhf,
Eq. rh_1c, US) and generalized spin (ghf, Eq. rh_2c, GS)."""
from __future__ import annotations

import numpy as np


def rhf(basis, mol, nocc, maxiter=200, conv=1e-11, h_add=None):
    """h_add: a static one-body term added to the core Hamiltonian (e.g. a
    field kappa V)."""
    S = basis.overlap()
    h = basis.one_electron("kinetic") + basis.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)
    if h_add is not None:
        h = h + h_add
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


def _diis(Fs, Es):
    """Pulay's DIIS combination of the stored Fock matrices (minimum norm of
    the combined commutator error, coefficients summing to one)."""
    m = len(Fs)
    B = -np.ones((m + 1, m + 1))
    B[m, m] = 0.0
    for i in range(m):
        for j in range(m):
            B[i, j] = np.real(np.vdot(Es[i], Es[j]))
    c = np.linalg.solve(B, np.r_[np.zeros(m), -1.0])[:m]
    return sum(ci * fi for ci, fi in zip(c, Fs))


def uhf(basis, mol, na, nb, maxiter=300, conv=1e-11):
    """Spin-unrestricted Hartree-Fock (paper: Eq. rh_1c, the US case):
    F^s = h + J[P^a + P^b] - K[P^s] for s in (a, b), one eigenproblem per
    spin, DIIS on the stacked pair.  Returns (Pa, Pb, E_elec)."""
    S = basis.overlap()
    h = basis.one_electron("kinetic") + basis.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)
    w, U = np.linalg.eigh(S)
    X = (U / np.sqrt(w)) @ U.T

    def dens(F, n):
        _, Cp = np.linalg.eigh(X @ F @ X)
        C = X @ Cp[:, :n]
        return C @ C.T

    Pa, Pb = dens(h, na), dens(h, nb)
    Fs, Es = [], []
    Eold = 0.0
    for _ in range(maxiter):
        J, K = basis.jk(np.stack([Pa, Pb]))
        Fa = h + J[0] + J[1] - K[0]
        Fb = h + J[0] + J[1] - K[1]
        E = 0.5 * float(np.sum(Pa * (h + Fa)) + np.sum(Pb * (h + Fb)))
        err = np.stack([X @ (Fa @ Pa @ S - S @ Pa @ Fa) @ X, X @ (Fb @ Pb @ S - S @ Pb @ Fb) @ X])
        Fs, Es = (Fs + [np.stack([Fa, Fb])])[-8:], (Es + [err])[-8:]
        F = _diis(Fs, Es) if len(Fs) > 1 else Fs[-1]
        Pa, Pb = dens(F[0], na), dens(F[1], nb)
        if abs(E - Eold) < conv and np.abs(err).max() < 1e-8:
            break
        Eold = E
    return Pa, Pb, E


def ghf(basis, mol, nel, P2_guess, maxiter=300, conv=1e-11):
    """Generalized-spin Hartree-Fock (paper: Eq. rh_2c, the GS case): one
    eigenproblem of twice the dimension for F^{2C} = h (x) 1 + G^{2C}(P^{2C}),
    G^{2C} from the Pauli components (Eq. 2c_fock, reading
    G^0 = 2J[P^0] - K[P^0], G^k = -K[P^k]); DIIS on F^{2C}.  Starts from the
    given spin-blocked density.  Returns (P2, E_elec)."""
    from oracle import twocomp
    S = basis.overlap()
    h = basis.one_electron("kinetic") + basis.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)
    n = S.shape[0]
    w, U = np.linalg.eigh(S)
    X = (U / np.sqrt(w)) @ U.T
    Z = np.zeros((n, n))
    S2, h2, X2 = np.block([[S, Z], [Z, S]]), np.block([[h, Z], [Z, h]]), np.block([[X, Z], [Z, X]])
    P2 = P2_guess.astype(complex)
    Fs, Es = [], []
    Eold = 0.0
    for _ in range(maxiter):
        G, _ = twocomp.fock2e(basis, P2)
        F = h2 + G
        E = 0.5 * float(np.real(np.trace(P2 @ (h2 + F))))
        err = X2 @ (F @ P2 @ S2 - S2 @ P2 @ F) @ X2
        Fs, Es = (Fs + [F])[-8:], (Es + [err])[-8:]
        Fd = _diis(Fs, Es) if len(Fs) > 1 else F
        _, Cp = np.linalg.eigh(X2 @ Fd @ X2)
        C = X2 @ Cp[:, :nel]
        P2 = C @ C.conj().T
        if abs(E - Eold) < conv and np.abs(err).max() < 1e-8:
            break
        Eold = E
    return P2, E
