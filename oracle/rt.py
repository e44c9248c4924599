"""Real-time step of the oracle (TEST INFRASTRUCTURE): the paper's EM2
propagator ("Real-Time Electronic Dynamics") in the orthonormal basis with the
exponential by Hermitian eigendecomposition (the exact-diagonalization option
the paper lists), and Fock matrices from the oracle's own J/K.

  F_FE-step: U_FE = exp(-i dt F'(P_k)), P_FE = U_FE P_k U_FE^dagger
  F'_m = (F'(P_k) + F'(P_FE)) / 2,  U = exp(-i dt F'_m),  P_{k+1} = U P_k U^dagger
Closed shell, per-spin P: F = h + 2 J[Re P] - K[Re P] - i K[Im P].
"""
from __future__ import annotations

import numpy as np


def expm_herm(H: np.ndarray, dt: float) -> np.ndarray:
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * dt * w)) @ V.conj().T


def fock_ortho(basis, h, X, Po):
    P = X @ Po @ X
    J, Kr = basis.jk(P.real)
    _, Ki = basis.jk(P.imag, want_j=False)
    F = h + 2.0 * J - Kr - 1j * Ki
    return X @ F @ X, P, F


def em2_step(basis, h, X, Po, dt):
    Fk, _, _ = fock_ortho(basis, h, X, Po)
    U = expm_herm(Fk, dt)
    Pfe = U @ Po @ U.conj().T
    Ffe, _, _ = fock_ortho(basis, h, X, Pfe)
    Um = expm_herm(0.5 * (Fk + Ffe), dt)
    return Um @ Po @ Um.conj().T


def energy_dipole(basis, h, X, Dz, Po, enuc=0.0, mu_nuc=0.0):
    _, P, F = fock_ortho(basis, h, X, Po)
    E = float(np.real(np.sum(P * np.conj(h + F)))) + enuc
    mu = -2.0 * float(np.real(np.sum(P * Dz))) + mu_nuc
    return E, mu
