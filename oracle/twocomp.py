"""Two-component (Pauli spin basis) pieces of the oracle (TEST INFRASTRUCTURE).

Paper, "General Infrastructure for the Unified Treatment of Electronic Spin":
* Eq. pauli_sep: X^{2C} = sum_I X^I (x) sigma_I with
  2X^0 = X^aa + X^bb, 2X^1 = X^ab + X^ba, -2i X^2 = X^ab - X^ba,
  2X^3 = X^aa - X^bb.
* Eq. 2c_expectation: Tr[O^{2C} P^{2C}] = 2 sum_I Tr[O^I P^I].
Paper, "Reference Wave Functions", Eq. 2c_fock, read with the factor that
the half in Eq. pauli_sep implies (with P^0 = (P^aa + P^bb)/2, the Coulomb
term of the full density is 2 J[P^0]):
  G^0 = 2 J[P^0] - K[P^0],   G^k = -K[P^k]   (k = 1, 2, 3).

The spin-blocked matrix is [[X^aa, X^ab], [X^ba, X^bb]] (rows/columns: all
alpha functions, then all beta functions).
"""
from __future__ import annotations

import numpy as np


def split(X2c: np.ndarray) -> list[np.ndarray]:
    """Spin-blocked 2n x 2n -> [X^0, X^1, X^2, X^3] (each n x n, complex)."""
    n = X2c.shape[0] // 2
    aa, ab = X2c[:n, :n], X2c[:n, n:]
    ba, bb = X2c[n:, :n], X2c[n:, n:]
    x0 = 0.5 * (aa + bb)
    x1 = 0.5 * (ab + ba)
    x2 = (ab - ba) / (-2j)
    x3 = 0.5 * (aa - bb)
    return [x0, x1, x2, x3]


PAULI = [
    np.eye(2, dtype=complex),
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
]


def merge(comps: list[np.ndarray]) -> np.ndarray:
    """[X^0..X^3] -> spin-blocked sum_I sigma_I kron X^I."""
    out = 0
    for s, x in zip(PAULI, comps):
        out = out + np.kron(s, x)
    return out


def real_parts(comps: list[np.ndarray]) -> tuple[np.ndarray, list[int]]:
    """The eight real matrices of a Hermitian Pauli set: Re X^0..3 (symmetric)
    then Im X^0..3 (antisymmetric); returns (stack, sym flags)."""
    mats = [c.real for c in comps] + [c.imag for c in comps]
    return np.stack(mats), [1, 1, 1, 1, -1, -1, -1, -1]


def fock2e_components(J0: np.ndarray, Kre: list[np.ndarray], Kim: list[np.ndarray]) -> list[np.ndarray]:
    """G^0 = 2J[P^0] - K[P^0]; G^k = -K[P^k], with K[P^I] = K[Re] + i K[Im]."""
    K = [kr + 1j * ki for kr, ki in zip(Kre, Kim)]
    return [2.0 * J0 - K[0], -K[1], -K[2], -K[3]]


def fock2e(basis, P2c: np.ndarray, full: bool = False) -> tuple[np.ndarray, dict]:
    """Two-electron part of the 2C Fock matrix, G^{2C}, from the oracle J/K."""
    comps = split(P2c)
    stack, _ = real_parts(comps)
    fn = basis.jk_full if full else basis.jk
    J, _ = fn(stack[0], want_j=True, want_k=False)
    _, K = fn(stack, want_j=False, want_k=True)
    G = fock2e_components(J, list(K[:4]), list(K[4:]))
    return merge(G), {"J0": J, "K": K, "comps": comps, "G": G}


def energy_2e_2c(P2c: np.ndarray, G2c: np.ndarray) -> float:
    """E_2e = 1/2 Tr[P^{2C} G^{2C}]."""
    return 0.5 * float(np.real(np.trace(P2c @ G2c)))


def energy_2e_closed(P: np.ndarray, J: np.ndarray, K: np.ndarray) -> float:
    """Closed shell with P the per-spin density: E_2e = 2 Tr(PJ) - Tr(PK)."""
    return float(2.0 * np.sum(P * J) - np.sum(P * K))
