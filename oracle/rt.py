"""Real-time step of the oracle (TEST INFRASTRUCTURE): the paper's EM2
propagator ("Real-Time Electronic Dynamics") in the orthonormal basis with the
exponential by Hermitian eigendecomposition (the exact-diagonalization option
the paper lists), and Fock matrices from the oracle's own J/K.

  F_FE-step: U_FE = exp(-i dt F'(P_k)), P_FE = U_FE P_k U_FE^dagger
  F'_m = (F'(P_k) + F'(P_FE)) / 2,  U = exp(-i dt F'_m),  P_{k+1} = U P_k U^dagger
Closed shell, per-spin P: F = h + 2 J[Re P] - K[Re P] - i K[Im P].

Also the self-consistent midpoint step (midpoint_step) and the paper's
default leap-frog integrator, MMUT, with EM2 seed and restart steps
(mmut_step, mmut_trajectory).

External perturbations (Eq. td_pert): F(P, t) = F_0(P) + f(t) V with
f(t) = kappa g(t) (Theta(t - t_on) - Theta(t - t_off)), g one of the paper's
envelopes (step, linear ramp, plane wave, Gaussian), Theta(0) = 1.  Each step
function takes the time t of P_k and a `field` (V, f) or None; the Fock
matrix of a density at time s uses h + f(s) V (EM2: t and t + dt; midpoint:
t + dt/2; MMUT: t).
"""
from __future__ import annotations

import numpy as np


def expm_herm(H: np.ndarray, dt: float) -> np.ndarray:
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * dt * w)) @ V.conj().T


ENVELOPES = {1: "step", 2: "linear ramp", 3: "plane wave", 4: "gaussian"}


def envelope(kind: int, kappa: float, param: float, t_on: float, t_off: float):
    """f(t) of one perturbation; param is omega (plane wave) or alpha (Gaussian)."""
    def f(t):
        if not (t >= t_on and not t >= t_off):
            return 0.0
        u = t - t_on
        g = {1: 1.0, 2: u, 3: np.cos(param * u), 4: np.exp(-param * u * u)}[kind]
        return kappa * g
    return f


def h_at(h, field, t):
    """Core Hamiltonian plus the perturbation at time t."""
    if field is None:
        return h
    V, f = field
    return h + f(t) * V


def fock_ortho(basis, h, X, Po):
    P = X @ Po @ X
    J, K = basis.jk(np.stack([P.real, P.imag]))
    F = h + 2.0 * J[0] - K[0] - 1j * K[1]
    return X @ F @ X, P, F


def em2_step(basis, h, X, Po, dt, t=0.0, field=None):
    Fk, _, _ = fock_ortho(basis, h_at(h, field, t), X, Po)
    U = expm_herm(Fk, dt)
    Pfe = U @ Po @ U.conj().T
    Ffe, _, _ = fock_ortho(basis, h_at(h, field, t + dt), X, Pfe)
    Um = expm_herm(0.5 * (Fk + Ffe), dt)
    return Um @ Po @ Um.conj().T


def energy_dipole(basis, h, X, Dz, Po, enuc=0.0, mu_nuc=0.0, t=0.0, field=None):
    ht = h_at(h, field, t)
    _, P, F = fock_ortho(basis, ht, X, Po)
    E = float(np.real(np.sum(P * np.conj(ht + F)))) + enuc
    mu = -2.0 * float(np.real(np.sum(P * Dz))) + mu_nuc
    return E, mu


def midpoint_step(basis, h, X, Po, dt, guess=None, tol=1e-12, max_iter=200, t=0.0, field=None):
    """Self-consistent midpoint Magnus-2 step (the corrector the survey
    names as the judge of the learned proposal): the midpoint density is
    iterated to a fixed point,
      P_mid^(i+1) = (P_k + U_i P_k U_i^dagger) / 2,  U_i = exp(-i dt F'(P_mid^(i))),
    starting from `guess` (default P_k), until max|P_mid^(i+1) - P_mid^(i)|
    < tol.  Returns (P_{k+1}, P_mid, iterations); P_{k+1} is the density the
    last evaluated propagator gives."""
    Pm = Po.copy() if guess is None else guess.copy()
    hm = h_at(h, field, t + 0.5 * dt)
    for it in range(1, max_iter + 1):
        F, _, _ = fock_ortho(basis, hm, X, Pm)
        U = expm_herm(F, dt)
        Pn = U @ Po @ U.conj().T
        Pm_new = 0.5 * (Po + Pn)
        d = np.abs(Pm_new - Pm).max()
        Pm = Pm_new
        if d < tol:
            return Pn, Pm, it
    raise RuntimeError("midpoint iteration did not converge")


def mmut_step(basis, h, X, P_prev, P_cur, dt, t=0.0, field=None):
    """One leap-frog step of the modified midpoint unitary transformation
    (paper: "Real-Time Electronic Dynamics", the MMUT propagator):
    P_{k+1} = U P_{k-1} U^dagger with U = exp(-2 i dt F'(P_k)), t the time of P_k."""
    F, _, _ = fock_ortho(basis, h_at(h, field, t), X, P_cur)
    U = expm_herm(F, 2.0 * dt)
    return U @ P_prev @ U.conj().T


def mmut_trajectory(basis, h, X, P0, dt, nsteps, restart, field=None):
    """MMUT with the paper's seed/restart step: step 0 -> 1 and every step
    k with k % restart == 0 is an EM2 step from P_k alone; the others are
    leap-frog steps.  Returns the list [P_0, ..., P_nsteps] and the Fock
    builds each step used."""
    Ps = [P0]
    builds = []
    for k in range(nsteps):
        if k % restart == 0:
            Ps.append(em2_step(basis, h, X, Ps[-1], dt, k * dt, field))
            builds.append(2)
        else:
            Ps.append(mmut_step(basis, h, X, Ps[-2], Ps[-1], dt, k * dt, field))
            builds.append(1)
    return Ps, builds
