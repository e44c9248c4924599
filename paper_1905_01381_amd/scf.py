"""Ground-state Hartree-Fock driver (paper: "General Infrastructure for the
Unified Treatment of Electronic Spin", Eqs. rh_1c and rh_2c; "Self-Consistent
Field Optimization"): spin restricted (RS), spin unrestricted (US) and
generalized spin (GS) Roothaan-Hall iterations with damping and DIIS.

Every Coulomb/exchange matrix comes from the library (cq_jk_build, or
cq_fock2e_2c for GS); the small dense eigenproblems of the Roothaan-Hall
equations are solved on the host with LAPACK through numpy, setup work around
the integral-direct builds.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SCFResult:
    P: np.ndarray          # per-spin AO density
    C: np.ndarray          # occupied orbitals
    energy: float          # total energy (electronic + nuclear repulsion)
    e_nuc: float
    h: np.ndarray
    S: np.ndarray
    X: np.ndarray          # S^{-1/2}
    iterations: int
    converged: bool


def nuclear_repulsion(Z, R) -> float:
    e = 0.0
    for i in range(len(Z)):
        for j in range(i):
            e += Z[i] * Z[j] / np.linalg.norm(R[i] - R[j])
    return float(e)


def _diis_extrapolate(Fs, Es):
    """Pulay DIIS: the combination of stored Fock matrices with coefficients
    summing to one that minimizes the norm of the combined commutator error."""
    m = len(Fs)
    B = -np.ones((m + 1, m + 1))
    B[m, m] = 0.0
    for i in range(m):
        for j in range(m):
            B[i, j] = float(np.real(np.vdot(Es[i], Es[j])))
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(B, rhs)[:m]
    return sum(ci * fi for ci, fi in zip(c, Fs))


def scf(gb, mol, kind: str = "RS", nalpha: int | None = None, nbeta: int | None = None, guess=None,
        maxiter: int = 200, conv: float = 1e-9, diis_n: int = 8, damping: float = 0.0, damp_until: float = 1e-2,
        verbose: bool = False) -> SCFResult:
    """Hartree-Fock ground state.

    kind "RS": closed shell, P per spin, F = h + 2 J[P] - K[P] (nalpha = nbeta
    doubly occupied orbitals); "US": F^s = h + J[P^a + P^b] - K[P^s]
    (Eq. rh_1c, two coupled eigenproblems); "GS": F^{2C} = h (x) 1 + G^{2C}
    (Eq. rh_2c, one eigenproblem of twice the dimension; nalpha + nbeta
    electrons).  guess: an initial density of the matching form (RS / US: the
    per-spin matrices, US as (Pa, Pb); GS: the 2n x 2n spin-blocked complex
    matrix); default the core-Hamiltonian guess.  damping: while the largest
    commutator error exceeds damp_until, the new density is mixed with
    `damping` of the old one.  Returns the converged density in `P` (US:
    array [2, n, n]; GS: complex [2n, 2n]) and orbitals in `C`."""
    import torch
    kind = kind.upper()
    if kind not in ("RS", "US", "GS"):
        raise ValueError("kind must be RS, US or GS")
    if nalpha is None:
        raise ValueError("nalpha is required")
    nbeta = nalpha if nbeta is None else nbeta
    if kind == "RS" and nalpha != nbeta:
        raise ValueError("RS needs nalpha == nbeta")
    S = gb.one_electron("overlap").cpu().numpy()
    T = gb.one_electron("kinetic").cpu().numpy()
    V = gb.one_electron("nuclear", charges=mol.charges, centers=mol.atoms).cpu().numpy()
    h = T + V
    lam, U = np.linalg.eigh(S)
    X = (U / np.sqrt(lam)) @ U.T
    enuc = nuclear_repulsion(mol.charges, mol.atoms)
    n = S.shape[0]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def occupy(F, Xm, k):
        _, Cp = np.linalg.eigh(Xm @ F @ Xm)
        C = Xm @ Cp[:, :k]
        return C @ C.conj().T, C

    if kind == "GS":
        Z = np.zeros((n, n))
        S2, h2, X2 = np.block([[S, Z], [Z, S]]), np.block([[h, Z], [Z, h]]), np.block([[X, Z], [Z, X]])
        P = (occupy(h2, X2, nalpha + nbeta)[0] if guess is None else np.asarray(guess)).astype(np.complex128)
    elif kind == "US":
        P = np.stack([occupy(h, X, nalpha)[0], occupy(h, X, nbeta)[0]]) if guess is None else np.stack(guess)
    else:
        P = occupy(h, X, nalpha)[0] if guess is None else np.asarray(guess)
    C = None
    Fs, Es = [], []
    E_old = 0.0
    converged = False
    it = 0
    for it in range(1, maxiter + 1):
        if kind == "RS":
            r = gb.jk([dev(P)])
            J, K = r.J[0].cpu().numpy(), r.K[0].cpu().numpy()
            F = h + 2.0 * J - K
            E = float(np.sum(P * (h + F))) + enuc
            err = X @ (F @ P @ S - S @ P @ F) @ X
        elif kind == "US":
            r = gb.jk([dev(P[0]), dev(P[1])])
            Jt = r.J[0].cpu().numpy() + r.J[1].cpu().numpy()
            F = np.stack([h + Jt - r.K[0].cpu().numpy(), h + Jt - r.K[1].cpu().numpy()])
            E = 0.5 * float(np.sum(P[0] * (h + F[0])) + np.sum(P[1] * (h + F[1]))) + enuc
            err = np.stack([X @ (F[s] @ P[s] @ S - S @ P[s] @ F[s]) @ X for s in range(2)])
        else:
            G = gb.fock2e_2c(dev(P)).cpu().numpy()
            F = h2 + G
            E = 0.5 * float(np.real(np.trace(P @ (h2 + F)))) + enuc
            err = X2 @ (F @ P @ S2 - S2 @ P @ F) @ X2
        Fs, Es = (Fs + [F])[-diis_n:], (Es + [err])[-diis_n:]
        Fd = F
        if len(Fs) > 1:
            try:
                Fd = _diis_extrapolate(Fs, Es)
            except np.linalg.LinAlgError:
                Fd = F
        if kind == "RS":
            P_new, C = occupy(Fd, X, nalpha)
        elif kind == "US":
            (Pa, Ca), (Pb, Cb) = occupy(Fd[0], X, nalpha), occupy(Fd[1], X, nbeta)
            P_new, C = np.stack([Pa, Pb]), (Ca, Cb)
        else:
            P_new, C = occupy(Fd, X2, nalpha + nbeta)
        en = float(np.abs(err).max())
        if damping > 0.0 and en > damp_until:
            P_new = (1.0 - damping) * P_new + damping * P
        dE = abs(E - E_old)
        if verbose:
            print(f"  scf {kind} {it:3d}  E = {E:.12f}  dE = {dE:.2e}  |[F,P]| = {en:.2e}", flush=True)
        E_old = E
        P = P_new
        if dE < conv and en < np.sqrt(conv):
            converged = True
            break
    return SCFResult(P, C, E_old, enuc, h, S, X, it, converged)


def rhf(gb, mol, nocc: int, maxiter: int = 100, conv: float = 1e-9, diis_n: int = 8, verbose=False) -> SCFResult:
    """Closed-shell ground state (the RS case of scf)."""
    return scf(gb, mol, "RS", nocc, nocc, maxiter=maxiter, conv=conv, diis_n=diis_n, verbose=verbose)


def ortho_density(res: SCFResult) -> np.ndarray:
    """P' = S^{1/2} P S^{1/2} (Loewdin orthonormal basis), complex."""
    Sh = res.S @ res.X
    return (Sh @ res.P @ Sh).astype(np.complex128)


def nuclear_dipole(mol, direction: int = 2, origin=(0.0, 0.0, 0.0)) -> float:
    return float(np.sum(mol.charges * (mol.atoms[:, direction] - origin[direction])))
