"""Ground-state setup for the real-time path: closed-shell Hartree-Fock with
damping and DIIS (paper: "Self-Consistent Field Optimization").

Every Coulomb/exchange matrix comes from the library (cq_jk_build); the small
dense eigenproblems of the Roothaan-Hall equations (Eq. rh_1c) are solved on
the host with LAPACK through numpy - setup work outside the propagated path.
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


def rhf(gb, mol, nocc: int, maxiter: int = 100, conv: float = 1e-9, diis_n: int = 8, verbose=False) -> SCFResult:
    import torch
    S = gb.one_electron("overlap").cpu().numpy()
    T = gb.one_electron("kinetic").cpu().numpy()
    V = gb.one_electron("nuclear", charges=mol.charges, centers=mol.atoms).cpu().numpy()
    h = T + V
    lam, U = np.linalg.eigh(S)
    X = (U / np.sqrt(lam)) @ U.T
    enuc = nuclear_repulsion(mol.charges, mol.atoms)

    def density(F):
        w, Cp = np.linalg.eigh(X @ F @ X)
        C = X @ Cp[:, :nocc]
        return C @ C.T, C

    P, C = density(h)
    Fs, Es = [], []
    E_old = 0.0
    converged = False
    it = 0
    for it in range(1, maxiter + 1):
        r = gb.jk([torch.from_numpy(np.ascontiguousarray(P)).cuda()])
        J = r.J[0].cpu().numpy()
        K = r.K[0].cpu().numpy()
        F = h + 2.0 * J - K
        E = float(np.sum(P * (h + F))) + enuc
        err = X @ (F @ P @ S - S @ P @ F) @ X
        Fs.append(F)
        Es.append(err)
        Fs, Es = Fs[-diis_n:], Es[-diis_n:]
        if len(Fs) > 1:
            m = len(Fs)
            B = -np.ones((m + 1, m + 1))
            B[m, m] = 0.0
            for i in range(m):
                for j in range(m):
                    B[i, j] = np.sum(Es[i] * Es[j])
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            try:
                cvec = np.linalg.solve(B, rhs)[:m]
                F = sum(c * f for c, f in zip(cvec, Fs))
            except np.linalg.LinAlgError:
                pass
        P_new, C = density(F)
        dE = abs(E - E_old)
        en = np.abs(err).max()
        if verbose:
            print(f"  scf {it:3d}  E = {E:.12f}  dE = {dE:.2e}  |[F,P]| = {en:.2e}", flush=True)
        E_old = E
        P = P_new
        if dE < conv and en < np.sqrt(conv):
            converged = True
            break
    return SCFResult(P, C, E_old, enuc, h, S, X, it, converged)


def ortho_density(res: SCFResult) -> np.ndarray:
    """P' = S^{1/2} P S^{1/2} (Loewdin orthonormal basis), complex."""
    Sh = res.S @ res.X
    return (Sh @ res.P @ Sh).astype(np.complex128)


def nuclear_dipole(mol, direction: int = 2, origin=(0.0, 0.0, 0.0)) -> float:
    return float(np.sum(mol.charges * (mol.atoms[:, direction] - origin[direction])))
