"""Pins of the oracle's real-time step and MLP (no GPU).

* exp(-i dt H) by eigendecomposition: unitary; equals the closed form for a
  diagonal H and for a 2x2 rotation generator.
* EM2 leaves a converged ground state stationary (it commutes with its own
  Fock matrix), conserves the trace and keeps the density Hermitian.
* EM2 is second order: halving dt cuts the error at fixed time ~4x.
* The MLP gradient matches central finite differences; one Adam step matches
  the published update written out for a single parameter.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp, rt, scf
from paper_1905_01381_amd import inputs


def test_expm_closed_forms():
    d = np.array([0.3, -1.2, 2.5])
    U = rt.expm_herm(np.diag(d), 0.7)
    assert np.allclose(U, np.diag(np.exp(-0.7j * d)), atol=1e-15)
    H = np.array([[0.0, 1.0], [1.0, 0.0]])
    U = rt.expm_herm(H, 0.4)
    ref = np.array([[np.cos(0.4), -1j * np.sin(0.4)], [-1j * np.sin(0.4), np.cos(0.4)]])
    assert np.allclose(U, ref, atol=1e-15)
    rng = np.random.default_rng(0)
    A = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    U = rt.expm_herm(A + A.conj().T, 0.3)
    assert np.abs(U @ U.conj().T - np.eye(20)).max() < 1e-13


@pytest.fixture(scope="module")
def ground():
    w = inputs.c1()
    ob = oracle.Basis.from_molecule(w.mol)
    P, h, S, X, E = scf.rhf(ob, w.mol, 3)
    Sh = S @ X
    Po = (Sh @ P @ Sh).astype(complex)
    Dz = ob.one_electron("dipole", direction=2)
    return w, ob, h, X, Dz, Po


def test_em2_ground_state_stationary(ground):
    w, ob, h, X, Dz, Po = ground
    P1 = rt.em2_step(ob, h, X, Po, 0.05)
    assert np.abs(P1 - Po).max() < 1e-8
    assert abs(np.trace(P1).real - 3.0) < 1e-12


def _kick(X, Dz, Po, kappa):
    U = rt.expm_herm(X @ Dz @ X, kappa)
    return U @ Po @ U.conj().T


def test_em2_trace_hermitian_and_second_order(ground):
    w, ob, h, X, Dz, Po = ground
    P0 = _kick(X, Dz, Po, 1e-2)
    T = 0.2

    def run(dt):
        P = P0.copy()
        for _ in range(int(round(T / dt))):
            P = rt.em2_step(ob, h, X, P, dt)
        return P

    Pa, Pb, Pc = run(0.02), run(0.01), run(0.005)
    for P in (Pa, Pb, Pc):
        assert abs(np.trace(P).real - 3.0) < 1e-11
        assert np.abs(P - P.conj().T).max() < 1e-13
        assert np.abs(P @ P - P).max() < 1e-10
    ratio = np.abs(Pa - Pc).max() / np.abs(Pb - Pc).max()
    # errors e(dt) ~ C dt^2: (e(4h) - e(h)) / (e(2h) - e(h)) = 15 / 3 = 5
    assert 4.0 < ratio < 6.0, ratio


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(354) * 0.3
    X = rng.standard_normal((50, 8))
    Y = rng.standard_normal((50, 2))
    _, g = mlp.loss_grad(w, X, Y)
    for k in rng.choice(354, 25, replace=False):
        e = np.zeros(354); e[k] = 1e-6
        fd = (mlp.loss_grad(w + e, X, Y)[0] - mlp.loss_grad(w - e, X, Y)[0]) / 2e-6
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-9)


def test_adam_single_parameter():
    w, m, v = mlp.adam(np.array([1.0]), np.array([0.5]), np.zeros(1), np.zeros(1), 0.01, 1)
    # first step: m_hat = g, v_hat = g^2 -> w - lr * g/(|g| + eps)
    assert w[0] == pytest.approx(1.0 - 0.01 * 0.5 / (0.5 + 1e-8), rel=1e-15)


# ------------------------------------------------------------ midpoint / MMUT
def test_midpoint_fixed_point_and_reversibility(ground):
    """The converged midpoint satisfies its own fixed-point equation, and
    the step is time-symmetric: a step of -dt from P_{k+1} returns P_k."""
    w, ob, h, X, Dz, Po = ground
    P0 = _kick(X, Dz, Po, 1e-2)
    P1, Pm, it = rt.midpoint_step(ob, h, X, P0, 0.05, tol=1e-13)
    assert it > 2
    F, _, _ = rt.fock_ortho(ob, h, X, Pm)
    U = rt.expm_herm(F, 0.05)
    assert np.abs(0.5 * (P0 + U @ P0 @ U.conj().T) - Pm).max() < 1e-12
    assert np.abs(P1 - P0).max() > 1e-4
    Pback, _, _ = rt.midpoint_step(ob, h, X, P1, -0.05, guess=Pm, tol=1e-13)
    assert np.abs(Pback - P0).max() < 1e-11
    # an explicit step with the Fock matrix of P_k alone is not reversible
    Fk, _, _ = rt.fock_ortho(ob, h, X, P0)
    Uk = rt.expm_herm(Fk, 0.05)
    Pe = Uk @ P0 @ Uk.conj().T
    Fe, _, _ = rt.fock_ortho(ob, h, X, Pe)
    Ue = rt.expm_herm(Fe, -0.05)
    assert np.abs(Ue @ Pe @ Ue.conj().T - P0).max() > 1e-6


def test_midpoint_invariants_and_second_order(ground):
    w, ob, h, X, Dz, Po = ground
    P1, _, _ = rt.midpoint_step(ob, h, X, Po, 0.05, tol=1e-13)
    assert np.abs(P1 - Po).max() < 1e-8
    P0 = _kick(X, Dz, Po, 1e-2)
    T = 0.16

    def run(dt):
        P, prev = P0.copy(), None
        for _ in range(int(round(T / dt))):
            guess = None if prev is None else P + 0.5 * (P - prev)
            prev = P
            P, _, _ = rt.midpoint_step(ob, h, X, P, dt, guess=guess, tol=1e-14)
        return P

    Pa, Pb, Pc = run(0.04), run(0.02), run(0.01)
    for P in (Pa, Pb, Pc):
        assert abs(np.trace(P).real - 3.0) < 1e-11
        assert np.abs(P - P.conj().T).max() < 1e-13
        assert np.abs(P @ P - P).max() < 1e-10
    ratio = np.abs(Pa - Pc).max() / np.abs(Pb - Pc).max()
    assert 4.0 < ratio < 6.0, ratio


def test_mmut_leapfrog_reversible_and_second_order(ground):
    """MMUT: P_{k-1} = U^dagger P_{k+1} U with the same U (leap-frog
    reversibility); ground state stationary; second order in dt with the
    EM2 seed step; invariants conserved."""
    w, ob, h, X, Dz, Po = ground
    Ps, nb = rt.mmut_trajectory(ob, h, X, Po, 0.05, 6, restart=1000)
    assert nb == [2, 1, 1, 1, 1, 1]
    assert max(np.abs(P - Po).max() for P in Ps) < 1e-8
    P0 = _kick(X, Dz, Po, 1e-2)
    Ps, _ = rt.mmut_trajectory(ob, h, X, P0, 0.05, 3, restart=1000)
    P3 = rt.mmut_step(ob, h, X, Ps[1], Ps[2], 0.05)
    assert np.abs(P3 - Ps[3]).max() < 1e-13
    back = rt.mmut_step(ob, h, X, P3, Ps[2], -0.05)
    assert np.abs(back - Ps[1]).max() < 1e-12
    T = 0.2

    def run(dt):
        Ps, _ = rt.mmut_trajectory(ob, h, X, P0, dt, int(round(T / dt)), restart=1000)
        return Ps[-1]

    Pa, Pb, Pc = run(0.02), run(0.01), run(0.005)
    for P in (Pa, Pb, Pc):
        assert abs(np.trace(P).real - 3.0) < 1e-11
        assert np.abs(P - P.conj().T).max() < 1e-13
        assert np.abs(P @ P - P).max() < 1e-10
    ratio = np.abs(Pa - Pc).max() / np.abs(Pb - Pc).max()
    assert 4.0 < ratio < 6.0, ratio
    # with restarts every 4 steps the step types alternate as the paper describes
    _, nb = rt.mmut_trajectory(ob, h, X, P0, 0.05, 9, restart=4)
    assert nb == [2, 1, 1, 1, 2, 1, 1, 1, 2]
