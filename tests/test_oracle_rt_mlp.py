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
