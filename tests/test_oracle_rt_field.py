"""Pins of the oracle's time-dependent perturbations (paper: "Real-Time
Electronic Dynamics", Eq. td_pert and the envelope list after it), no GPU.

* A static field switched on for all t: the ground state of h + kappa V is
  stationary under EM2, the self-consistent midpoint and MMUT, while the
  field-free ground state moves (the field enters the Fock matrix with the
  sign and weight of the SCF's h + kappa V).
* A field switched on after the last step changes nothing (the window
  Theta(t - t_on) - Theta(t - t_off)).
* With a plane-wave field EM2 and the midpoint step stay second order:
  halving dt cuts the error ~4x, which fails if the field is evaluated at
  the wrong time within a step (first order).
"""
import numpy as np
import pytest

import oracle
from oracle import rt, scf
from paper_1905_01381_amd import inputs


@pytest.fixture(scope="module")
def c1():
    w = inputs.c1()
    ob = oracle.Basis.from_molecule(w.mol)
    Dz = ob.one_electron("dipole", direction=2)
    return w, ob, Dz


def _ortho(S, X, P):
    Sh = S @ X
    return (Sh @ P @ Sh).astype(complex)


def test_envelopes_window():
    f = rt.envelope(1, 0.3, 0.0, 1.0, 2.0)
    assert f(0.999) == 0.0 and f(1.0) == 0.3 and f(1.999) == 0.3 and f(2.0) == 0.0
    g = rt.envelope(4, 0.5, 3.0, 1.0, 9.0)
    assert g(1.0) == 0.5 and g(1.5) == pytest.approx(0.5 * np.exp(-0.75), rel=1e-15)
    assert rt.envelope(2, 2.0, 0.0, 1.0, 9.0)(1.25) == pytest.approx(0.5)
    assert rt.envelope(3, 1.0, 2.0, 0.5, 9.0)(0.5 + np.pi / 4) == pytest.approx(0.0, abs=1e-15)


def test_static_field_ground_state_stationary(c1):
    w, ob, Dz = c1
    kappa = 0.05
    P, h, S, X, E = scf.rhf(ob, w.mol, 3, h_add=kappa * Dz)
    h0 = h - kappa * Dz
    Po = _ortho(S, X, P)
    field = (Dz, rt.envelope(1, kappa, 0.0, 0.0, 1e9))
    dt = 0.05
    assert np.abs(rt.em2_step(ob, h0, X, Po, dt, 0.0, field) - Po).max() < 1e-8
    P1, _, _ = rt.midpoint_step(ob, h0, X, Po, dt, tol=1e-13, t=0.0, field=field)
    assert np.abs(P1 - Po).max() < 1e-8
    Ps, _ = rt.mmut_trajectory(ob, h0, X, Po, dt, 4, 3, field=field)
    assert max(np.abs(Q - Po).max() for Q in Ps) < 1e-8
    # without the field the same density is not stationary
    assert np.abs(rt.em2_step(ob, h0, X, Po, dt) - Po).max() > 1e-5


def test_field_outside_window_changes_nothing(c1):
    w, ob, Dz = c1
    P, h, S, X, E = scf.rhf(ob, w.mol, 3)
    Po = _ortho(S, X, P)
    U = rt.expm_herm(X @ Dz @ X, 1e-2)
    P0 = U @ Po @ U.conj().T
    late = (Dz, rt.envelope(3, 0.1, 1.5, 10.0, 20.0))
    Pa, Pb = P0, P0
    for k in range(4):
        Pa = rt.em2_step(ob, h, X, Pa, 0.05, k * 0.05, late)
        Pb = rt.em2_step(ob, h, X, Pb, 0.05, k * 0.05)
    # equal up to the oracle's threaded summation order
    assert np.abs(Pa - Pb).max() < 1e-13


@pytest.mark.parametrize("stepper", ["em2", "midpoint"])
def test_plane_wave_second_order(c1, stepper):
    w, ob, Dz = c1
    P, h, S, X, E = scf.rhf(ob, w.mol, 3)
    Po = _ortho(S, X, P)
    field = (Dz, rt.envelope(3, 0.05, 6.0, 0.0, 1e9))
    T = 0.16

    def run(dt):
        Q = Po.copy()
        for k in range(int(round(T / dt))):
            if stepper == "em2":
                Q = rt.em2_step(ob, h, X, Q, dt, k * dt, field)
            else:
                Q, _, _ = rt.midpoint_step(ob, h, X, Q, dt, tol=1e-14, t=k * dt, field=field)
        return Q

    Pa, Pb, Pc = run(0.04), run(0.02), run(0.01)
    assert np.abs(Pc - Po).max() > 1e-4  # the field drives the density
    ratio = np.abs(Pa - Pc).max() / np.abs(Pb - Pc).max()
    # errors e(dt) ~ C dt^2: (e(4h) - e(h)) / (e(2h) - e(h)) = 15 / 3 = 5
    assert 4.0 < ratio < 6.0, ratio
