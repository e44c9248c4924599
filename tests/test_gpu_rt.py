"""GPU real-time path (cq_rt_*, cq_expm, MLP kernels) against the oracle and
against exact identities.  Initial states for oracle comparisons are built
with oracle-only code (oracle SCF, numpy kick)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp, rt, scf
from paper_1905_01381_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.name}", flush=True)
    sys.stdout.flush()
    yield


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    from paper_1905_01381_amd import cq
    cq.lib()
    return torch


def _d(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _kick(X, Dz, Po, kappa):
    U = rt.expm_herm(X @ Dz @ X, kappa)
    return U @ Po @ U.conj().T


@pytest.fixture(scope="module")
def c1_state(torch_cuda):
    from paper_1905_01381_amd import cq
    w = inputs.c1()
    ob = oracle.Basis.from_molecule(w.mol)
    P, h, S, X, E = scf.rhf(ob, w.mol, 3)
    Sh = S @ X
    Po = (Sh @ P @ Sh).astype(complex)
    Dz = ob.one_electron("dipole", direction=2)
    gb = cq.Basis.from_molecule(w.mol)
    return w, ob, gb, h, X, Dz, Po


def test_zgemm_against_numpy(torch_cuda):
    """The matrix-core complex GEMM of the real-time path, A B and A B^H,
    on ragged sizes (tiles of 32, K chunks of 16) against numpy."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    rng = np.random.default_rng(9)
    for n in (1, 5, 16, 31, 33, 100, 257):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        for conj in (False, True):
            C = cq.zgemm(_d(torch, A), _d(torch, B), conj).cpu().numpy()
            ref = A @ (B.conj().T if conj else B)
            assert np.abs(C - ref).max() < 1e-13 * n * np.abs(A).max() * np.abs(B).max(), (n, conj)


def test_expm_against_eigendecomposition(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    rng = np.random.default_rng(2)
    n = 48
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = 30.0 * (A + A.conj().T)
    for dt in (0.05, 1e-3):
        U = cq.expm(_d(torch, H), dt).cpu().numpy()
        ref = rt.expm_herm(H, dt)
        assert np.abs(U - ref).max() < 1e-11
        assert np.abs(U @ U.conj().T - np.eye(n)).max() < 1e-12


def test_em2_steps_against_oracle(c1_state, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    P0 = _kick(X, Dz, Po, 1e-2)
    r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, P0), 0.05, cq.RT_EM2)
    _, mu, nb = r.step(3)
    Pg = r.density().cpu().numpy()
    P = P0
    for _ in range(3):
        P = rt.em2_step(ob, h, X, P, 0.05)
    assert list(nb) == [2, 2, 2]
    assert np.abs(Pg - P).max() < 1e-10 * np.abs(P).max()
    _, mu_ref = rt.energy_dipole(ob, h, X, Dz, P)
    assert abs(mu[-1] - mu_ref) < 1e-10


def test_ground_state_stationary(c1_state, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, Po), 0.05, cq.RT_EM2)
    r.step(10, dipole=False)
    assert np.abs(r.density().cpu().numpy() - Po).max() < 1e-8


def test_invariants_midpoint(c1_state, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    P0 = _kick(X, Dz, Po, 1e-2)
    r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, P0), 0.05, cq.RT_MIDPOINT)
    r.set_params(sc_tol=1e-11, max_iter=40)
    E, mu, nb = r.step(60, energy=True)
    P = r.density().cpu().numpy()
    assert abs(np.trace(P).real - 3.0) < 1e-10
    assert np.abs(P - P.conj().T).max() < 1e-13
    assert np.abs(P @ P - P).max() < 1e-9
    drift = np.abs(E - E[0]).max()
    print(f"midpoint: builds/step {nb[3:].mean():.2f}, energy drift {drift:.2e}, dipole range {np.ptp(mu):.2e}",
          flush=True)
    # second-order Magnus steps conserve the field-free energy to O(dt^2)
    assert drift < 1e-5
    assert np.ptp(mu) > 1e-6


def test_second_order_in_dt(c1_state, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    P0 = _kick(X, Dz, Po, 1e-2)
    out = []
    for dt in (0.02, 0.01, 0.005):
        r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, P0), dt, cq.RT_EM2)
        r.step(int(round(0.2 / dt)), dipole=False)
        out.append(r.density().cpu().numpy())
        r.close()
    ratio = np.abs(out[0] - out[2]).max() / np.abs(out[1] - out[2]).max()
    assert 4.0 < ratio < 6.0, ratio


def test_mmut_against_oracle(c1_state, torch_cuda):
    """MMUT (the paper's default leap-frog integrator) with EM2 seed and
    restart every 4 steps against the oracle's MMUT trajectory: step types,
    densities at 1e-10 after 9 steps, and the dipole."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    P0 = _kick(X, Dz, Po, 1e-2)
    r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, P0), 0.05, cq.RT_MMUT)
    r.set_restart(4)
    _, mu, nb = r.step(9)
    Pg = r.density().cpu().numpy()
    Ps, nb_ref = rt.mmut_trajectory(ob, h, X, P0, 0.05, 9, restart=4)
    assert list(nb) == nb_ref == [2, 1, 1, 1, 2, 1, 1, 1, 2]
    assert np.abs(Pg - Ps[-1]).max() < 1e-10 * np.abs(Ps[-1]).max()
    _, mu_ref = rt.energy_dipole(ob, h, X, Dz, Ps[-1])
    assert abs(mu[-1] - mu_ref) < 1e-9
    assert abs(np.trace(Pg).real - 3.0) < 1e-10


@pytest.mark.parametrize("mode", ["em2", "midpoint", "mmut"])
def test_field_trajectory_against_oracle(c1_state, torch_cuda, mode):
    """A plane-wave field switched on at t = 0.1 (Eq. td_pert) from the
    ground state: every integrator against the oracle's trajectory with the
    same field (densities at 1e-10 after 8 steps, dipole, and the energy
    including the interaction)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    dt, n = 0.05, 8
    kappa, omega, t_on = 0.05, 6.0, 0.1
    field = (Dz, rt.envelope(3, kappa, omega, t_on, 1e9))
    m = {"em2": cq.RT_EM2, "midpoint": cq.RT_MIDPOINT, "mmut": cq.RT_MMUT}[mode]
    r = cq.RT(gb, _d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, Po.copy()), dt, m)
    r.set_field("plane_wave", kappa, omega, t_on)
    r.set_params(sc_tol=1e-13, max_iter=60, accept_tol=1e-13)
    r.set_restart(3)
    E, mu, nb = r.step(n, energy=True)
    Pg = r.density().cpu().numpy()
    if mode == "mmut":
        Ps, _ = rt.mmut_trajectory(ob, h, X, Po, dt, n, 3, field=field)
        P = Ps[-1]
    else:
        P = Po.copy()
        for k in range(n):
            if mode == "em2" or k < 3:
                # the GPU's midpoint mode starts with EM2 steps until it has a history
                P = rt.em2_step(ob, h, X, P, dt, k * dt, field)
            else:
                P, _, _ = rt.midpoint_step(ob, h, X, P, dt, tol=1e-14, t=k * dt, field=field)
    assert np.abs(P - Po).max() > 1e-5
    assert np.abs(Pg - P).max() < 1e-10 * np.abs(P).max(), np.abs(Pg - P).max()
    E_ref, mu_ref = rt.energy_dipole(ob, h, X, Dz, P, t=n * dt, field=field)
    assert abs(mu[-1] - mu_ref) < 1e-9
    assert abs(E[-1] - E_ref) < 1e-9


def test_mlp_kernels_against_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    rng = np.random.default_rng(7)
    w = (rng.standard_normal(354) * 0.3).astype(np.float32)
    X = rng.standard_normal((3000, 8)).astype(np.float32)
    Y = rng.standard_normal((3000, 2)).astype(np.float32)
    loss, g = cq.mlp_eval(_d(torch, w), _d(torch, X), _d(torch, Y))
    lr, gr = mlp.loss_grad(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert float(loss.cpu()) == pytest.approx(lr, rel=1e-4)
    g = g.cpu().numpy().astype(np.float64)
    assert np.abs(g - gr).max() < 1e-4 * np.abs(gr).max()
    m = np.zeros(354, np.float32)
    v = np.zeros(354, np.float32)
    wd, gd, md, vd = _d(torch, w.copy()), _d(torch, g.astype(np.float32)), _d(torch, m), _d(torch, v)
    cq.mlp_adam(wd, gd, md, vd, 1e-2, 1)
    wr, _, _ = mlp.adam(w.astype(np.float64), g, m.astype(np.float64), v.astype(np.float64), 1e-2, 1)
    assert np.abs(wd.cpu().numpy() - wr).max() < 1e-6


def test_learned_proposal_vs_plain(c1_state, torch_cuda):
    """The learned proposal against the plain self-consistent midpoint and
    against its own ablation, every run accepting a first midpoint iterate at
    the same tolerance (1e-6): the network is trained on the first 150 steps
    of the run, then propagates 150 more steps.  The learned run needs fewer
    builds per step than both, and its dipole stays within 1e-5 a.u. of a
    plain run converged to 1e-10.  The ablation zeroes the network, leaving
    the proposal baseline (the midpoint of P_k and the previous step's
    propagator applied to P_k)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, h, X, Dz, Po = c1_state
    P0 = _kick(X, Dz, Po, 1e-3)
    dt, ntrain, nrun = 0.05, 150, 150
    args = (_d(torch, h), _d(torch, X), _d(torch, Dz), _d(torch, P0))
    plain = cq.RT(gb, *args, dt, cq.RT_MIDPOINT)
    plain.set_params(sc_tol=1e-10, max_iter=40)
    _, mu_all, _ = plain.step(ntrain + nrun)
    mu_plain = mu_all[ntrain:]
    same = cq.RT(gb, *args, dt, cq.RT_MIDPOINT)
    same.set_params(sc_tol=1e-10, max_iter=40, accept_tol=1e-6)
    _, _, nb_all = same.step(ntrain + nrun)
    nb_plain = nb_all[ntrain:]

    def trained_run(epochs, zero, acc):
        r = cq.RT(gb, *args, dt, cq.RT_MIDPOINT)
        r.set_params(sc_tol=1e-10, max_iter=40, accept_tol=acc)
        r.record(True, 4096, 1)
        r.step(ntrain)
        r.record(False)
        loss = r.train(epochs=epochs, lr=3e-3)
        if zero:
            r.weights(np.zeros(354, np.float32))
        r.set_mode(cq.RT_LEARNED)
        _, mu, nb = r.step(nrun)
        print(f"  epochs {epochs}: loss {loss:.3e}, target scale {r.scales()[1]:.3e}, stats {r.stats()}, "
              f"max dipole diff {np.abs(mu - mu_plain).max():.2e}", flush=True)
        return loss, mu, nb, r.stats()

    # a proposal is accepted when the midpoint it produces reproduces it to
    # 1e-6: well inside the O(dt^3) local error of the second-order step
    loss, mu_l, nb_l, st = trained_run(200, False, 1e-6)
    _, mu_z, nb_z, st_z = trained_run(0, True, 1e-6)
    err = np.abs(mu_l - mu_plain).max()
    print(f"train loss {loss:.3e}; builds/step plain {nb_plain.mean():.2f} learned {nb_l.mean():.2f} "
          f"ablation {nb_z.mean():.2f}; max dipole diff {err:.2e}; learned {st}; ablation {st_z}", flush=True)
    assert err < 1e-5
    assert nb_l.mean() < nb_plain.mean()
    assert nb_l.mean() < nb_z.mean()
