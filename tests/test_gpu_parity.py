"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the
same seeded inputs.  Tolerance: FP64 J/K within 1e-10 relative per matrix
(max |GPU - oracle| / max |oracle|); individual integrals and the Boys
function to 1e-12 / 1e-13 relative."""
import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import twocomp
from paper_1905_01381_amd import inputs
from tests.gpu_common import case_2c, case_real, rel_err

pytestmark = pytest.mark.gpu

TOL_JK = 1e-10


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.name}", flush=True)
    sys.stdout.flush()
    yield


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1905_01381_amd import cq
    cq.lib()
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_boys_against_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    T = np.concatenate([[0.0, 1e-12, 1e-6, 0.49999, 0.5, 35.99999, 36.0, 36.00001, 49.0, 50.0, 51.0, 120.0, 1e3, 1e5],
                        np.random.default_rng(0).uniform(0, 40, 400)])
    for mmax in (0, 3, 8, 16):
        F = cq.boys(mmax, _dev(torch, T)).cpu().numpy()
        ref = oracle.boys_table(mmax, T)
        err = np.abs(F - ref) / np.maximum(np.abs(ref), 1e-300)
        assert err.max() < 1e-13, (mmax, err.max(), T[np.unravel_index(err.argmax(), err.shape)[0]])


@pytest.fixture(scope="module")
def spd_case(torch_cuda):
    from paper_1905_01381_amd import cq
    w, ob, P = case_real(3, inputs.SHELLS_3S2P1D, seed=11, lo=0.3, hi=50.0)
    gb = cq.Basis.from_molecule(w.mol)
    return w, ob, gb, P


def test_eri_quartets_every_class_and_orientation(spd_case):
    w, ob, gb, _ = spd_case
    ls = w.mol.shell_l
    by_l = {l: [int(s) for s in np.where(ls == l)[0]] for l in (0, 1, 2)}
    rng = np.random.default_rng(1)
    worst = (0.0, None)
    count = 0
    for la, lb, lc, ld in itertools.product(range(3), repeat=4):
        for _ in range(2):
            sh = [by_l[x][rng.integers(len(by_l[x]))] for x in (la, lb, lc, ld)]
            got = gb.eri_quartet(*sh)
            ref = ob.eri_shell(*sh)
            e = rel_err(got, ref)
            worst = max(worst, (e, tuple(sh)), key=lambda t: t[0])
            count += 1
    print(f"worst block relative error {worst[0]:.3e} at shells {worst[1]}", flush=True)
    # Two FP64 algorithms (HRR-based on the GPU, Hermite expansion in the
    # oracle) agree to ~1e-12 per block; 1e-11 is kept, 10x inside the 1e-10
    # bar that J and K must meet.
    assert worst[0] < 1e-11, worst
    assert count == 162


def test_schwarz_against_oracle(spd_case, torch_cuda):
    w, ob, gb, _ = spd_case
    Q = gb.schwarz().cpu().numpy()
    ref = ob.schwarz()
    # two FP64 algorithms (HRR-based here, Hermite expansion in the oracle);
    # the order of the primitive sum moves the largest diagonal blocks by
    # ~1e-12 of the largest factor; 1e-11 is the block bar
    assert np.abs(Q - ref).max() / ref.max() < 1e-11


def _jk_gpu(torch, gb, mats, sym, want_j=True, want_k=True, th=None):
    Ps = [_dev(torch, m) for m in mats]
    r = gb.jk(Ps, sym=sym, want_j=want_j, want_k=want_k, th=th)
    torch.cuda.synchronize()
    J = [j.cpu().numpy() if j is not None else None for j in r.J]
    K = [k.cpu().numpy() if k is not None else None for k in r.K]
    return J, K


def test_c1_full_parity(torch_cuda):
    """6 atoms, 2s1p, nbf 30, 5 orbitals (the small workload) - every element."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.c1()
    ob = oracle.Basis.from_molecule(w.mol)
    P = oracle.density_real(ob.overlap(), w.orbitals)
    gb = cq.Basis.from_molecule(w.mol)
    assert gb.nbf == 30
    J, K = _jk_gpu(torch, gb, [P], [1])
    Jr, Kr = ob.jk_full(P)
    assert rel_err(J[0], Jr) < TOL_JK
    assert rel_err(K[0], Kr) < TOL_JK


def test_multi_density_sym_antisym_spd(spd_case, torch_cuda):
    torch = torch_cuda
    w, ob, gb, P = spd_case
    rng = np.random.default_rng(5)
    A = inputs.random_symmetric(gb.nbf, rng, -1)
    S2 = inputs.random_symmetric(gb.nbf, rng, 1)
    J, K = _jk_gpu(torch, gb, [P, A, S2], [1, -1, 1], want_j=[True, False, True])
    Jr, Kr = ob.jk(np.stack([P, A, S2]))
    assert J[1] is None
    for m in (0, 2):
        assert rel_err(J[m], Jr[m]) < TOL_JK, m
    for m in range(3):
        assert rel_err(K[m], Kr[m]) < TOL_JK, m
    assert np.abs(K[1] + K[1].T).max() < 1e-13 * np.abs(K[1]).max()


def test_sixteen_densities_mixed_symmetry(spd_case, torch_cuda):
    """The maximum number of densities per build (16, mixed symmetric and
    antisymmetric): the exchange partial sums that do not depend on the ket
    shell c are kept per lane in LDS over a task, except where 16 slots of
    them do not fit (the (pp|pp) class), which adds them straight to K'."""
    torch = torch_cuda
    w, ob, gb, P = spd_case
    rng = np.random.default_rng(17)
    sym = [1] + [1 if k % 3 else -1 for k in range(1, 16)]
    mats = [P] + [inputs.random_symmetric(gb.nbf, rng, sym[k]) for k in range(1, 16)]
    J, K = _jk_gpu(torch, gb, mats, sym, want_j=[x == 1 for x in sym])
    Jr, Kr = ob.jk(np.stack(mats))
    for m in range(16):
        if sym[m] == 1:
            assert rel_err(J[m], Jr[m]) < TOL_JK, m
        else:
            assert J[m] is None
        assert rel_err(K[m], Kr[m]) < TOL_JK, m


def test_concurrent_classes_equal_serialized(spd_case, torch_cuda):
    """Classes normally run concurrently on internal streams (the staged ones
    in order on one of them, since they share the stage workspace); with
    per-class timing on they run one after another.  The same plan forms the
    same partial sums and the fixed-point additions are exact, so J and K
    are bitwise equal."""
    torch = torch_cuda
    w, ob, gb, P = spd_case
    rng = np.random.default_rng(23)
    mats = [P, inputs.random_symmetric(gb.nbf, rng, -1)]
    J0, K0 = _jk_gpu(torch, gb, mats, [1, -1], want_j=[True, False])
    gb.profile(True, reset=True)
    J1, K1 = _jk_gpu(torch, gb, mats, [1, -1], want_j=[True, False])
    gb.profile(False)
    assert len(gb.profile_read()) > 0
    assert np.array_equal(J1[0], J0[0])
    for m in range(2):
        assert np.array_equal(K1[m], K0[m]), m


def test_xcd_task_deal_bitwise(spd_case, torch_cuda):
    """Dealing the task list to the XCDs in contiguous eighths (task order
    flag 2) changes which workgroup runs a task, not what a task sums, so
    with exact fixed-point accumulation J and K are bitwise unchanged; the
    grid caps (one wave per task, 2048 waves, ragged task counts) exercise
    the padding of the deal."""
    torch = torch_cuda
    w, ob, gb, P = spd_case
    J0, K0 = _jk_gpu(torch, gb, [P], [1])
    base = gb.plan()
    for grid in (0, 2048, 13):
        gb.set_plan([dict(p, rot=2, grid=grid) for p in base])
        J1, K1 = _jk_gpu(torch, gb, [P], [1])
        assert np.array_equal(J1[0], J0[0]) and np.array_equal(K1[0], K0[0]), grid
    gb.set_plan(base)


def test_tiles_span_rows_and_ragged_tail(torch_cuda):
    """12 atoms of 2s1p: rows of up to 5 tiles of 64 with ragged ends."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, P = case_real(12, inputs.SHELLS_2S1P, seed=3, lo=0.15, hi=30.0)
    gb = cq.Basis.from_molecule(w.mol)
    J, K = _jk_gpu(torch, gb, [P], [1])
    Jr, Kr = ob.jk(P)
    assert rel_err(J[0], Jr) < TOL_JK
    assert rel_err(K[0], Kr) < TOL_JK


def test_accumulate_flag_and_single_shell(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, P = case_real(1, [2], seed=2, nocc=2, lo=0.5, hi=5.0)
    gb = cq.Basis.from_molecule(w.mol)
    Pd = _dev(torch, P)
    J0 = _dev(torch, np.ones_like(P))
    K0 = _dev(torch, np.full_like(P, 2.0))
    gb.jk([Pd], out=([J0], [K0]), th=cq.thresholds(accumulate=True))
    torch.cuda.synchronize()
    Jr, Kr = ob.jk(P)
    assert rel_err(J0.cpu().numpy() - 1.0, Jr) < TOL_JK
    assert rel_err(K0.cpu().numpy() - 2.0, Kr) < TOL_JK


def test_two_component_small_full(torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, P2 = case_2c(3, inputs.SHELLS_3S2P1D, seed=4, lo=0.3, hi=50.0)
    gb = cq.Basis.from_molecule(w.mol)
    G = gb.fock2e_2c(_dev(torch, P2))
    torch.cuda.synchronize()
    Gr, _ = twocomp.fock2e(ob, P2)
    assert rel_err(G.cpu().numpy(), Gr) < TOL_JK
    E = twocomp.energy_2e_2c(P2, G.cpu().numpy())
    Er = twocomp.energy_2e_2c(P2, Gr)
    assert abs(E - Er) < 1e-10 * abs(Er)


def test_screening_bound(torch_cuda):
    """With a skip threshold the change in each element stays within the
    number of skipped quartet contributions times the threshold (loose)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, P = case_real(12, inputs.SHELLS_2S1P, seed=3, lo=0.15, hi=30.0)
    gb = cq.Basis.from_molecule(w.mol)
    J0, K0 = _jk_gpu(torch, gb, [P], [1])
    J1, K1 = _jk_gpu(torch, gb, [P], [1], th=cq.thresholds(skip=1e-9))
    nq = (gb.nshell * (gb.nshell + 1) // 2) ** 2
    assert np.abs(J1[0] - J0[0]).max() <= 8 * nq * 1e-9
    assert np.abs(K1[0] - K0[0]).max() <= 8 * nq * 1e-9
    Jr, Kr = ob.jk(P)
    assert rel_err(J1[0], Jr) < 1e-6


def test_c2_fullsize_sampled_blocks(torch_cuda):
    """The two-component workload at full size (40 atoms, nbf 600): one
    cq_fock2e_2c build, checked on sampled shell blocks that the oracle
    computes straight from the definition."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w = inputs.c2()
    ob = oracle.Basis.from_molecule(w.mol)
    S = ob.overlap()
    P2 = oracle.density_2c(S, w.orbitals)
    gb = cq.Basis.from_molecule(w.mol)
    assert gb.nbf == 600
    G = gb.fock2e_2c(_dev(torch, P2)).cpu().numpy()
    n = gb.nbf
    comps = twocomp.split(P2)
    stack, _ = twocomp.real_parts(comps)
    o = ob.offsets
    ls = w.mol.shell_l
    d_sh = int(np.where(ls == 2)[0][7])
    p_sh = int(np.where(ls == 1)[0][30])
    s_sh = int(np.where(ls == 0)[0][50])
    for a, b in [(d_sh, p_sh), (s_sh, d_sh)]:
        jb = ob.j_block(a, b, stack[:1])[0]
        kb = ob.k_block(a, b, stack)
        Kc = [kb[I] + 1j * kb[4 + I] for I in range(4)]
        Gc = [2 * jb - Kc[0], -Kc[1], -Kc[2], -Kc[3]]
        blocks = {
            (0, 0): Gc[0] + Gc[3], (0, 1): Gc[1] - 1j * Gc[2],
            (1, 0): Gc[1] + 1j * Gc[2], (1, 1): Gc[0] - Gc[3],
        }
        for (s, t), ref in blocks.items():
            got = G[s * n + o[a]: s * n + o[a + 1], t * n + o[b]: t * n + o[b + 1]]
            assert rel_err(got, ref) < TOL_JK, (a, b, s, t, rel_err(got, ref))


def test_one_electron_against_oracle(spd_case, torch_cuda):
    w, ob, gb, _ = spd_case
    mol = w.mol
    for kind in ("overlap", "kinetic"):
        got = gb.one_electron(kind).cpu().numpy()
        ref = ob.one_electron(kind)
        assert rel_err(got, ref) < 1e-12, kind
    for d in range(3):
        got = gb.one_electron("dipole", direction=d, origin=(0.3, -0.2, 0.1)).cpu().numpy()
        ref = ob.one_electron("dipole", direction=d, origin=(0.3, -0.2, 0.1))
        assert rel_err(got, ref) < 1e-12, d
    got = gb.one_electron("nuclear", charges=mol.charges, centers=mol.atoms).cpu().numpy()
    ref = ob.one_electron("nuclear", charges=mol.charges, centers=mol.atoms)
    assert rel_err(got, ref) < 1e-12


def _energy(P, J, K):
    return 2.0 * float(np.sum(P * J)) - float(np.sum(P * K))


def test_routed_all_fp32(spd_case, torch_cuda):
    """Every batch forced to FP32: errors at FP32 level, counters say so."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, gb, P = spd_case
    J, K = _jk_gpu(torch, gb, [P], [1], th=cq.thresholds(mode=1, fp32_below=1e300))
    st = gb.build_stats()
    assert st["fp64"] == 0 and st["fp32"] > 0 and st["skipped"] == 0
    Jr, Kr = ob.jk(P)
    scale = np.abs(Jr).max()
    ej = np.abs(J[0] - Jr).max() / scale
    ek = np.abs(K[0] - Kr).max() / scale
    E = _energy(P, Jr, Kr)
    dE = abs(_energy(P, J[0], K[0]) - E)
    print(f"all-FP32 max|dJ|/max|J| {ej:.2e} max|dK|/max|J| {ek:.2e} dE {dE:.2e} (E {E:.3f})", flush=True)
    # Forcing every batch to FP32 is a stress case: the FP32 Obara-Saika terms
    # PA [..] + WP [..]^(m+1) cancel for distant pairs (large |P-A|), so
    # exchange elements lose ~2 digits beyond FP32 rounding.  Such pairs have
    # small Schwarz factors, which is why routing sends only small-bound
    # batches to FP32 (checked to 1e-6 Eh in the mixed test below).
    assert 1e-12 < ej < 5e-6 and 1e-12 < ek < 5e-5
    assert dE < 1e-5 * abs(E), dE


def test_routed_mixed_threshold(torch_cuda):
    """12 atoms of 2s1p (exponents 0.3..30, localized): the smallest bound
    threshold that sends some batches to FP32 and keeps others in FP64; the
    energy stays within 1e-6 Eh of the oracle there and at 1e-5."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    w, ob, P = case_real(12, inputs.SHELLS_2S1P, seed=21, lo=0.3, hi=30.0)
    gb = cq.Basis.from_molecule(w.mol)
    J64, K64 = _jk_gpu(torch, gb, [P], [1])
    st64 = gb.build_stats()
    Jr, Kr = ob.jk(P)
    assert rel_err(J64[0], Jr) < TOL_JK and rel_err(K64[0], Kr) < TOL_JK
    E = _energy(P, Jr, Kr)
    split = None
    for thr in (1e-5, 1e-4, 1e-3, 1e-2, 3e-2, 1e-1):
        J, K = _jk_gpu(torch, gb, [P], [1], th=cq.thresholds(mode=1, fp32_below=thr))
        st = gb.build_stats()
        assert st["fp32"] + st["fp64"] == st64["fp64"]
        dE = abs(_energy(P, J[0], K[0]) - E)
        frac = st["fp32"] / (st["fp32"] + st["fp64"])
        print(f"fp32_below {thr:.0e}: fp32 fraction {frac:.3f} dE {dE:.2e} "
              f"max|dJ| {np.abs(J[0] - Jr).max():.2e} max|dK| {np.abs(K[0] - Kr).max():.2e}", flush=True)
        if thr == 1e-5:
            assert dE < 1e-6
        if st["fp32"] > 0 and st["fp64"] > 0:
            split = thr
            assert dE < 1e-6
            break
    assert split is not None
