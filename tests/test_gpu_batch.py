"""GPU parity of the batched uneven launch (one handle over many molecules,
each class in one launch spanning all of them) and of the autotuner: the
batch against the oracle per molecule, against one handle per molecule, and
unchanged by the tuned plan."""
import sys

import numpy as np
import pytest

import oracle
from paper_1905_01381_amd import inputs
from tests.gpu_common import rel_err

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


@pytest.fixture(scope="module")
def ragged(torch_cuda):
    """Four molecules of uneven size and shell content: one with s, p and d
    shells, one without d, one of s shells only, and a larger s/p/d one, so
    that some classes have no work in some molecules."""
    ws = [inputs.small(3, inputs.SHELLS_3S2P1D, seed=11),
          inputs.small(5, inputs.SHELLS_2S1P, seed=12),
          inputs.small(2, [0, 0], seed=13, nocc=1),
          inputs.small(4, inputs.SHELLS_3S2P1D, seed=14)]
    obs = [oracle.Basis.from_molecule(w.mol) for w in ws]
    Ps = [oracle.density_real(ob.overlap(), w.orbitals) for w, ob in zip(ws, obs)]
    rng = np.random.default_rng(21)
    As = [inputs.random_symmetric(ob.nbf, rng, -1) for ob in obs]
    return ws, obs, Ps, As


def _batch_jk(torch, gb, Ps, As, th=None):
    P = gb.pack([_dev(torch, p) for p in Ps])
    A = gb.pack([_dev(torch, a) for a in As])
    r = gb.jk([P, A], sym=[1, -1], want_j=[True, False], th=th)
    torch.cuda.synchronize()
    J = [x.cpu().numpy() for x in gb.unpack(r.J[0])]
    K0 = [x.cpu().numpy() for x in gb.unpack(r.K[0])]
    K1 = [x.cpu().numpy() for x in gb.unpack(r.K[1])]
    return J, K0, K1


def test_batch_against_oracle(ragged, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws, obs, Ps, As = ragged
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    assert gb.nmol == 4 and gb.mol_nbf == [ob.nbf for ob in obs]
    J, K0, K1 = _batch_jk(torch, gb, Ps, As)
    for i, ob in enumerate(obs):
        Jr, Kr = ob.jk(np.stack([Ps[i], As[i]]))
        assert rel_err(J[i], Jr[0]) < TOL_JK, i
        assert rel_err(K0[i], Kr[0]) < TOL_JK, i
        assert rel_err(K1[i], Kr[1]) < TOL_JK, i
    counts = gb.quartet_counts()
    per_mol = [cq.Basis.from_molecule(w.mol).quartet_counts() for w in ws]
    for cls, n in counts.items():
        assert n == sum(c.get(cls, 0) for c in per_mol), cls


def test_batch_equals_per_molecule_handles(ragged, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws, obs, Ps, As = ragged
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    J, K0, K1 = _batch_jk(torch, gb, Ps, As)
    for i, w in enumerate(ws):
        g1 = cq.Basis.from_molecule(w.mol)
        r = g1.jk([_dev(torch, Ps[i]), _dev(torch, As[i])], sym=[1, -1], want_j=[True, False])
        assert rel_err(J[i], r.J[0].cpu().numpy()) < 1e-13, i
        assert rel_err(K0[i], r.K[0].cpu().numpy()) < 1e-13, i
        assert rel_err(K1[i], r.K[1].cpu().numpy()) < 1e-13, i


def test_single_molecule_batch_equals_plain_handle(ragged, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws, obs, Ps, As = ragged
    w = ws[3]
    gb = cq.Basis.from_molecules([w.mol])
    g1 = cq.Basis.from_molecule(w.mol)
    P = _dev(torch, Ps[3])
    rb = gb.jk([P.reshape(-1).contiguous()])
    r1 = g1.jk([P])
    assert rel_err(rb.J[0].cpu().numpy().reshape(P.shape), r1.J[0].cpu().numpy()) < 1e-13
    assert rel_err(rb.K[0].cpu().numpy().reshape(P.shape), r1.K[0].cpu().numpy()) < 1e-13


def test_autotune_keeps_results(ragged, torch_cuda):
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws, obs, Ps, As = ragged
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    J0, K00, K10 = _batch_jk(torch, gb, Ps, As)
    before = gb.plan()
    plan = gb.autotune(nmat=2, reps=2)
    print("tuned plan:", plan, flush=True)
    assert [p["cls"] for p in plan] == [p["cls"] for p in before]
    for p in plan:
        assert p["cl"] >= 1 and p["grid"] in (0, 2048) and p["tasks"] > 0 and p["ms"] > 0
        assert p["acc"] in (-1, 0, 1, 2) and p["rot"] in (0, 1, 2, 3)
    J, K0, K1 = _batch_jk(torch, gb, Ps, As)
    for i in range(len(ws)):
        assert rel_err(J[i], J0[i]) < 1e-13
        assert rel_err(K0[i], K00[i]) < 1e-13
        assert rel_err(K1[i], K10[i]) < 1e-13
    # the same plan set on a fresh handle forms the same partial sums: bitwise equal
    g2 = cq.Basis.from_molecules([w.mol for w in ws])
    g2.set_plan(plan)
    assert [(p["cls"], p["cl"], p["grid"], p["exchanged"], p["acc"], p["rot"]) for p in g2.plan()] == \
        [(p["cls"], p["cl"], p["grid"], p["exchanged"], p["acc"], p["rot"]) for p in plan]
    J2, K02, K12 = _batch_jk(torch, g2, Ps, As)
    for i in range(len(ws)):
        assert np.array_equal(J2[i], J[i]) and np.array_equal(K02[i], K0[i]) and np.array_equal(K12[i], K1[i]), i
    with pytest.raises(cq.CqError):
        g2.set_plan([dict(plan[0], cl=65)])


def test_batch_routed_modes(ragged, torch_cuda):
    """Routed mode on a batch: a zero FP32 bound routes every wave step to
    FP64 (same result as FP64 mode); an infinite one routes all of them to
    FP32 (the error bounds of the FP32 path)."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    ws, obs, Ps, As = ragged
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    J64, K64, _ = _batch_jk(torch, gb, Ps, As)
    st64 = gb.build_stats()
    J, K, _ = _batch_jk(torch, gb, Ps, As, th=cq.thresholds(mode=1, fp32_below=0.0))
    st = gb.build_stats()
    assert st["fp32"] == 0 and st["fp64"] == st64["fp64"]
    for i in range(len(ws)):
        assert rel_err(J[i], J64[i]) < 1e-13 and rel_err(K[i], K64[i]) < 1e-13
    J, K, _ = _batch_jk(torch, gb, Ps, As, th=cq.thresholds(mode=1, fp32_below=1e300))
    st = gb.build_stats()
    assert st["fp64"] == 0 and st["fp32"] == st64["fp64"]
    # every quartet in FP32 (a stress case the router never picks for large
    # bounds): with d shells and exponents up to 1e3 the recurrences carry
    # intermediates far larger than the result, so the error reaches several
    # hundred FP32 unit roundoffs (u = 6e-8) of the largest element (s/p-only
    # molecules stay near 1 u); the accuracy that matters, |dE| <= 1e-6 Eh
    # under the router's own thresholds, is tested with the routed builds
    for i in range(len(ws)):
        ej, ek = rel_err(J[i], J64[i]), rel_err(K[i], K64[i])
        print(f"molecule {i}: all-FP32 rel err J {ej:.2e} K {ek:.2e}", flush=True)
        assert 0 < ej < 2e-5 and 0 < ek < 1e-4, i


def test_c4_smallest_molecules_sampled_blocks(torch_cuda):
    """The eight smallest molecules of the batched workload (64 molecules of
    U{10..120} atoms, 3s2p1d) at their real sizes in one batch handle, tuned;
    sampled J and K shell blocks of every molecule against the oracle."""
    torch = torch_cuda
    from paper_1905_01381_amd import cq
    sizes = inputs.c4_sizes()
    pick = [int(i) for i in np.argsort(sizes, kind="stable")[:8]]
    ws = [inputs.c4_molecule(i) for i in pick]
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    obs = [oracle.Basis.from_molecule(w.mol) for w in ws]
    Ps = [oracle.density_real(ob.overlap(), w.orbitals) for w, ob in zip(ws, obs)]
    gb.autotune(nmat=1, reps=1)
    P = gb.pack([_dev(torch, p) for p in Ps])
    r = gb.jk([P])
    J = [x.cpu().numpy() for x in gb.unpack(r.J[0])]
    K = [x.cpu().numpy() for x in gb.unpack(r.K[0])]
    for i, (w, ob) in enumerate(zip(ws, obs)):
        ls = w.mol.shell_l
        o = ob.offsets
        d_sh = int(np.where(ls == 2)[0][i % 3])
        p_sh = int(np.where(ls == 1)[0][-1 - i % 2])
        s_sh = int(np.where(ls == 0)[0][(5 * i) % len(np.where(ls == 0)[0])])
        for a, b in [(d_sh, p_sh), (s_sh, d_sh)]:
            jb = ob.j_block(a, b, Ps[i][None])[0]
            kb = ob.k_block(a, b, Ps[i][None])[0]
            assert rel_err(J[i][o[a]:o[a + 1], o[b]:o[b + 1]], jb) < TOL_JK, (i, a, b)
            assert rel_err(K[i][o[a]:o[a + 1], o[b]:o[b + 1]], kb) < TOL_JK, (i, a, b)
