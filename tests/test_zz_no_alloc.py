"""cq_jk_build_noalloc (static scratch, no device allocation) against
cq_jk_build through the C-ABI: two calls in a row, the second on a smaller
input, each bitwise equal to the allocating entry point (both accumulate
deterministically) and within 1e-10 of the oracle; an oversized build is
refused before any work."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1905_01381_amd import inputs
from tests.gpu_common import case_real, rel_err

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(torch, gb, mats, sym, want_j):
    out = []
    for noalloc in (False, True):
        r = gb.jk([_dev(torch, m) for m in mats], sym=sym, want_j=want_j, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append(([j.cpu().numpy() if j is not None else None for j in r.J],
                    [k.cpu().numpy() for k in r.K]))
    return out


def test_noalloc_matches_allocating_build_twice():
    import torch
    from paper_1905_01381_amd import cq
    print("\n[gpu-case] noalloc: 5-atom 3s2p1d, 3 densities; then 2-atom 2s1p, 1 density", flush=True)
    sys.stdout.flush()
    w, ob, P = case_real(5, inputs.SHELLS_3S2P1D, seed=8, nocc=10)
    gb = cq.Basis.from_molecule(w.mol)
    rng = np.random.default_rng(4)
    A = inputs.random_symmetric(gb.nbf, rng, -1)
    S2 = inputs.random_symmetric(gb.nbf, rng, 1)
    (Ja, Ka), (Jn, Kn) = _both(torch, gb, [P, A, S2], [1, -1, 1], [True, False, True])
    Jr, Kr = ob.jk(np.stack([P, A, S2]))
    for m in range(3):
        assert np.array_equal(Kn[m], Ka[m]), m
        assert rel_err(Kn[m], Kr[m]) < 1e-10, m
        if m != 1:
            assert np.array_equal(Jn[m], Ja[m]), m
            assert rel_err(Jn[m], Jr[m]) < 1e-10, m
    # second call: a smaller basis and one density (the scratch keeps the
    # first call's contents; the build must clear what it uses)
    w2, ob2, P2 = case_real(2, inputs.SHELLS_2S1P, seed=3, lo=0.15, hi=30.0)
    g2 = cq.Basis.from_molecule(w2.mol)
    (Ja, Ka), (Jn, Kn) = _both(torch, g2, [P2], [1], [True])
    J2, K2 = ob2.jk(P2)
    assert np.array_equal(Jn[0], Ja[0]) and np.array_equal(Kn[0], Ka[0])
    assert rel_err(Jn[0], J2) < 1e-10 and rel_err(Kn[0], K2) < 1e-10
    # and the first basis again, after the smaller call
    (Ja3, Ka3), (Jn3, Kn3) = _both(torch, gb, [P], [1], [True])
    assert np.array_equal(Jn3[0], Ja3[0]) and np.array_equal(Kn3[0], Ka3[0])


def test_noalloc_refuses_oversized_build():
    """Densities and partial sums beyond the 512 MiB scratch: CQ_ENOMEM
    before any work, and the handle still builds through the allocating
    entry point afterwards."""
    import torch
    from paper_1905_01381_amd import cq
    print("\n[gpu-case] noalloc: oversized build refused", flush=True)
    w = inputs.small(120, inputs.SHELLS_2S1P, seed=1, lo=0.15, hi=30.0, nocc=4)
    gb = cq.Basis.from_molecule(w.mol)   # nbf 600
    n = gb.nbf
    mats = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(16)]
    for m in mats:
        m.fill_diagonal_(1e-3)
    # 16 densities with J and K: nel * 8 * (16 + 2 * 32) = 230 MB < 512 MiB -> runs
    gb.jk(mats, noalloc=True)
    torch.cuda.synchronize()
    wb = inputs.small(300, inputs.SHELLS_2S1P, seed=1, lo=0.15, hi=30.0, nocc=4)
    big = cq.Basis.from_molecule(wb.mol)  # nbf 1500: nel * 8 * (16 + 64) = 1.44 GB
    nb = big.nbf
    bm = [torch.zeros((nb, nb), dtype=torch.float64, device="cuda") for _ in range(16)]
    with pytest.raises(cq.CqError) as ei:
        big.jk(bm, noalloc=True)
    assert ei.value.status == cq.CQ_ENOMEM
    assert "scratch" in str(ei.value)
    r = gb.jk(mats[:1])
    torch.cuda.synchronize()
    assert torch.isfinite(r.J[0]).all()
