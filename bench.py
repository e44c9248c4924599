"""Benchmark: two-component integral-direct Fock build on one MI355X.

Workload (the two-component generalized J/K configuration): 40 atoms on a
jittered cubic lattice, 3s2p1d Cartesian shells with 3 primitives each
(exponents geometric 0.1..1e3), nbf = 600; a complex Hermitian 1200 x 1200
spin-blocked density from 60 random S-orthonormal spinors.  One step = one
cq_fock2e_2c call: Pauli split (Eq. pauli_sep), one integral pass forming
J[Re P^0] and K of the eight real Pauli parts, and the merge into G^{2C}
(Eq. 2c_fock), FP64, no screening.  Inputs are resident in HBM before the
timed region.

Output: one JSON line (metric, value = builds/s, quartets/s, roofline of the
dominant electron-repulsion kernel measured with HIP events inside the timed
region, and the CPU oracle timed on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64 (datasheet)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="approximate CPU sample budget")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args()


def build_inputs(torch, cq, inputs):
    w = inputs.c2()
    gb = cq.Basis.from_molecule(w.mol)
    n = gb.nbf
    S = gb.one_electron("overlap").cpu().numpy()
    lam, U = np.linalg.eigh(S)
    X = (U / np.sqrt(lam)) @ U.T
    Q = w.orbitals
    C = np.empty_like(Q)
    C[:n] = X @ Q[:n]
    C[n:] = X @ Q[n:]
    P2 = C @ C.conj().T
    return w, gb, torch.from_numpy(np.ascontiguousarray(P2)).cuda()


def cpu_baseline(w, budget_s: float):
    """Oracle (plain FP64 C, OpenMP) on a bounded sample of the same
    workload: sampled exchange blocks K_(a,c) of the eight Pauli parts and
    one Coulomb block, each summing every ordered shell quartet (a b|c d)
    over all b, d.  The full build is extrapolated from the time per
    evaluated quartet times the unique quartets of one build."""
    import oracle
    from oracle import twocomp
    ob = oracle.Basis.from_molecule(w.mol)
    S = ob.overlap()
    P2 = oracle.density_2c(S, w.orbitals)
    stack, _ = twocomp.real_parts(twocomp.split(P2))
    ls = w.mol.shell_l
    ns = ob.nshell
    picks = [(int(np.where(ls == 2)[0][3]), int(np.where(ls == 1)[0][11])),
             (int(np.where(ls == 2)[0][30]), int(np.where(ls == 2)[0][12])),
             (int(np.where(ls == 1)[0][70]), int(np.where(ls == 2)[0][5])),
             (int(np.where(ls == 2)[0][17]), int(np.where(ls == 0)[0][60])),
             (int(np.where(ls == 1)[0][40]), int(np.where(ls == 0)[0][7])),
             (int(np.where(ls == 0)[0][90]), int(np.where(ls == 2)[0][20])),
             (int(np.where(ls == 0)[0][3]), int(np.where(ls == 0)[0][5]))]
    t0 = time.time()
    nq = 0
    done = 0
    ob.j_block(picks[0][0], picks[0][1], stack[:1])
    nq += ns * ns
    for a, c in picks:
        ob.k_block(a, c, stack)
        nq += ns * ns
        done += 1
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    per_q = dt / nq
    return per_q, nq, dt, done, oracle.num_threads()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU design is described in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_01381_amd import cq, flops, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w, gb, P2 = build_inputs(torch, cq, inputs)
    G = torch.empty_like(P2)
    counts = gb.quartet_counts()
    nq = sum(counts.values())
    print(f"[bench] nbf={gb.nbf} nshell={gb.nshell} unique shell quartets/build={nq:.4e}", file=sys.stderr, flush=True)
    for i in range(a.warmup):
        gb.fock2e_2c(P2, out=G)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{a.warmup} done", file=sys.stderr, flush=True)
    gb.profile(True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        gb.fock2e_2c(P2, out=G)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gb.profile(False)
    prof = gb.profile_read()
    print(f"[bench] {a.steps} timed steps done", file=sys.stderr, flush=True)
    if a.calib_copy_mib > 0:
        nel = a.calib_copy_mib * (1 << 20) // 8
        x = torch.ones(nel, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    dt = t1 - t0
    builds_s = a.steps / dt
    # dominant kernel: largest summed time over the timed region
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    cls, (ms_tot, launches) = dom
    avg_s = ms_tot / launches / 1e3
    fq = flops.per_quartet(*cls, nJ=1, nK=8)
    achieved = fq * counts[cls] / avg_s / 1e12
    traffic = None
    try:
        with open(a.traffic_json) as f:
            tj = json.load(f)
        key = "eri_jk_" + "".join("spd"[x] for x in cls)
        if tj.get("kernel") == key and tj.get("workload") == "c2":
            traffic = tj.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    rec = {
        "metric": "J+K builds/sec & quartets/s at |dE|<=1e-6 Eh vs FP64 oracle; mixed/learned vs plain",
        "value": builds_s,
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "two-component generalized J/K: 40 atoms, 3s2p1d Cartesian (3 primitives), nbf 600, "
                        "60 complex spinors; J[Re P0] + K of 8 real Pauli parts per build; FP64, no screening",
            "nbf": gb.nbf,
            "quartets_per_build": nq,
            "mode": "fp64",
        },
        "quartets_per_s": nq * builds_s,
        "roofline": {
            "bound": "alu",
            "kernel": "eri_jk_" + "".join("spd"[x] for x in cls),
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_per_quartet": fq,
            "quartets_per_launch": counts[cls],
            "avg_launch_ms": avg_s * 1e3,
        },
        "per_class_ms": {"".join("spd"[x] for x in k): v[0] / v[1] for k, v in sorted(prof.items())},
    }
    if not a.no_cpu_baseline:
        per_q, nqs, dts, done, thr = cpu_baseline(w, a.cpu_seconds)
        rec["cpu_baseline"] = {
            "value": 1.0 / (per_q * nq),
            "unit": "builds/s",
            "cores": thr,
            "kind": "oracle",
            "sample": f"oracle J block + {done} K blocks (8 Pauli parts) of this workload: {nqs} ordered shell "
                      f"quartets in {dts:.1f} s; one build extrapolated as {nq} unique quartets at that rate",
            "quartets_per_s": 1.0 / per_q,
        }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
