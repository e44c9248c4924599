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

Other workloads (one JSON line each, same top-level keys; not the headline):
  --workload c3   mixed-precision routed build vs FP64 on the 3s2p1d lattice
                  recipe (skip 1e-11, FP32 below 1e-5): builds/s of both
                  modes, |dE|, max|dJ|, max|dK|, FP64/FP32/skip counts;
                  --atoms scales the molecule (200 = the full workload)
  --workload c4   batched uneven build: one handle over the --nmol smallest
                  molecules of the 64-molecule set, one launch per class
                  spanning all of them, default vs autotuned plan, against one
                  handle per molecule built in turn
  --workload c5   real-time Magnus-2 steps (EM2) on the 60-atom Z=1 workload:
                  time per step and per Fock build after an RHF ground state
                  and a delta kick; --atoms scales the molecule
  --workload c5l  the learned-midpoint protocol on the same recipe (default
                  12 atoms): plain self-consistent midpoint, learned proposal
                  (records the first --rt-train steps, trains the network on
                  the GPU, then proposes midpoints) and its ablation (network
                  zeroed), all at one first-iterate acceptance tolerance
                  (--accept-tol); EM2 and MMUT beside them.  Reports
                  builds/step, dipole error against a tightly converged
                  midpoint trajectory and energy drift
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
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "c5l", "f"])
    ap.add_argument("--no-tune", action="store_true", help="c4: skip the autotuner (default plan only)")
    ap.add_argument("--kick", type=float, default=1e-4, help="c5/c5l: delta-kick strength along z (a.u.)")
    ap.add_argument("--dt", type=float, default=0.05, help="c5l: time step (a.u.)")
    ap.add_argument("--rt-chunk", type=int, default=50,
                    help="c5l: steps per progress line (each line adds one uncounted energy build)")
    ap.add_argument("--serialize", action="store_true",
                    help="c2: run every build with per-class timing on (classes one after another), e.g. under a "
                         "kernel-trace profiler so that each kernel's duration is its own")
    ap.add_argument("--atoms", type=int, default=0, help="c3/c5/f: atoms (0 = the full workload; f: 6)")
    ap.add_argument("--nmol", type=int, default=16, help="c4: number of molecules (smallest first)")
    ap.add_argument("--c4-variants", default="batched,single",
                    help="c4: comma list of batched (one handle) and single (one handle per molecule)")
    ap.add_argument("--rt-steps", type=int, default=2000, help="c5l: trajectory length")
    ap.add_argument("--rt-train", type=int, default=500, help="c5l: steps recorded for training")
    ap.add_argument("--epochs", type=int, default=200, help="c5l: training epochs")
    ap.add_argument("--accept-tol", type=float, default=1e-8,
                    help="c5l: first-iterate acceptance tolerance shared by plain, learned and ablation")
    ap.add_argument("--mmut-restart", type=int, default=50, help="c5l: MMUT EM2 restart period")
    ap.add_argument("--rt-variants", default="reference,plain,learned,ablation,em2,mmut",
                    help="c5l: runs to make (plain always; without reference, dipole errors are against plain)")
    return ap.parse_args()


def kernel_source_hash(cls: str) -> str:
    """sha256 of a class's generated kernel source, the common header it
    includes and the host code that builds its inputs (pair records,
    primitive cut, task lists): what a counter profile of that kernel was
    taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_01381_amd", "csrc")
    for p in (os.path.join(csrc, "gen", f"eri_{cls}.hip"), os.path.join(csrc, "eri_common.hpp"),
              os.path.join(csrc, "cq_api.hip")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _clean(x):
    """NaN (a variant that was not run) -> None, so that the line stays JSON."""
    if isinstance(x, float) and x != x:
        return None
    if isinstance(x, dict):
        return {k: _clean(v) for k, v in x.items()}
    if isinstance(x, list):
        return [_clean(v) for v in x]
    return x


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _ortho_density(S, Q):
    lam, U = np.linalg.eigh(S)
    X = (U / np.sqrt(lam)) @ U.T
    C = X @ Q
    return C @ C.T


def bench_c3(a, torch, cq, inputs):
    """Routed vs FP64 build on the 3s2p1d lattice recipe (full size: 200
    atoms, 400 occupied orbitals)."""
    natom = a.atoms or 200
    w = inputs.c3(natom=natom, nocc=2 * natom)
    gb = cq.Basis.from_molecule(w.mol)
    gb.trace(True)  # a progress line per class (builds of minutes)
    S = gb.one_electron("overlap").cpu().numpy()
    P = torch.from_numpy(np.ascontiguousarray(_ortho_density(S, w.orbitals))).cuda()
    counts = sum(gb.quartet_counts().values())
    _log(f"c3: {natom} atoms, nbf {gb.nbf}, {counts:.3e} unique quartets unscreened")
    th64 = cq.thresholds(skip=1e-11)
    thr = cq.thresholds(skip=1e-11, mode=1, fp32_below=1e-5)
    out = {}
    for name, th in (("fp64", th64), ("routed", thr)):
        res = {}

        def run():
            res["r"] = gb.jk([P], th=th)
        dt = _timed(torch, run, a.steps, a.warmup)
        st = gb.build_stats()
        J, K = res["r"].J[0], res["r"].K[0]
        E = 2.0 * float((P * J).sum()) - float((P * K).sum())
        out[name] = {"s_per_build": dt, "stats": st, "E2": E, "J": J, "K": K}
        _log(f"c3 {name}: {dt:.3f} s/build, {st}")
    dJ = float((out["routed"]["J"] - out["fp64"]["J"]).abs().max())
    dK = float((out["routed"]["K"] - out["fp64"]["K"]).abs().max())
    st = out["routed"]["stats"]
    ev = st["fp64"] + st["fp32"]
    return {
        "metric": "J+K builds/sec at |dE|<=1e-6 Eh: precision-routed vs FP64 (skip 1e-11, FP32 below 1e-5)",
        "value": 1.0 / out["routed"]["s_per_build"], "unit": "builds/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": out["routed"]["s_per_build"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"mixed-precision routed J/K: {natom} atoms 3s2p1d (3 primitives), nbf {gb.nbf}, "
                               f"{2 * natom} occupied orbitals; skip 1e-11, FP32 below 1e-5", "nbf": gb.nbf,
                   "quartets_unscreened": counts},
        "fp64_builds_per_s": 1.0 / out["fp64"]["s_per_build"],
        "speedup_routed_vs_fp64": out["fp64"]["s_per_build"] / out["routed"]["s_per_build"],
        "dE_Eh": abs(out["routed"]["E2"] - out["fp64"]["E2"]), "E2_fp64": out["fp64"]["E2"],
        "max_abs_dJ": dJ, "max_abs_dK": dK,
        "fp32_fraction": st["fp32"] / ev if ev else 0.0,
        "counts_routed": st, "counts_fp64": out["fp64"]["stats"],
        "quartets_per_s_routed": ev / out["routed"]["s_per_build"],
    }


def bench_c4(a, torch, cq, inputs):
    """Batched uneven build over the smallest molecules of the 64-molecule set."""
    sizes = inputs.c4_sizes()
    pick = [int(i) for i in np.argsort(sizes, kind="stable")[:a.nmol]]
    ws = [inputs.c4_molecule(i) for i in pick]
    gb = cq.Basis.from_molecules([w.mol for w in ws])
    Ps = []
    for w in ws:
        g1 = cq.Basis.from_molecule(w.mol)
        S = g1.one_electron("overlap").cpu().numpy()
        Ps.append(torch.from_numpy(np.ascontiguousarray(_ortho_density(S, w.orbitals))).cuda())
        g1.close()
    P = gb.pack(Ps)
    counts = sum(gb.quartet_counts().values())
    _log(f"c4: {len(ws)} molecules ({min(sizes[pick])}..{max(sizes[pick])} atoms), nbf {gb.mol_nbf[0]}.."
         f"{gb.mol_nbf[-1]}, {counts:.3e} quartets")
    variants = a.c4_variants.split(",")
    long_run = counts > 1e11  # builds of minutes: a progress line per class
    gb.trace(long_run)
    t_default = _timed(torch, lambda: gb.jk([P]), a.steps, a.warmup) if "batched" in variants else float("nan")
    _log(f"c4 batched default plan: {t_default:.3f} s/build")
    if a.no_tune or "batched" not in variants:
        # cq_autotune times every candidate on the whole batch: about 30
        # launches per class, too long for batches of minutes per build
        plan, t_tune, t_tuned = gb.plan(), 0.0, t_default
    else:
        t0 = time.perf_counter()
        plan = gb.autotune(nmat=1, reps=1)
        t_tune = time.perf_counter() - t0
        t_tuned = _timed(torch, lambda: gb.jk([P]), a.steps, a.warmup)
        _log(f"c4 batched tuned plan: {t_tuned:.3f} s/build (autotune {t_tune:.1f} s)")
    t_single = float("nan")
    if "single" in variants:
        singles = [cq.Basis.from_molecule(w.mol) for w in ws]
        for g1 in singles:
            g1.trace(long_run)

        def per_mol():
            for g1, p in zip(singles, Ps):
                g1.jk([p])
        t_single = _timed(torch, per_mol, a.steps, a.warmup)
        _log(f"c4 one handle per molecule: {t_single:.3f} s/build")
    if "batched" not in variants:
        t_tuned = t_single
    return {
        "metric": ("J+K builds/sec, batched uneven launch (all molecules per class launch, "
                   + ("default plan)" if a.no_tune else "autotuned)")) if "batched" in variants
                  else "J+K builds/sec, one handle per molecule",
        "value": 1.0 / t_tuned, "unit": "builds/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t_tuned * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched uneven J/K: the {len(ws)} smallest of 64 molecules of U{{10..120}} atoms, "
                               f"3s2p1d; one J and one K each; FP64, no screening", "nmol": len(ws),
                   "atoms": [int(sizes[i]) for i in pick], "quartets_per_build": counts},
        "quartets_per_s": counts / t_tuned,
        "batched_default_builds_per_s": 1.0 / t_default,
        "per_molecule_builds_per_s": 1.0 / t_single,
        "speedup_batched_tuned_vs_per_molecule": t_single / t_tuned,
        "speedup_tuned_vs_default": t_default / t_tuned,
        "autotune_s": t_tune,
        "tuned": not a.no_tune,
        "plan": [{"cls": "".join("spd"[x] for x in p["cls"]), "cl": p["cl"], "grid": p["grid"], "exchanged": p["exchanged"],
                  "acc": p["acc"], "rot": p["rot"],
                  "ms": round(p["ms"], 3)} for p in plan],
    }


def _c5_state(a, torch, cq, inputs, natom):
    from paper_1905_01381_amd import scf
    w = inputs.c5(natom=natom)
    gb = cq.Basis.from_molecule(w.mol)
    if natom >= 40:
        gb.trace(True)  # a progress line per class (builds of seconds)
    t0 = time.perf_counter()
    res = scf.rhf(gb, w.mol, natom // 2)
    _log(f"{natom} atoms, nbf {gb.nbf}; RHF E = {res.energy:.8f} in {res.iterations} iterations "
         f"({time.perf_counter() - t0:.1f} s)")
    Dz = gb.one_electron("dipole", direction=2).cpu().numpy()
    X = res.X
    Sh = res.S @ X
    Po = Sh @ res.P @ Sh
    lam, U = np.linalg.eigh(X @ Dz @ X)
    Uk = (U * np.exp(-1j * a.kick * lam)) @ U.T
    P0 = Uk @ Po @ Uk.conj().T
    d = lambda m: torch.from_numpy(np.ascontiguousarray(m)).cuda()
    return gb, res, (d(res.h), d(X), d(Dz), d(P0))


def _rt_steps(r, n, label, chunk=50):
    """r.step(n) in chunks; the energy (one extra, uncounted Fock build) is
    taken at the last step of each chunk only; one progress line per chunk.
    Returns (steps with an energy, energies, dipoles, builds per step)."""
    Es, Ei, mus, nbs = [], [], [], []
    done = 0
    while done < n:
        k = min(chunk, n - done)
        if k > 1:
            _, mu, nb = r.step(k - 1, energy=False)
            mus.append(mu)
            nbs.append(nb)
        E, mu, nb = r.step(1, energy=True)
        mus.append(mu)
        nbs.append(nb)
        done += k
        Es.append(float(E[0]))
        Ei.append(done - 1)
        _log(f"{label}: {done}/{n} steps, {np.concatenate(nbs).mean():.3f} builds/step")
    return np.array(Ei), np.array(Es), np.concatenate(mus), np.concatenate(nbs)


def bench_c5l(a, torch, cq, inputs):
    """Builds per step of the learned midpoint proposal against the plain
    self-consistent midpoint corrector and its own ablation (network zeroed:
    the propagator-reuse baseline alone), all accepting the first midpoint
    iterate at the same tolerance; EM2 (2 builds/step) and MMUT (1 build per
    step plus EM2 restarts) beside them.  Dipole errors are measured against
    a reference midpoint trajectory converged to 1e-12."""
    natom = a.atoms or 12
    gb, res, args = _c5_state(a, torch, cq, inputs, natom)
    dt, nt, nall, acc = a.dt, a.rt_train, a.rt_steps, a.accept_tol
    runs = {}

    def plain(mode, label, sc_tol=1e-10, accept=acc, restart=None):
        r = cq.RT(gb, *args, dt, mode)
        r.set_params(sc_tol=sc_tol, max_iter=60, accept_tol=accept)
        if restart:
            r.set_restart(restart)
        t0 = time.perf_counter()
        ei, E, mu, nb = _rt_steps(r, nall, label, a.rt_chunk)
        torch.cuda.synchronize()
        runs[label] = {"E_idx": ei, "E": E, "mu": mu, "nb": nb, "s": time.perf_counter() - t0, "stats": r.stats()}
        r.close()

    def learned(zero, label):
        r = cq.RT(gb, *args, dt, cq.RT_MIDPOINT)
        r.set_params(sc_tol=1e-10, max_iter=60, accept_tol=acc)
        r.record(True, 4096, 1)
        t0 = time.perf_counter()
        e1, E1, mu1, nb1 = _rt_steps(r, nt, label + " (recording)", a.rt_chunk)
        r.record(False)
        t1 = time.perf_counter()
        loss = r.train(epochs=0 if zero else a.epochs, lr=3e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        if zero:
            r.weights(np.zeros(354, np.float32))
        r.set_mode(cq.RT_LEARNED)
        t2 = time.perf_counter()
        e2, E2, mu2, nb2 = _rt_steps(r, nall - nt, label, a.rt_chunk)
        torch.cuda.synchronize()
        runs[label] = {"E_idx": np.concatenate([e1, e2 + nt]), "E": np.concatenate([E1, E2]),
                       "mu": np.concatenate([mu1, mu2]), "nb": np.concatenate([nb1, nb2]),
                       "s": time.perf_counter() - t2, "s_record": t1 - t0, "s_train": t_train, "loss": loss,
                       "stats": r.stats()}
        r.close()

    want = a.rt_variants.split(",")
    for v in want:
        if v not in ("reference", "plain", "learned", "ablation", "em2", "mmut"):
            raise SystemExit(f"unknown --rt-variants entry {v!r}")
    if "reference" in want:
        plain(cq.RT_MIDPOINT, "reference", sc_tol=1e-12, accept=1e-12)
    plain(cq.RT_MIDPOINT, "plain")
    if "learned" in want:
        learned(False, "learned")
    if "ablation" in want:
        learned(True, "ablation")
    if "em2" in want:
        plain(cq.RT_EM2, "em2")
    if "mmut" in want:
        plain(cq.RT_MMUT, "mmut", restart=a.mmut_restart)
    # dipole errors against the converged reference, else against the plain
    # corrector (converged to sc_tol = 1e-10 whenever its first iterate is refused)
    ref_name = "reference" if "reference" in runs else "plain"
    mu_ref = runs[ref_name]["mu"]
    out = {}
    for k, r in runs.items():
        after = r["nb"][nt:]
        out[k] = {"builds_per_step": float(after.mean()),
                  "max_dipole_err_vs_reference": float(np.abs(r["mu"] - mu_ref).max()),
                  "energy_drift": float(np.abs(r["E"] - r["E"][0]).max()),
                  "s_per_step": r["s"] / (nall - nt if k in ("learned", "ablation") else nall),
                  "stats": r["stats"]}
    for k in ("learned", "ablation"):
        if k in runs:
            out[k]["train_loss"] = runs[k]["loss"]
            out[k]["train_s"] = runs[k]["s_train"]
    return {
        "metric": "RT-TDSCF J/K builds per step: learned midpoint proposal vs plain midpoint corrector at equal "
                  "acceptance tolerance",
        "value": out["learned"]["builds_per_step"] if "learned" in out else None, "unit": "builds/step", "n_gpus": 1, "steps": nall - nt,
        "warmup": nt, "ms_per_step": out["learned"]["s_per_step"] * 1e3 if "learned" in out else None,
        "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (MLP f32)", "data": "synthetic",
        "config": {"workload": f"RT-TDSCF learned midpoint: {natom} atoms Z=1, 3s2p1d, nbf {gb.nbf}, "
                               f"{natom // 2} doubly occupied; kick {a.kick:g} along z; dt {dt:g}; {nall} steps, network "
                               f"trained on the first {nt}; first-iterate acceptance {acc:g} for plain, learned "
                               f"and ablation; MMUT restart every {a.mmut_restart} steps", "nbf": gb.nbf,
                   "dipole_reference": ref_name},
        "runs": out,
    }


def bench_f(a, torch, cq, inputs):
    """Shells up to f: one J and one K per build of a real density on atoms
    of the 4s3p2d1f recipe (exponents 0.1..1e3).  Reports builds/s and,
    from a pass with per-class timing, the time of the classes with an f
    shell (workgroup-per-quartet kernel) against the generated classes."""
    natom = a.atoms or 6
    w = inputs.small(natom, inputs.SHELLS_4S3P2D1F, seed=1, lo=0.1, hi=1.0e3)
    gb = cq.Basis.from_molecule(w.mol)
    S = gb.one_electron("overlap").cpu().numpy()
    P = torch.from_numpy(np.ascontiguousarray(_ortho_density(S, w.orbitals))).cuda()
    qc = gb.quartet_counts()
    nq = sum(qc.values())
    nq_f = sum(v for k, v in qc.items() if 3 in k)
    _log(f"f: {natom} atoms, nbf {gb.nbf}, {nq:.4e} unique quartets, {nq_f:.4e} with an f shell")
    sec = _timed(torch, lambda: gb.jk([P]), a.steps, a.warmup)
    gb.profile(True, reset=True)
    gb.jk([P])
    torch.cuda.synchronize()
    prof = gb.profile_read()
    gb.profile(False)
    t_f = sum(v[0] for k, v in prof.items() if 3 in k)
    t_all = sum(v[0] for v in prof.values())
    top = sorted(((k, v[0]) for k, v in prof.items() if 3 in k), key=lambda kv: -kv[1])[:5]
    return {"metric": "J+K builds/sec, shells up to f", "value": 1.0 / sec, "unit": "builds/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"shells up to f: {natom} atoms 4s3p2d1f (3 primitives), nbf {gb.nbf}, "
                                   "one real density", "nbf": gb.nbf, "quartets": nq, "quartets_f": nq_f},
            "serialized_ms": {"f_classes": t_f, "other_classes": t_all - t_f},
            "f_quartets_per_s": nq_f / (t_f / 1e3), "other_quartets_per_s": (nq - nq_f) / ((t_all - t_f) / 1e3),
            "slowest_f_classes_ms": {"".join("spdf"[x] for x in k): ms for k, ms in top}}


def bench_c5(a, torch, cq, inputs):
    """EM2 real-time steps on the Z=1 lattice workload after an RHF ground
    state and a delta kick along z."""
    natom = a.atoms or 60
    gb, res, args = _c5_state(a, torch, cq, inputs, natom)
    rt = cq.RT(gb, *args, 0.05, cq.RT_EM2)
    if a.warmup > 0:
        rt.step(a.warmup, dipole=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, mu, nb = rt.step(a.steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    counts = sum(gb.quartet_counts().values())
    builds = float(np.mean(nb))
    return {
        "metric": "RT-TDSCF Magnus-2 steps/sec (EM2: two J/K builds per step)",
        "value": 1.0 / dt, "unit": "steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"RT-TDSCF: {natom} atoms Z=1, 3s2p1d, nbf {gb.nbf}, {natom // 2} doubly occupied; "
                               f"kick {a.kick:g} a.u. along z, dt 0.05 a.u.; EM2", "nbf": gb.nbf,
                   "quartets_per_build": counts},
        "builds_per_step": builds, "s_per_build": dt / builds,
        "quartets_per_s": counts * builds / dt, "scf_energy": res.energy, "dipole_last": float(mu[-1]),
    }


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
    # seeded (a, c) shell pairs, every pair of angular momenta in turn; the
    # loop below stops at the time budget
    rng = np.random.default_rng(11)
    by_l = [np.where(ls == l)[0] for l in range(3)]
    picks = []
    for k in range(90):
        la, lc = (k // 3) % 3, k % 3
        picks.append((int(rng.choice(by_l[la])), int(rng.choice(by_l[lc]))))
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
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): the build shards by class tasks with one "
              f"all-reduce of the J'/K' partial sums, which is not implemented here", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_01381_amd import cq, flops, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.workload != "c2":
        fn = {"c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "c5l": bench_c5l, "f": bench_f}[a.workload]
        print(json.dumps(_clean(fn(a, torch, cq, inputs))), flush=True)
        return
    w, gb, P2 = build_inputs(torch, cq, inputs)
    G = torch.empty_like(P2)
    th = cq.thresholds()
    counts = gb.quartet_counts()
    nq = sum(counts.values())
    print(f"[bench] nbf={gb.nbf} nshell={gb.nshell} unique shell quartets/build={nq:.4e}", file=sys.stderr, flush=True)
    if a.serialize:
        gb.profile(True, reset=True)
    for i in range(a.warmup):
        gb.fock2e_2c(P2, th=th, out=G)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{a.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        gb.fock2e_2c(P2, th=th, out=G)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] {a.steps} timed steps done", file=sys.stderr, flush=True)
    # roofline: the same steps again with per-class HIP events, which run the
    # classes one after another so that each event pair times one kernel
    gb.profile(True, reset=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(a.steps):
        gb.fock2e_2c(P2, th=th, out=G)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    gb.profile(False)
    prof = gb.profile_read()
    print(f"[bench] {a.steps} per-class timed steps done", file=sys.stderr, flush=True)
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
    # algorithmic work: per primitive quartet above the primitive cut, plus
    # per shell quartet (transfers, digestion)
    f_prim, f_fixed = flops.parts(*cls, nJ=1, nK=8)
    nprimq = gb.prim_quartet_counts()[cls]
    work = f_prim * nprimq + f_fixed * counts[cls]
    fq = work / counts[cls]
    achieved = work / avg_s / 1e12
    # HBM bytes per launch of the dominant kernel from the committed counter
    # profile, only while the kernel's source is the one that was profiled
    traffic = None
    try:
        with open(a.traffic_json) as f:
            tj = json.load(f)
        key = "eri_jk_" + "".join("spd"[x] for x in cls)
        if tj.get("kernel") == key and tj.get("workload") == "c2" and \
                tj.get("source_sha256") == kernel_source_hash("".join("spd"[x] for x in cls)):
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
            "accumulation": "deterministic fixed point",
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
            "flops_per_prim_quartet": f_prim,
            "flops_per_quartet_fixed": f_fixed,
            "prim_quartets_per_launch": nprimq,
            "quartets_per_launch": counts[cls],
            "avg_launch_ms": avg_s * 1e3,
            "timing": "per-class HIP events over a second timed pass of the same steps, classes serialized",
            "serialized_ms_per_step": (t3 - t2) / a.steps * 1e3,
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
