"""Markdown summaries of rocprofv3 result databases (rocpd SQLite) for the
library's kernels: kernel-trace statistics, HBM traffic from FETCH_SIZE /
WRITE_SIZE calibrated against a plain device copy, and VALU counters.

    python -m paper_1905_01381_amd.rocpd_summary trace DB
    python -m paper_1905_01381_amd.rocpd_summary traffic FETCH_DB WRITE_DB COPY_MIB
    python -m paper_1905_01381_amd.rocpd_summary valu DB

Only the standard library is used; nothing here touches the GPU.
"""
from __future__ import annotations

import collections
import sqlite3
import sys

SIMDS = 256 * 4          # compute units x SIMDs
FP64_ISSUE = 0.25        # wave64 FP64 VALU instructions per SIMD and cycle (16 lanes per cycle)


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def trace(db: str) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels").fetchall()
    per = collections.defaultdict(list)
    for n, d in rows:
        per[_short(n)].append(d / 1e6)
    total = sum(sum(v) for v in per.values())
    out = ["| kernel | calls | total ms | avg ms | min ms | max ms | % |", "|---|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {k} | {len(v)} | {sum(v):.2f} | {sum(v) / len(v):.3f} | {min(v):.3f} | {max(v):.3f} | "
                   f"{100 * sum(v) / total:.1f} |")
    return "\n".join(out)


def _pmc(db: str):
    """{dispatch: (kernel, duration ns, {counter: (sum over instances, max over instances)})}"""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, name, duration, counter_name, counter_value from pmc_events").fetchall()
    out = {}
    for d, n, du, cn, cv in rows:
        k, _, cnt = out.setdefault(d, (_short(n), du, {}))
        s, m = cnt.get(cn, (0.0, 0.0))
        cnt[cn] = (s + cv, max(m, cv))
    return out


def traffic(fetch_db: str, write_db: str, copy_mib: float) -> str:
    f, w = _pmc(fetch_db), _pmc(write_db)

    def calib(p, cn):
        best = max((v[2][cn][0] for v in p.values() if "copyBuffer" in v[0] and cn in v[2]), default=0.0)
        return copy_mib * 1024.0 / best if best else float("nan"), best

    ff, fr = calib(f, "FETCH_SIZE")
    wf, wr = calib(w, "WRITE_SIZE")
    per = collections.defaultdict(lambda: [0.0, 0.0, 0.0, 0.0, 0, 0])
    for p, cn, i in ((f, "FETCH_SIZE", 0), (w, "WRITE_SIZE", 1)):
        for k, du, cnt in p.values():
            if not k.startswith("eri_") or cn not in cnt:
                continue
            per[k][i] += cnt[cn][0]
            per[k][4 + i] += 1
            per[k][2 + i] += du
    out = [f"Calibration: a {copy_mib:g} MiB device copy reads FETCH_SIZE {fr:.0f} KiB (factor {ff:.4f}) and "
           f"WRITE_SIZE {wr:.0f} KiB (factor {wf:.4f}); each value below is the raw counter per dispatch times "
           "its factor, averaged over the kernel's dispatches.", "",
           "| kernel | avg ms | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | HBM read GB | HBM write GB | GB/s |",
           "|---|---|---|---|---|---|---|"]
    for k, (fs, ws, fd, wd, nf, nw) in sorted(per.items(), key=lambda kv: -(kv[1][2] / max(kv[1][4], 1))):
        if not nf or not nw:
            continue
        fk, wk = fs / nf, ws / nw
        rd, wrt = fk * ff * 1024 / 1e9, wk * wf * 1024 / 1e9
        ms = (fd / nf + wd / nw) / 2 / 1e6
        out.append(f"| {k} | {ms:.2f} | {fk:.4g} | {wk:.4g} | {rd:.2f} | {wrt:.2f} | {(rd + wrt) / ms * 1e3:.0f} |")
    return "\n".join(out)


def valu(db: str) -> str:
    p = _pmc(db)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    n = collections.Counter()
    for k, du, cnt in p.values():
        if not k.startswith("eri_"):
            continue
        n[k] += 1
        per[k]["ms"] += du / 1e6
        for cn, (s, m) in cnt.items():
            per[k][cn] += m if cn == "GRBM_GUI_ACTIVE" else s
    out = ["| kernel | avg ms | VALU instr (wave) | FP64 flops executed | FP64 TFLOP/s executed | VALU issue / FP64 rate | waves |",
           "|---|---|---|---|---|---|---|"]
    for k in sorted(per, key=lambda k: -per[k]["ms"] / n[k]):
        a, c = per[k], n[k]
        ms = a["ms"] / c
        flops = a.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) / c * 64
        cyc = a.get("GRBM_GUI_ACTIVE", 0.0) / c
        issue = (a.get("SQ_INSTS_VALU", 0.0) / c) / SIMDS / cyc / FP64_ISSUE if cyc else float("nan")
        out.append(f"| {k} | {ms:.2f} | {a.get('SQ_INSTS_VALU', 0) / c:.3e} | {flops:.3e} | {flops / ms / 1e9:.1f} | "
                   f"{issue:.2f} | {a.get('SQ_WAVES', 0) / c:.0f} |")
    return "\n".join(out)


def main(argv):
    if len(argv) >= 2 and argv[0] == "trace":
        print(trace(argv[1]))
    elif len(argv) >= 4 and argv[0] == "traffic":
        print(traffic(argv[1], argv[2], float(argv[3])))
    elif len(argv) >= 2 and argv[0] == "valu":
        print(valu(argv[1]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
