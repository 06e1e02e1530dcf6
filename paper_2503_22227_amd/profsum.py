"""Summarise rocprofv3 result databases (``*_results.db``) as short text tables.

    python -m paper_2503_22227_amd.profsum stats  <results.db>
    python -m paper_2503_22227_amd.profsum pmc    <results.db>
    python -m paper_2503_22227_amd.profsum valu   <results.db>
    python -m paper_2503_22227_amd.profsum traffic <fetch.db> <write.db> <copy_fetch.db> <copy_write.db> <copy_bytes>
    python -m paper_2503_22227_amd.profsum micro  <bench.py --ntt-microbench output>

``stats``: per kernel, launches and average / min / max duration.
``pmc``: per kernel, launches and the average value of every collected counter.
``valu``: per kernel, VALU instructions per launch, the fraction of the chip's
VALU issue slots they take, mean resident waves per SIMD and LDS instructions
(from SQ_INSTS_VALU, SQ_WAVE_CYCLES, SQ_INSTS_LDS of a --kernel-trace --pmc run).
``traffic``: per kernel, HBM bytes per launch from FETCH_SIZE and WRITE_SIZE
(KiB per dispatch), each scaled by what the same counter reads for a plain
device copy of ``copy_bytes`` bytes (expected: copy_bytes read and written).
``micro``: the NTT pass sweep of ``bench.py --ntt-microbench`` (its JSON line) as
one row per pass and launch size.
"""
from __future__ import annotations

import re
import sqlite3
import sys
from collections import defaultdict


def short(name: str) -> str:
    name = re.sub(r"\(.*\)$", "", name)
    name = name.replace("void ", "").replace("rf::", "")
    return name.strip()


def dispatches(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    con.close()
    return [(short(n), d) for n, d in rows]


def counters(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, dispatch_id, counter_name, counter_value from pmc_events").fetchall()
    con.close()
    per = defaultdict(lambda: defaultdict(list))
    for n, did, cname, v in rows:
        per[short(n)][cname].append(v)
    return per


def stats(db: str) -> str:
    acc = defaultdict(list)
    for n, d in dispatches(db):
        acc[n].append(d)
    total = sum(sum(v) for v in acc.values())
    lines = ["| kernel | launches | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for n, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| %s | %d | %.2f | %.2f | %.2f | %.1f%% |" % (
            n, len(v), sum(v) / len(v) / 1e3, min(v) / 1e3, max(v) / 1e3, 100.0 * sum(v) / total))
    return "\n".join(lines)


def pmc(db: str) -> str:
    per = counters(db)
    names = sorted({c for v in per.values() for c in v})
    lines = ["| kernel | launches | " + " | ".join("avg %s" % c for c in names) + " |",
             "|---|---|" + "---|" * len(names)]
    for n, cs in sorted(per.items()):
        cnt = max(len(x) for x in cs.values())
        lines.append("| %s | %d | " % (n, cnt) + " | ".join(
            "%.1f" % (sum(cs[c]) / len(cs[c])) if cs.get(c) else "-" for c in names) + " |")
    return "\n".join(lines)


def valu(db: str) -> str:
    """Per-kernel VALU work and occupancy from one rocprofv3 --kernel-trace --pmc run
    with SQ_WAVES, SQ_INSTS_VALU, SQ_WAVE_CYCLES, SQ_INSTS_LDS (and others).  A
    counter of a dispatch is the sum over the instances it is reported for.
    VALU issue = wave-instructions x 4 cycles / (duration x 2.4 GHz x 1024 SIMDs),
    the fraction of the chip's issue slots if every instruction took 4 cycles;
    waves/SIMD = SQ_WAVE_CYCLES (quad-cycles) x 4 / (duration cycles x 1024),
    the mean number of resident waves per SIMD over the kernel."""
    con = sqlite3.connect(db)
    disp = {did: (short(n), dur, vg, agpr, lds, scr, gx * gy * gz)
            for did, n, dur, vg, agpr, lds, scr, gx, gy, gz in con.execute(
                "select dispatch_id, name, duration, vgpr_count, accum_vgpr_count, lds_size, scratch_size, "
                "grid_x, grid_y, grid_z from kernels")}
    sums = defaultdict(lambda: defaultdict(float))
    for did, cname, v in con.execute("select dispatch_id, counter_name, counter_value from pmc_events"):
        sums[did][cname] += v
    con.close()
    per = defaultdict(list)
    for did, (n, dur, vg, agpr, lds, scr, threads) in disp.items():
        per[n].append((dur, vg + agpr, lds, scr, threads, sums.get(did, {})))
    lines = ["| kernel | launches | avg us | LDS B | scratch B | waves/launch | VALU Minstr/launch "
             "| VALU issue | waves/SIMD | LDS instr/launch |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for n, rows in sorted(per.items(), key=lambda kv: -sum(r[0] for r in kv[1])):
        k = len(rows)
        dur = sum(r[0] for r in rows) / k
        valu_i = sum(r[5].get("SQ_INSTS_VALU", 0.0) for r in rows) / k
        wcyc = sum(r[5].get("SQ_WAVE_CYCLES", 0.0) for r in rows) / k
        lds_i = sum(r[5].get("SQ_INSTS_LDS", 0.0) for r in rows) / k
        cycles = dur * 2.4  # ns -> cycles at 2.4 GHz
        issue = valu_i * 4 / (cycles * 1024) if cycles else float("nan")
        occ = wcyc * 4 / (cycles * 1024) if cycles else float("nan")
        lines.append("| %s | %d | %.2f | %d | %d | %d | %.2f | %.2f | %.2f | %.0f |" % (
            n, k, dur / 1e3, rows[0][2], rows[0][3], rows[0][4] // 64, valu_i / 1e6, issue, occ, lds_i))
    return "\n".join(lines)


def _avg(per, kernel_pred, cname):
    vals = [v for n, cs in per.items() if kernel_pred(n) for v in cs.get(cname, [])]
    return sum(vals) / len(vals) if vals else float("nan")


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes) -> str:
    f, w = counters(fetch_db), counters(write_db)
    cf, cw = counters(copy_fetch_db), counters(copy_write_db)
    copy_kernel = lambda n: "copybuffer" in n.lower()  # noqa: E731
    kf = _avg(cf, copy_kernel, "FETCH_SIZE")
    kw = _avg(cw, copy_kernel, "WRITE_SIZE")
    sf = copy_bytes / (kf * 1024.0)
    sw = copy_bytes / (kw * 1024.0)
    lines = ["copy calibration: %d B per launch read FETCH_SIZE %.1f KiB (scale %.4f), "
             "WRITE_SIZE %.1f KiB (scale %.4f)" % (copy_bytes, kf, sf, kw, sw), "",
             "| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MB | HBM write MB | total MB |",
             "|---|---|---|---|---|---|---|"]
    for n in sorted(set(f) | set(w)):
        fv = f.get(n, {}).get("FETCH_SIZE", [])
        wv = w.get(n, {}).get("WRITE_SIZE", [])
        if not fv or not wv:
            continue
        af, aw = sum(fv) / len(fv), sum(wv) / len(wv)
        rd, wr = af * 1024 * sf / 1e6, aw * 1024 * sw / 1e6
        lines.append("| %s | %d | %.1f | %.1f | %.2f | %.2f | %.2f |" % (n, len(fv), af, aw, rd, wr, rd + wr))
    return "\n".join(lines)


def micro(path: str) -> str:
    import json
    line = [l for l in open(path).read().splitlines() if l.startswith("{")][-1]
    d = json.loads(line)["limbs"]
    out = ["| pass | limbs | avg us | us per limb | algorithmic MB | HBM frac | VALU frac (24 ops) |",
           "|---|---|---|---|---|---|---|"]
    names = sorted({k for ks in d.values() for k in ks})
    for k in names:
        for limbs in sorted(d, key=int):
            v = d[limbs].get(k)
            if v:
                out.append("| %s | %s | %.2f | %.4f | %.1f | %.3f | %.3f |" % (
                    k, limbs, v["avg_us"], v["us_per_limb"], v["mb"], v["hbm_frac"], v["valu_frac_24ops"]))
    return "\n".join(out)


def source_digest() -> str:
    """sha1 over the library's HIP sources: a counter table is valid only for the code it measured."""
    import hashlib
    import os
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha1()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def main(argv):
    mode = argv[1]
    if mode == "stats":
        print(stats(argv[2]))
    elif mode == "pmc":
        print(pmc(argv[2]))
    elif mode == "valu":
        print(valu(argv[2]))
    elif mode == "micro":
        print(micro(argv[2]))
    elif mode == "traffic":
        print(traffic(argv[2], argv[3], argv[4], argv[5], int(argv[6])))
        print()
        print("source-sha1: %s" % source_digest())
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
