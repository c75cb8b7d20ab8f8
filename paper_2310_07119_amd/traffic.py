"""Summaries of rocprofv3 runs: per-kernel durations and the HBM traffic of the
dominant kernel.

  python -m paper_2310_07119_amd.traffic kernels --dir DIR --timed-launches K \
      --bench-log LOG --command CMD --out FILE.md
      reads a `rocprofv3 --kernel-trace --stats` output directory and writes a
      markdown summary: the stats table, and for every pass kernel the average
      of its last K dispatches (the timed region of a bench run, after the
      autotuner's and warmup launches) next to the per-launch average the
      bench measured itself with HIP events (taken from the JSON line in LOG).

The traffic figure takes two counter runs and a calibration:

  python -m paper_2310_07119_amd.traffic copy --mib 1024
      a plain device-to-device copy of a known size (run it under
      `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE`): the counters' reading
      for it, divided by the bytes it must move, is the scale factor of each counter.

  python -m paper_2310_07119_amd.traffic summarize --fetch DIR --write DIR \
      --copy-fetch DIR --copy-write DIR --kind pass_kick_drift --out FILE
      reads the four counter-collection CSVs, averages FETCH_SIZE and WRITE_SIZE
      (KiB per dispatch) over the dispatches of the kernel kind, scales them and
      writes a JSON summary together with a digest of the kernel sources, so a
      reader can tell whether the kernels changed since the counters were taken.

  python -m paper_2310_07119_amd.traffic counters --dirs DIR [DIR ...] --out FILE.md
      per-dispatch SQ counters of the pass kernels of one precision and length
      (from one or more --pmc runs) with rocprofv3's own derived figures:
      VALU busy, LDS activity, bank-conflict cycles and conflicts per access,
      and the FP64 FLOP rate from the instruction counts.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))

# kernel kinds (as reported by tw_plan_get_profile) -> pass mode in the
# compiled kernel names (pass_kernel<T, N, MODE, ROWS> / cols_kernel<T, N, MODE>)
KIND_MODES = {"pass_drift": 0, "pass_drift_rho": 1, "pass_zfwd": 2, "pass_zpoisson": 3, "pass_zinv": 4,
              "pass_kick_drift": 5, "pass_rho": 6, "pass_kin_sum": 7, "pass_pot_sum": 8}
# xy-plane passes of D = 3 (slab_kernel<T, N, MODE>)
SLAB_MODES = {"pass_slab_drift": 0, "pass_slab_drift_rho": 1, "pass_slab_poisson": 2, "pass_slab_kick_drift": 3}
SOURCES = ("csrc/fft.hpp", "csrc/common.hpp", "csrc/pass_common.hpp", "csrc/pass_rows.hpp", "csrc/pass_cols.hpp",
           "csrc/kernels_step.hip", "csrc/kernels_cols.hip", "csrc/kernels_slab.hip")


def source_digest():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                r["_run"] = d  # dispatch ids repeat across runs: keys are (run, dispatch)
                out.append(r)
    return out


def _per_dispatch(rows, counter, match):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        if not match(name):
            continue
        key = (r.get("_run"), r.get("Dispatch_Id") or r.get("Correlation_Id"))
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def summarize(a):
    ctype = "double" if a.precision == "fp64" else "float"
    if a.kind in SLAB_MODES:
        tag = f"slab_kernel<{ctype}, {a.length}, {SLAB_MODES[a.kind]}>"
        match = lambda n: tag in n
    else:
        tag = f"<{ctype}, {a.length}, {KIND_MODES[a.kind]}"
        match = lambda n: ("pass_kernel" in n or "cols_kernel" in n) and tag in n
    fetch = _per_dispatch(_rows(a.fetch), "FETCH_SIZE", match)
    write = _per_dispatch(_rows(a.write), "WRITE_SIZE", match)
    copy_match = lambda n: "copy" in n.lower() or "elementwise" in n.lower()
    cf = _per_dispatch(_rows(a.copy_fetch), "FETCH_SIZE", copy_match)
    cw = _per_dispatch(_rows(a.copy_write), "WRITE_SIZE", copy_match)
    copy_bytes = a.copy_mib * 1024 * 1024
    # counters are in KiB per dispatch; the factor maps counter bytes to true bytes
    f_fac = copy_bytes / (max(cf) * 1024.0)
    w_fac = copy_bytes / (max(cw) * 1024.0)
    fb = sum(fetch) / len(fetch) * 1024.0 * f_fac
    wb = sum(write) / len(write) * 1024.0 * w_fac
    out = {"kind": a.kind, "dispatches": [len(fetch), len(write)], "fetch_bytes_per_launch": fb,
           "write_bytes_per_launch": wb, "traffic_bytes_per_launch": fb + wb,
           "copy_scale": {"fetch": f_fac, "write": w_fac, "copy_mib": a.copy_mib},
           "source_digest": source_digest(), "commands": a.commands}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    md = os.path.splitext(a.out)[0] + ".md"
    with open(md, "w") as f:
        f.write(f"# HBM traffic of {a.kind} (rocprofv3 counters)\n\n"
                f"Commands (from the repository root, each its own run):\n\n```\n"
                + a.commands.replace(" ; ", "\n") + "\n```\n\n"
                f"| quantity | value |\n|---|---:|\n"
                f"| dispatches averaged (FETCH, WRITE) | {len(fetch)}, {len(write)} |\n"
                f"| FETCH_SIZE per dispatch, raw KiB | {sum(fetch) / len(fetch):.0f} |\n"
                f"| WRITE_SIZE per dispatch, raw KiB | {sum(write) / len(write):.0f} |\n"
                f"| copy calibration ({a.copy_mib} MiB device copy): true bytes / counter bytes, fetch | {f_fac:.4f} |\n"
                f"| copy calibration, write | {w_fac:.4f} |\n"
                f"| fetched bytes per launch (scaled) | {fb:.4e} |\n"
                f"| written bytes per launch (scaled) | {wb:.4e} |\n"
                f"| total HBM bytes per launch | {fb + wb:.4e} |\n"
                f"| kernel source digest | `{out['source_digest']}` |\n")
    print(json.dumps(out))


MODE_KIND = {m: k for k, m in KIND_MODES.items()}
SLAB_KIND = {m: k for k, m in SLAB_MODES.items()}


def _kind_of(name):
    """(precision, kernel kind) of a pass kernel from its compiled name, else None."""
    import re
    m = re.search(r"(pass|cols|slab)_kernel<(double|float), (\d+), (\d+)", name)
    if not m:
        return None
    kinds = SLAB_KIND if m.group(1) == "slab" else MODE_KIND
    return ("fp64" if m.group(2) == "double" else "fp32"), kinds[int(m.group(4))]


def kernels(a):
    stats = list(csv.DictReader(open(glob.glob(os.path.join(a.dir, "**", "*kernel_stats.csv"), recursive=True)[0])))
    trace = list(csv.DictReader(open(glob.glob(os.path.join(a.dir, "**", "*kernel_trace.csv"), recursive=True)[0])))
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    lines = [f"# rocprofv3 kernel summary: {a.title}", "", "Command (from the repository root):", "",
             "```", a.command, "```", ""]
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    lines += ["## --stats table (all dispatches of the run, autotuner and warmup included)", "",
              "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---:|---:|---:|---:|---:|"]
    for r in stats[: a.top]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", f"Total kernel time {total / 1e6:.1f} ms.", ""]
    if a.timed_launches:
        # last dispatches of every pass kernel name = the timed region of its leg
        kinds = {}
        for r in trace:
            k = _kind_of(r["Kernel_Name"])
            if k is None:
                continue
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            kinds.setdefault(k, []).append((r["Kernel_Name"], dur))
        bench = {}
        if a.bench_log:
            for ln in open(a.bench_log):
                if ln.startswith("{") and '"metric"' in ln:
                    d = json.loads(ln)
                    bench[(d["config"]["precision"], d["roofline"]["kernel"])] = d["roofline"]["avg_launch_ms"] * 1e3
        skip = f", before the last {a.skip_last}" if a.skip_last else ""
        lines += [f"## Timed region: pass kernels, last {a.timed_launches} launches of each kind{skip}", "",
                  "(bench.py runs the K timed steps, then the same K steps once more, profiled, outside the",
                  "timed region; --skip-last K selects the timed launches, which the HIP-event column measures.)", "",
                  "The 2D passes alternate the axis they transform every step, so a kind's launches split",
                  "between its row kernel (`..., true>`) and its strided kernel. Kinds launched fewer times",
                  "per run than this (moments, energies) include warmup launches.", "",
                  "| precision | kind | kernel | launches | avg us |", "|---|---|---|---:|---:|"]
        summary = []
        for (prec, kind), seq in sorted(kinds.items()):
            sel = seq[-(a.timed_launches + a.skip_last):len(seq) - a.skip_last]
            if not sel:  # kinds launched only outside the timed steps (moments, energies)
                continue
            names = {}
            for name, d in sel:
                names.setdefault(name, []).append(d)
            for name, d in names.items():
                lines.append(f"| {prec} | {kind} | `{name[:70]}` | {len(d)} | {sum(d) / len(d):.1f} |")
            summary.append((prec, kind, len(sel), sum(d for _, d in sel) / len(sel)))
        lines += ["", "| precision | kind | launches | rocprofv3 avg us | bench HIP-event avg us |",
                  "|---|---|---:|---:|---:|"]
        for prec, kind, n, avg in summary:
            b = bench.get((prec, kind))
            lines.append(f"| {prec} | {kind} | {n} | {avg:.1f} | {f'{b:.1f}' if b else '-'} |")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def copy(a):
    import torch
    n = a.mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x3", flush=True)


def counters(a):
    """Per-dispatch SQ counters of the pass kernels of one precision and length
    (several --pmc runs), with the derived figures rocprofv3 itself defines:
    VALUBusy = SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE(max), LDS active
    likewise from SQ_LDS_IDX_ACTIVE, LDSBankConflict and conflicts per access
    from SQ_LDS_BANK_CONFLICT. GRBM_GUI_ACTIVE is read as the sum over the XCD
    instances (the per-XCD maximum is taken as sum / xcds)."""
    ctype = "double" if a.precision == "fp64" else "float"
    rows = []
    for d in a.dirs:
        rows.extend(_rows(d))
    lines = [f"# SQ counters of the pass kernels: {a.title}", "", "Commands (from the repository root):", "", "```"]
    lines += a.commands.splitlines() + ["```", ""]
    lines += ["Per dispatch, averaged over the dispatches of each kernel; derived figures as rocprofv3 defines them",
              f"(CU_NUM = {a.cus}, GRBM_GUI_ACTIVE summed over {a.xcds} XCDs).", ""]
    names = sorted({r["Kernel_Name"] for r in rows if _kind_of(r["Kernel_Name"])})
    names = [n for n in names if f"<{ctype}, {a.length}," in n]
    fp = "F64" if a.precision == "fp64" else "F32"
    table = [f"| kernel | kind | dispatches | VALU busy | {fp} FLOP/s (TFLOP/s) | LDS active | LDS bank-conflict cycles | "
             "conflicts per LDS access | wave time waiting | wave time issuing |",
             "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for n in names:
        mode = int(n.split(",")[2].split(">")[0].strip())
        vals = {}
        for cname in sorted({r["Counter_Name"] for r in rows if r["Kernel_Name"] == n}):
            v = _per_dispatch(rows, cname, lambda k, n=n: k == n)
            if v:
                vals[cname] = sum(v) / len(v)
        g = vals.get("GRBM_GUI_ACTIVE")
        if not g:
            continue
        gmax = g / a.xcds
        cyc = a.cus * gmax
        valu = vals.get("SQ_ACTIVE_INST_VALU")
        lds = vals.get("SQ_LDS_IDX_ACTIVE")
        conf = vals.get("SQ_LDS_BANK_CONFLICT")
        wait, issue, wcyc = vals.get("SQ_WAIT_ANY"), vals.get("SQ_ACTIVE_INST_ANY"), vals.get("SQ_WAVE_CYCLES")
        fl = None
        if all(f"SQ_INSTS_VALU_{op}_{fp}" in vals for op in ("ADD", "MUL", "FMA")):
            fl = 64 * (vals[f"SQ_INSTS_VALU_ADD_{fp}"] + vals[f"SQ_INSTS_VALU_MUL_{fp}"] + 2 * vals[f"SQ_INSTS_VALU_FMA_{fp}"])
        durs = {}
        for r in rows:
            if r["Kernel_Name"] == n:
                durs[r.get("Dispatch_Id")] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        dur_s = sum(durs.values()) / len(durs)
        f = lambda x, pct=True: "-" if x is None else (f"{100 * x:.1f}%" if pct else f"{x:.2f}")
        table.append(f"| `{n[:52]}` | {(_kind_of(n) or (None, mode))[1]} | {int(len(_per_dispatch(rows, 'GRBM_GUI_ACTIVE', lambda k, n=n: k == n)))} | "
                     f"{f(valu / cyc if valu else None)} | {f(fl / dur_s / 1e12 if fl else None, False)} | "
                     f"{f(lds / cyc if lds else None)} | {f(conf / cyc if conf else None)} | "
                     f"{f(conf / (lds - conf) if (lds and conf) else None, False)} | "
                     f"{f(wait / wcyc if (wait and wcyc) else None)} | {f(issue / wcyc if (issue and wcyc) else None)} |")
    lines += table
    peak = "FP64 vector peak 78.6" if fp == "F64" else "FP32 vector peak 157.3"
    lines += ["", f"FLOP/s: 64 lanes x (ADD_{fp} + MUL_{fp} + 2 FMA_{fp}) instructions over the dispatch's own "
              f"duration (its end minus start timestamp in the counter run); {peak} TFLOP/s. Wave time waiting "
              "and issuing: SQ_WAIT_ANY and SQ_ACTIVE_INST_ANY over SQ_WAVE_CYCLES (the share of the waves' "
              "lifetime spent waiting on any dependency, and issuing any instruction).", ""]
    raw = ["| kernel | " + " | ".join(c.replace("SQ_", "").replace("GRBM_", "") for c in a.raw) + " |",
           "|---|" + "---:|" * len(a.raw)]
    for n in names:
        cells = []
        for cname in a.raw:
            v = _per_dispatch(rows, cname, lambda k, n=n: k == n)
            cells.append(f"{sum(v) / len(v):.4g}" if v else "-")
        raw.append(f"| `{n[:52]}` | " + " | ".join(cells) + " |")
    lines += ["Raw per-dispatch averages:", ""] + raw + [""]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(table))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    s = sub.add_parser("summarize")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        s.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    s.add_argument("--kind", default="pass_kick_drift")
    s.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    s.add_argument("--length", type=int, default=512, help="transform length of the pass kernels")
    s.add_argument("--copy-mib", dest="copy_mib", type=int, default=1024)
    s.add_argument("--commands", default="")
    k = sub.add_parser("kernels")
    k.add_argument("--dir", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--command", default="")
    k.add_argument("--title", default="")
    k.add_argument("--bench-log", dest="bench_log", default="")
    k.add_argument("--timed-launches", dest="timed_launches", type=int, default=0)
    k.add_argument("--skip-last", dest="skip_last", type=int, default=0)
    k.add_argument("--top", type=int, default=25)
    q = sub.add_parser("counters")
    q.add_argument("--dirs", nargs="+", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    q.add_argument("--length", type=int, default=512)
    q.add_argument("--title", default="")
    q.add_argument("--commands", default="")
    q.add_argument("--cus", type=int, default=256)
    q.add_argument("--xcds", type=int, default=8)
    q.add_argument("--raw", nargs="*", default=["SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_SALU",
                                                 "SQ_ACTIVE_INST_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT",
                                                 "SQ_WAIT_INST_LDS", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "SQ_WAVES",
                                                 "GRBM_GUI_ACTIVE"])
    a = ap.parse_args()
    if a.cmd == "counters":
        counters(a)
        return 0
    if a.cmd == "copy":
        copy(a)
    elif a.cmd == "kernels":
        kernels(a)
    else:
        summarize(a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
