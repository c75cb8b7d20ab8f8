"""HBM traffic of the dominant kernel from rocprofv3 counter runs.

Two steps, each a command of its own:

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
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))

# kernel kinds (as reported by tw_plan_get_profile) -> substrings of their
# compiled names as rocprofv3 prints them
KIND_PATTERNS = {
    "pass_kick_drift": (", 5, true>", "cols_kernel<double, 512, 5>", "cols_kernel<float, 512, 5>",
                        ", 5, false>"),
    "pass_drift_rho": (", 1, true>", ", 1, false>", "cols_kernel<double, 512, 1>", "cols_kernel<float, 512, 1>"),
}
SOURCES = ("csrc/fft.hpp", "csrc/common.hpp", "csrc/pass_common.hpp", "csrc/pass_rows.hpp", "csrc/pass_cols.hpp",
           "csrc/kernels_step.hip", "csrc/kernels_cols.hip")


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
            out.extend(csv.DictReader(f))
    return out


def _per_dispatch(rows, counter, match):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        if not match(name):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def summarize(a):
    pats = KIND_PATTERNS[a.kind]
    is_kind = lambda n: "pass_kernel" in n or "cols_kernel" in n
    match = lambda n: is_kind(n) and any(p in n for p in pats)
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
    print(json.dumps(out))


def copy(a):
    import torch
    n = a.mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x3", flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    s = sub.add_parser("summarize")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        s.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    s.add_argument("--kind", default="pass_kick_drift")
    s.add_argument("--copy-mib", dest="copy_mib", type=int, default=1024)
    s.add_argument("--commands", default="")
    a = ap.parse_args()
    if a.cmd == "copy":
        copy(a)
    else:
        summarize(a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
