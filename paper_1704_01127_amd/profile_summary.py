"""Summarise rocprofv3 output for the committed profiles.

Reads a kernel-trace stats CSV (``--kernel-trace --stats``) and, optionally,
two counter-collection CSVs (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``)
plus the same counters for a calibration kernel of known traffic (the stream
probe's in-place pass over ``--cal-bytes`` bytes, which reads and writes each
byte once). Writes a short Markdown summary and a JSON record of calibrated
HBM bytes per launch for each kernel.

    python -m paper_1704_01127_amd.profile_summary --stats S.csv --fetch F.csv --write W.csv \\
        --cal-fetch CF.csv --cal-write CW.csv --cal-bytes 8589934592 --command "..." \\
        --out-md profiles/x.md --out-json profiles/x.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_sha() -> str:
    with open(os.path.join(HERE, "csrc", "qsim_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def demangle(name: str) -> str:
    """Itanium-demangled name (rocprofv3 leaves some names mangled)."""
    if not name.startswith("_Z"):
        return name
    import re
    import subprocess
    try:
        r = subprocess.run(["c++filt", name], capture_output=True, text=True, timeout=10)
        out = r.stdout.strip()
    except (OSError, subprocess.SubprocessError):
        out = ""
    if out and out != name:
        return out
    # c++filt does not know _Float16 vector parameters: read the qualified
    # name and its bool template arguments by hand
    m = re.match(r"_ZN4qsim(\d+)", name)
    if not m:
        return name
    ln = int(m.group(1))
    base = name[m.end():m.end() + ln]
    rest = name[m.end() + ln:]
    t = re.match(r"I((?:Lb[01]E)+)E", rest)
    if not t:
        return base
    args = ["true" if b == "1" else "false" for b in re.findall(r"Lb([01])E", t.group(1))]
    return base + "<%s>" % ", ".join(args)


def short(name: str) -> str:
    n = demangle(name).split("(")[0]
    for p in ("void ", "qsim::"):
        n = n.replace(p, "")
    return n.strip()


def counters(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return d


PEAK_TFLOPS = {"F16": 2500.0, "F32": 157.3, "F64": 78.6}  # MI355X dense matrix-core peaks


def mfma_table(path):
    """Per kernel: matrix-core FLOP rate from SQ_INSTS_VALU_MFMA_MOPS_* (units
    of 512 FLOP) over the dispatches' own durations."""
    disp = collections.defaultdict(dict)
    for r in csv.DictReader(open(path)):
        d = disp[(short(r["Kernel_Name"]), r["Dispatch_Id"])]
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    for (k, _), d in disp.items():
        a = agg[k]
        a["n"] += 1
        for c, v in d.items():
            a[c] += v
    lines = ["| kernel | dispatches | avg ms | MFMA TFLOP/s (f16 / f32 / f64) | % of that dtype's peak |",
             "|---|---:|---:|---|---:|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["ns"]):
        sec = a["ns"] * 1e-9
        rates = {t: a.get("SQ_INSTS_VALU_MFMA_MOPS_" + t, 0.0) * 512 / sec / 1e12 if sec > 0 else 0.0
                 for t in ("F16", "F32", "F64")}
        if sum(rates.values()) == 0:
            continue
        top = max(rates, key=rates.get)
        lines.append("| `%s` | %d | %.3f | %.1f / %.1f / %.1f | %.1f %% (%s) |" % (
            k, a["n"], a["ns"] / a["n"] / 1e6, rates["F16"], rates["F32"], rates["F64"],
            100 * rates[top] / PEAK_TFLOPS[top], top.lower()))
    return lines


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cal-fetch")
    ap.add_argument("--cal-write")
    ap.add_argument("--cal-kernel", default="k_inplace<4, true>")
    ap.add_argument("--cal-bytes", type=float, default=8589934592.0)
    ap.add_argument("--command", required=True)
    ap.add_argument("--pmc-command", default="")
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--algorithmic", default="",
                    help="kernel=bytes,... algorithmic bytes per launch to compare with")
    ap.add_argument("--mfma", help="counter CSV of SQ_INSTS_VALU_MFMA_MOPS_F16 / F32 / F64")
    ap.add_argument("--mfma-command", default="")
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json")
    args = ap.parse_args(argv)

    rows = list(csv.DictReader(open(args.stats)))
    lines = ["# " + args.title, "", "Command (kernel trace):", "", "    " + args.command, ""]
    lines += ["| kernel | calls | avg ms | total ms | % GPU time |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append("| `%s` | %s | %.4f | %.1f | %.2f |" % (short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e6,
                                                         float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    rec = {"kernel_source_sha": kernel_source_sha(), "kernels": {}}
    if args.fetch and args.write and args.cal_fetch and args.cal_write:
        cf, cw = counters(args.cal_fetch), counters(args.cal_write)
        f_fac = args.cal_bytes / (sum(cf[args.cal_kernel]) / len(cf[args.cal_kernel]) * 1024)
        w_fac = args.cal_bytes / (sum(cw[args.cal_kernel]) / len(cw[args.cal_kernel]) * 1024)
        fe, wr = counters(args.fetch), counters(args.write)
        alg = {}
        for item in filter(None, args.algorithmic.split(";")):
            k, v = item.rsplit("=", 1)
            alg[k.strip()] = float(v)
        lines += ["", "HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, separate runs):", "",
                  "    " + args.pmc_command, "",
                  "Calibration: `%s` over %.0f bytes read and written once reads FETCH_SIZE x %.3f and "
                  "WRITE_SIZE x %.3f of the true bytes; the factors below are applied." % (
                      args.cal_kernel, args.cal_bytes, 1 / f_fac, 1 / w_fac), "",
                  "| kernel | launches | fetch GB | write GB | total GB | algorithmic GB |",
                  "|---|---:|---:|---:|---:|---:|"]
        for k in fe:
            if k not in wr:
                continue
            f = sum(fe[k]) / len(fe[k]) * 1024 * f_fac
            w = sum(wr[k]) / len(wr[k]) * 1024 * w_fac
            rec["kernels"][k] = {"fetch_bytes": f, "write_bytes": w, "bytes_per_launch": f + w, "launches": len(fe[k])}
            a = alg.get(k)
            lines.append("| `%s` | %d | %.3f | %.3f | %.3f | %s |" % (k, len(fe[k]), f / 1e9, w / 1e9, (f + w) / 1e9,
                                                                   "%.3f" % (a / 1e9) if a else ""))
        rec["fetch_factor"], rec["write_factor"] = f_fac, w_fac
    if args.mfma:
        lines += ["", "Matrix-core use per kernel (rocprofv3 --pmc, its own run; rate = MOPS x 512 FLOP over the "
                  "dispatch durations of that run, peaks: f16 2.5 PFLOP/s, f32 157.3, f64 78.6 TFLOP/s dense):", "",
                  "    " + args.mfma_command, ""] + mfma_table(args.mfma)
    lines += ["", "Kernel source sha256[:16] of qsim_kernels.hip: `%s`" % rec["kernel_source_sha"], ""]
    with open(args.out_md, "w") as f:
        f.write("\n".join(lines))
    if args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
