"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1408_4495_amd.profile_summary stats <kernel_stats.csv> <title> <command>
        per-kernel time table (markdown) from a --kernel-trace --stats run;
    python -m paper_1408_4495_amd.profile_summary counters <counter_collection.csv> <kernel_trace.csv> <title> <cmd>
        per-kernel counter means (duration-weighted) and sums from one --pmc run;
    python -m paper_1408_4495_amd.profile_summary traffic <fetch.csv> <write.csv> <title> <cmd_fetch> <cmd_write>
        per-kernel HBM bytes from two --pmc runs (FETCH_SIZE, then WRITE_SIZE,
        counter_collection.csv each) of profile_probe, which ends with a
        device-to-device copy of known size: each counter is scaled by what
        it reads for that copy.  Kernels are keyed like the library's timing
        registry ("bwd [c64]"), with the SHA-256 of the source file holding
        the kernel, so a reader can tell whether the record still applies.
"""
import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
SOURCE = {"fwd": "frontal.hip", "bwd": "frontal.hip", "diag_lu": "frontal.hip", "panel_trsm": "frontal.hip",
          "gemm_update": "frontal.hip", "update_lu": "frontal.hip", "pair_update": "frontal.hip",
          "cross_update": "frontal.hip", "assemble_front": "frontal.hip",
          "strip_first": "frontal.hip", "panel_step": "frontal.hip", "form_fwd": "frontal.hip",
          "form_bwd": "frontal.hip", "bsweep": "sweep.hip", "mchain": "sweep.hip",
          "fwd_mchain": "sweep.hip", "bwd_mchain": "sweep.hip",
          "half_lines": "fft.hip", "full_lines": "fft.hip",
          "gram": "stencil.hip", "gram_reduce": "stencil.hip", "eigen": "stencil.hip", "applyQ": "stencil.hip",
          "dots_partial": "krylov.hip", "dots_final": "krylov.hip", "axpy": "krylov.hip", "cgs": "krylov.hip",
          "scale_norm": "krylov.hip", "givens": "krylov.hip", "ktable": "greens.hip"}
FFT_KIND = {"0": "fft_first", "1": "fft_axis_fwd", "2": "fft_conv", "3": "fft_axis_inv", "4": "fft_last"}


def short(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("lsp::", "")
    return re.sub(r"\(.*", "", name).strip()


def registry_key(name):
    """Kernel symbol -> the timing-registry name, e.g. bwd_kernel<float, 1, true> -> 'bwd [c64]'."""
    s = short(name)
    m = re.match(r"(\w+?)_kernel(?:<(.*)>)?$", s)
    if not m:
        return None, None
    base, targs = m.group(1), (m.group(2) or "")
    args = [a.strip() for a in targs.split(",")] if targs else []
    if base == "half_lines" and len(args) == 4:
        base = FFT_KIND.get(args[2], base)
    if base == "full_lines":
        base = "fft_full"
    if base == "gemm_update" and args and args[-1] == "true":
        base = "update_lu"  # fused with the next diagonal-block factorisation
    if base in ("fwd_small", "bwd_small"):
        base = base[:3]  # the small-front levels' sweeps, timed under the same name
    if base in ("mchain_fwd", "mchain_bwd"):
        base = base[7:] + "_mchain"  # timed as fwd_mchain / bwd_mchain
    if base == "fwd" and len(args) >= 2 and args[-2] == "true":
        # the forward chain (or the transposed backward one) run on unit
        # vectors: formation of a dense level's operators
        base = "form_bwd" if args[-1] == "true" else "form_fwd"
    prec = ""
    if args:
        if re.match(r"(HIP_vector_type<)?float\b", args[0]):
            prec = " [c64]"
        elif re.match(r"(HIP_vector_type<)?double\b", args[0]):
            prec = " [c128]"
    src = SOURCE.get(base) or SOURCE.get(base.split("_")[0]) or ("fft.hip" if base.startswith("fft_") else None)
    return base + prec, src


def stats(path, title, cmd):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", "Command (from the repository root, on the MI355X):", "", "```", cmd, "```", "",
           f"Total kernel time {tot / 1e6:.3f} ms.", "",
           "| kernel | calls | total ms | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        t = float(r["TotalDurationNs"])
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {t / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {100 * t / tot:.1f}% |")
    # the same launches grouped under the library's timing names (template
    # instances of one kernel together), whose averages bench.py's live
    # timing reports
    agg = {}
    for r in rows:
        key, _ = registry_key(r["Name"])
        if key is None:
            continue
        a = agg.setdefault(key, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
    out += ["", "Grouped by the library's timing names (all template instances of a kernel):", "",
            "| timing name | calls | total ms | avg us |", "|---|---|---|---|"]
    for key, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:25]:
        out.append(f"| `{key}` | {c} | {t / 1e6:.3f} | {t / c / 1e3:.2f} |")
    return "\n".join(out) + "\n"


def traffic(fetch_csv, write_csv, title, cmd_f, cmd_w):
    def load(path):
        rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
        return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]
    f, w = load(fetch_csv), load(write_csv)
    if [a for a, _ in f] != [a for a, _ in w]:
        raise SystemExit("the two runs dispatched different kernel sequences")
    # calibration: the last dispatch is the device-to-device copy of known size
    copy_name, copy_f = f[-1]
    copy_w = w[-1][1]
    copy_bytes = int(os.environ.get("LSP_COPY_BYTES", str(256 << 20)))
    fs = copy_bytes / (copy_f * 1024.0)
    ws = copy_bytes / (copy_w * 1024.0)
    agg = {}
    for (name, fv), (_, wv) in zip(f[:-1], w[:-1]):
        key, src = registry_key(name)
        if key is None or src is None:
            continue
        a = agg.setdefault(key, {"launches": 0, "fetch_kib": 0.0, "write_kib": 0.0, "source": src})
        a["launches"] += 1
        a["fetch_kib"] += fv
        a["write_kib"] += wv
    kernels = {}
    lines = [f"# {title}", "", "Commands (from the repository root, on the MI355X):", "", "```", cmd_f, cmd_w, "```", "",
             f"Calibration: the final `{short(copy_name)}` moves {copy_bytes} bytes each way and reads "
             f"FETCH_SIZE {copy_f:.1f} KiB, WRITE_SIZE {copy_w:.1f} KiB, so HBM bytes = "
             f"FETCH_SIZE x 1024 x {fs:.3f} + WRITE_SIZE x 1024 x {ws:.3f}.", "",
             "| kernel | launches | read MB | written MB | bytes per launch |", "|---|---|---|---|---|"]
    for key, a in sorted(agg.items(), key=lambda kv: -(kv[1]["fetch_kib"] * fs + kv[1]["write_kib"] * ws)):
        rd = a["fetch_kib"] * 1024 * fs
        wr = a["write_kib"] * 1024 * ws
        per = (rd + wr) / a["launches"]
        sha = hashlib.sha256(open(os.path.join(CSRC, a["source"]), "rb").read()).hexdigest()
        kernels[key] = {"launches": a["launches"], "bytes_per_launch": per, "source": a["source"], "sha256": sha}
        lines.append(f"| `{key}` | {a['launches']} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | {per:.0f} |")
    rec = {"fetch_scale": fs, "write_scale": ws, "command": cmd_f + " ; " + cmd_w, "kernels": kernels}
    lines += ["", "<!-- traffic-json: " + json.dumps(rec) + " -->"]
    return "\n".join(lines) + "\n"


def counters(csv_path, trace_path, title, cmd):
    """Per-kernel sums of the counters of one --pmc run (derived metrics as
    rocprofv3 reports them per dispatch, averaged over a kernel's dispatches
    weighted by duration), with the durations from the same run's trace."""
    rows = list(csv.DictReader(open(csv_path)))
    dur = {}
    for r in csv.DictReader(open(trace_path)):
        dur[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    per = {}
    for r in rows:
        key, _ = registry_key(r["Kernel_Name"])
        if key is None:
            continue
        a = per.setdefault(key, {"dispatches": set(), "time": 0.0, "vals": {}})
        did = r["Dispatch_Id"]
        t = dur.get(did, 0.0)
        if did not in a["dispatches"]:
            a["dispatches"].add(did)
            a["time"] += t
        v = a["vals"].setdefault(r["Counter_Name"], [0.0, 0.0])
        v[0] += float(r["Counter_Value"]) * t   # duration-weighted (rates, percentages)
        v[1] += float(r["Counter_Value"])       # plain sum (counts, flops)
    names = sorted({n for a in per.values() for n in a["vals"]})
    out = [f"# {title}", "", "Command (from the repository root, on the MI355X):", "", "```", cmd, "```", "",
           "Per kernel: dispatches, summed duration, and for each counter the duration-weighted mean "
           "(percentages) and the sum over dispatches (counts).", "",
           "| kernel | dispatches | ms | " + " | ".join(f"{n} (mean) | {n} (sum)" for n in names) + " |",
           "|---|---|---|" + "---|---|" * len(names)]
    for key, a in sorted(per.items(), key=lambda kv: -kv[1]["time"])[:20]:
        cells = []
        for n in names:
            v = a["vals"].get(n, [0.0, 0.0])
            cells += [f"{v[0] / a['time']:.3g}" if a["time"] > 0 else "-", f"{v[1]:.4g}"]
        out.append(f"| `{key}` | {len(a['dispatches'])} | {a['time'] * 1e3:.3f} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def main():
    mode = sys.argv[1]
    if mode == "stats":
        sys.stdout.write(stats(*sys.argv[2:5]))
    elif mode == "traffic":
        sys.stdout.write(traffic(*sys.argv[2:7]))
    elif mode == "counters":
        sys.stdout.write(counters(*sys.argv[2:6]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()
