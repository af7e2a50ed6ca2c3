"""Short text summaries of rocprofv3 output for one kernel.

  python -m paper_1505_07368_amd.profsum --kernel drain_kernel_light \\
      --trace T/bench_kernel_trace.csv --last 10 \\
      --fetch F/bench_counter_collection.csv --write W/bench_counter_collection.csv \\
      --copy-fetch CF/copy_counter_collection.csv --copy-write CW/copy_counter_collection.csv \\
      --copy-kernel neg_kernel --copy-bytes 1073741824 --command "..." ...

prints a markdown summary: per-dispatch durations of the kernel from a
--kernel-trace run, optionally matrix-core utilisation from a --pmc run
(--mfma), and its HBM traffic per dispatch from two --pmc runs
(FETCH_SIZE, WRITE_SIZE, in KiB per dispatch).  Each counter is scaled by what
it reads for a copy kernel of known size (bytes read = bytes written =
--copy-bytes per dispatch), since the counters need not count every byte
once.  The summary ends with machine-readable `key: value` lines, including a
digest of the kernel sources, so a reader can tell whether the figures still
describe the code.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "tiles.h",
                                                          "caf_internal.h")]


def source_digest() -> str:
    """sha256 over the device-code sources, in a fixed order."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def dispatch_durations_ns(trace_csv: str, kernel: str) -> list[int]:
    """End - start of every dispatch of `kernel` (substring of the name), in
    dispatch order."""
    rows = [r for r in _rows(trace_csv) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]


def counter_kib(pmc_csv: str, kernel: str, counter: str) -> list[float]:
    rows = [r for r in _rows(pmc_csv) if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows]


def mfma_dispatches(pmc_csv: str, kernel: str, n_xcc: int, simds: int) -> list[dict]:
    """Per dispatch of `kernel`: matrix-core utilisation and flops from
    SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE and SQ_INSTS_VALU_MFMA_MOPS_*
    (512 flops per MOP).  GRBM_GUI_ACTIVE is reported summed over the
    chip's XCCs, so the active cycles of one XCC are that sum / n_xcc."""
    by = {}
    for r in _rows(pmc_csv):
        if kernel in r["Kernel_Name"]:
            by.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    out = []
    for did in sorted(by):
        c = by[did]
        active = c.get("GRBM_GUI_ACTIVE", 0.0) / n_xcc
        busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        mops = sum(v for k, v in c.items() if k.startswith("SQ_INSTS_VALU_MFMA_MOPS_"))
        out.append({"dispatch": did, "util": busy / (active * simds) if active else float("nan"),
                     "flops": mops * 512.0, "active_cycles": active})
    return out


def read_summary(path: str) -> dict:
    """The `key: value` lines of a summary written by this module."""
    out = {}
    if not os.path.exists(path):
        return out
    seen = False
    with open(path) as f:
        for line in f:
            line = line.strip()
            seen = seen or line == "Machine-readable:"
            if seen and line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                out[k.strip()] = v.strip()
    return out


def _mean(v):
    return sum(v) / len(v) if v else float("nan")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--last", type=int, default=0, help="summarise the last N dispatches only")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-kernel", default="neg_kernel")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--pmc-last", type=int, default=0)
    ap.add_argument("--mfma", help="--pmc csv with SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE, "
                    "SQ_INSTS_VALU_MFMA_MOPS_*")
    ap.add_argument("--counters", action="append", default=[],
                    help="--pmc csv of any counters: their per-dispatch means are listed")
    ap.add_argument("--iters", type=float, default=0.0,
                    help="algorithmic escape-time iterations per dispatch: the instruction "
                    "counters are also given per iteration, and SQ_INSTS_VALU as lane "
                    "operations per second over the mean dispatch duration")
    ap.add_argument("--ops-per-iter", type=float, default=9.0)
    ap.add_argument("--valu-peak", type=float, default=0.0,
                    help="VALU lane operations per second of the chip, for the fractions")
    ap.add_argument("--xcc", type=int, default=8)
    ap.add_argument("--simds", type=int, default=1024)
    ap.add_argument("--note", action="append", default=[])
    ap.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)

    dur = dispatch_durations_ns(a.trace, a.kernel)
    sel = dur[-a.last:] if a.last else dur
    lines = [f"# {a.title or a.kernel}", "", "Commands (run from the repository root on the GPU; "
             "`cd /tmp && export TMPDIR=/tmp` first):", ""]
    lines += [f"    {c}" for c in a.command]
    which = f"the last {len(sel)} are the timed steps" if a.last else "all are summarised"
    lines += ["", f"Kernel `{a.kernel}`: {len(dur)} dispatches in the trace; {which}.", ""]
    lines += ["| dispatches | mean ms | min ms | max ms |", "|---|---|---|---|",
              f"| {len(sel)} | {_mean(sel) / 1e6:.4f} | {min(sel) / 1e6:.4f} | "
              f"{max(sel) / 1e6:.4f} |", ""]
    kv = {"kernel": a.kernel, "source_digest": source_digest(),
          "avg_dispatch_ms": f"{_mean(sel) / 1e6:.4f}"}
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        cf = _mean(counter_kib(a.copy_fetch, a.copy_kernel, "FETCH_SIZE")) * 1024.0
        cw = _mean(counter_kib(a.copy_write, a.copy_kernel, "WRITE_SIZE")) * 1024.0
        kf_all = counter_kib(a.fetch, a.kernel, "FETCH_SIZE")
        kw_all = counter_kib(a.write, a.kernel, "WRITE_SIZE")
        n = a.pmc_last
        kf = kf_all[-n:] if n else kf_all
        kw = kw_all[-n:] if n else kw_all
        sf, sw = a.copy_bytes / cf, a.copy_bytes / cw
        fb, wb = _mean(kf) * 1024.0 * sf, _mean(kw) * 1024.0 * sw
        lines += ["HBM traffic per dispatch (counter KiB x 1024 x scale; the scale makes the "
                  f"copy kernel read and write {a.copy_bytes / 2**30:g} GiB per dispatch):", "",
                  "| counter | copy kernel raw bytes | scale | kernel raw KiB (mean) | "
                  "kernel bytes (scaled) |", "|---|---|---|---|---|",
                  f"| FETCH_SIZE | {cf:.4g} | {sf:.3f} | {_mean(kf):.1f} | {fb:.4g} |",
                  f"| WRITE_SIZE | {cw:.4g} | {sw:.3f} | {_mean(kw):.1f} | {wb:.4g} |", ""]
        kv.update({"fetch_scale": f"{sf:.4f}", "write_scale": f"{sw:.4f}",
                   "fetch_bytes_per_dispatch": f"{fb:.0f}",
                   "write_bytes_per_dispatch": f"{wb:.0f}",
                   "traffic_bytes_per_dispatch": f"{fb + wb:.0f}"})
    if a.mfma:
        md = mfma_dispatches(a.mfma, a.kernel, a.xcc, a.simds)
        lines += [f"Matrix cores per dispatch (busy cycles / (active cycles of one XCC x "
                  f"{a.simds} SIMDs); flops = MFMA MOPs x 512):", "",
                  "| dispatch | MFMA utilisation | GFLOP |", "|---|---|---|"]
        lines += [f"| {d['dispatch']} | {100 * d['util']:.1f}% | {d['flops'] / 1e9:.2f} |"
                  for d in md]
        lines += [""]
    if a.counters:
        means = {}
        for path in a.counters:
            by = {}
            for r in _rows(path):
                if a.kernel in r["Kernel_Name"]:
                    by.setdefault(r["Counter_Name"], {})[int(r["Dispatch_Id"])] = \
                        float(r["Counter_Value"])
            for name, per in by.items():
                vals = [per[k] for k in sorted(per)]
                vals = vals[-a.pmc_last:] if a.pmc_last else vals
                means[name] = _mean(vals)
        per_iter = a.iters > 0
        lines += ["Counters, mean per dispatch" + (" (instruction counts are wave "
                  "instructions; per iteration = / the dispatch's algorithmic iterations)"
                  if per_iter else "") + ":", "",
                  "| counter | per dispatch |" + (" per iteration |" if per_iter else ""),
                  "|---|---|" + ("---|" if per_iter else "")]
        for name in sorted(means):
            row = f"| {name} | {means[name]:.6g} |"
            if per_iter:
                row += f" {means[name] / a.iters:.4f} |" if name.startswith("SQ_INSTS") else " |"
            lines.append(row)
        lines.append("")
        for name, v in means.items():
            kv[f"pmc_{name}"] = f"{v:.6g}"
        if per_iter and "SQ_INSTS_VALU" in means:
            t = _mean(sel) * 1e-9
            lane_ops = means["SQ_INSTS_VALU"] * 64.0
            alg = a.iters * a.ops_per_iter
            lines += [f"- Executed VALU lane operations per dispatch (SQ_INSTS_VALU x 64): "
                      f"{lane_ops:.4g}, {lane_ops / t / 1e12:.2f}e12 per second over the "
                      f"mean dispatch; algorithmic ({a.ops_per_iter:g} per iteration): "
                      f"{alg:.4g}, {alg / t / 1e12:.2f}e12 per second; executed / "
                      f"algorithmic = {lane_ops / alg:.4f}."]
            kv.update({"iters_per_dispatch": f"{a.iters:.0f}",
                       "valu_lane_ops_per_s": f"{lane_ops / t:.6g}",
                       "alg_ops_per_s": f"{alg / t:.6g}"})
            if a.valu_peak:
                lines += [f"- Against {a.valu_peak / 1e12:.2f}e12 lane operations per second: "
                          f"executed {lane_ops / t / a.valu_peak:.4f}, algorithmic "
                          f"{alg / t / a.valu_peak:.4f}."]
                kv["alg_frac"] = f"{alg / t / a.valu_peak:.4f}"
            lines.append("")
    lines += [f"- {n}" for n in a.note] + ([""] if a.note else [])
    lines += ["Machine-readable:", ""] + [f"- {k}: {v}" for k, v in kv.items()]
    print("\n".join(lines))


if __name__ == "__main__":
    main()
