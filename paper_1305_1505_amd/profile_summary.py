"""Summaries of rocprofv3 output for this library (run on the host after a profiled run).

    python -m paper_1305_1505_amd.profile_summary trace  <kernel_stats.csv> [out.md]
    python -m paper_1305_1505_amd.profile_summary traffic <fetch counter_collection.csv>
                                                         <write counter_collection.csv> <out.json> [out.md]
    python -m paper_1305_1505_amd.profile_summary issue <SQ counter_collection.csv> <out.json> [out.md]
    python -m paper_1305_1505_amd.profile_summary overlap <kernel_trace.csv>   (serving concurrency)
    (--n=<N> anywhere: the passes of grid size N instead of 512)

`trace` turns a `rocprofv3 --kernel-trace --stats --output-format csv` kernel-stats file into a
markdown table.  `traffic` turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
`bench.py --copy-probe` into HBM bytes per dispatch for each kernel, each counter scaled by what
it reads for the plain device copies of the probe (three 1 GiB copies,
`__amd_rocclr_copyBuffer`, all dispatches together), and records the hash of the kernel sources the counters belong to:
`bench.py` reports the traffic only while the sources still hash to that value.  `issue` turns
one `rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD
SQ_INSTS_VMEM_WR ...` run into instructions per wave for the three per-radius passes, and the
time their VALU instructions alone take to issue: one wave64 instruction per 4 cycles on each
of the 1024 SIMDs (256 CUs x 4, 16 lanes each), at 2.4 GHz.
"""

import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("kernels.hpp", "fft_core.hpp", "collapse_dev.hpp", "trig_poly.hpp", "grf.hpp", "inst.hip")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 3 << 30          # bench.py --copy-probe copies 2^28 float32 (1 GiB) three times

# kernel-class name used by bench.py -> substring of the kernel name at grid size N, float32
KERNEL_PATTERNS = {
    "xpass_hessian": "k_xpass<float, {n}, 0>",
    "ypass_hessian": "k_ypass_packed<float, {n}, 0>",
    "zpass_collapse": "k_zpass<float, {n}, 3, 0>",
}
KERNEL_KEYS = {k: v.format(n=512) for k, v in KERNEL_PATTERNS.items()}


def set_grid_size(n):
    """Summarise the passes of grid size n (default 512)."""
    KERNEL_KEYS.update({k: v.format(n=n) for k, v in KERNEL_PATTERNS.items()})


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def per_kernel_counter(path, counter):
    """{kernel name: [(grid size, value) per dispatch]} for one counter (KiB as rocprofv3 reports
    them; rows repeated for one dispatch are counted once)."""
    out, seen = {}, set()
    for r in _rows(path):
        if r.get("Counter_Name") != counter or r["Dispatch_Id"] in seen:
            continue
        seen.add(r["Dispatch_Id"])
        out.setdefault(r["Kernel_Name"], []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def _probe_kib(per_kernel):
    """Counter total over the copy probe's dispatches: the copy-kernel launches with the largest
    grid (other copies the runtime makes are small)."""
    copies = [gv for k, gvs in per_kernel.items() if COPY_KERNEL in k for gv in gvs]
    if not copies:
        raise SystemExit("the copy probe is missing from the counter runs")
    g = max(gv[0] for gv in copies)
    return sum(v for grid, v in copies if grid == g)


def traffic(fetch_csv, write_csv):
    fetch = per_kernel_counter(fetch_csv, "FETCH_SIZE")
    write = per_kernel_counter(write_csv, "WRITE_SIZE")
    sf = COPY_BYTES / (_probe_kib(fetch) * 1024.0)
    sw = COPY_BYTES / (_probe_kib(write) * 1024.0)
    kernels = {}
    for cls, key in KERNEL_KEYS.items():
        fk = [v for k, gvs in fetch.items() if key in k for _, v in gvs]
        wk = [v for k, gvs in write.items() if key in k for _, v in gvs]
        if fk and wk:
            kernels[cls] = {"fetch_bytes": sf * 1024.0 * sum(fk) / len(fk),
                            "write_bytes": sw * 1024.0 * sum(wk) / len(wk),
                            "dispatches": len(fk)}
    return {"kernel_source_sha256": kernel_source_hash(), "copy_scale_fetch": sf, "copy_scale_write": sw,
            "kernels": kernels}


def traffic_table(t):
    lines = [f"copy calibration: FETCH_SIZE x {t['copy_scale_fetch']:.4f}, WRITE_SIZE x {t['copy_scale_write']:.4f}",
             "", "| kernel | dispatches | fetch GB / launch | write GB / launch | total GB / launch |",
             "|---|---:|---:|---:|---:|"]
    for cls, k in t["kernels"].items():
        lines.append(f"| {cls} | {k['dispatches']} | {k['fetch_bytes'] / 1e9:.4f} | {k['write_bytes'] / 1e9:.4f} | "
                     f"{(k['fetch_bytes'] + k['write_bytes']) / 1e9:.4f} |")
    lines.append(f"\nkernel sources sha256: `{t['kernel_source_sha256']}`")
    return "\n".join(lines)


SIMDS = 1024
CLOCK_HZ = 2.4e9


def issue(sq_csv):
    """Per-dispatch averages of the SQ instruction counters for the three passes, with the hash of
    the kernel sources."""
    counters = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR")
    per = {c: per_kernel_counter(sq_csv, c) for c in counters}
    dur = {}
    for r in _rows(sq_csv):
        dur.setdefault(r["Kernel_Name"], {})[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    kernels = {}
    for cls, key in KERNEL_KEYS.items():
        ds = [d for k, dd in dur.items() if key in k for d in dd.values()]
        if not ds:
            continue
        avg = {}
        for c in counters:
            vals = [v for k, gvs in per[c].items() if key in k for _, v in gvs]
            avg[c] = sum(vals) / len(vals) if vals else float("nan")
        kernels[cls] = {"dispatches": len(ds), "counters": avg, "dispatch_ns": sum(ds) / len(ds),
                        "valu_issue_ns": avg["SQ_INSTS_VALU"] * 4 / SIMDS / CLOCK_HZ * 1e9}
    return {"kernel_source_sha256": kernel_source_hash(), "simds": SIMDS, "clock_hz": CLOCK_HZ, "kernels": kernels}


def issue_table(t):
    lines = ["| kernel | dispatches | waves | VALU / wave | SALU / wave | LDS / wave | VMEM rd / wave | "
             "VMEM wr / wave | VALU issue time | dispatch time (counter run) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for cls, k in t["kernels"].items():
        avg = k["counters"]
        waves = avg["SQ_WAVES"]
        lines.append(f"| {cls} | {k['dispatches']} | {waves:.0f} | {avg['SQ_INSTS_VALU'] / waves:.0f} | "
                     f"{avg['SQ_INSTS_SALU'] / waves:.0f} | {avg['SQ_INSTS_LDS'] / waves:.0f} | "
                     f"{avg['SQ_INSTS_VMEM_RD'] / waves:.1f} | {avg['SQ_INSTS_VMEM_WR'] / waves:.1f} | "
                     f"{k['valu_issue_ns'] / 1e6:.3f} ms | {k['dispatch_ns'] / 1e6:.3f} ms |")
    lines.append(f"\nkernel sources sha256: `{t['kernel_source_sha256']}`")
    return "\n".join(lines)


def trace_table(stats_csv):
    rows = _rows(stats_csv)
    lines = ["| kernel | calls | total ns | average ns | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:16]:
        name = r.get("Name", "")
        name = name if len(name) < 90 else name[:87] + "..."
        lines.append(f"| `{name}` | {r.get('Calls')} | {r.get('TotalDurationNs')} | "
                     f"{float(r.get('AverageNs', 0)):.0f} | {float(r.get('Percentage', 0)):.2f} |")
    return "\n".join(lines)


def overlap(trace_csv, window_s=0.5, dense=0.8):
    """Concurrency of the served requests in a `rocprofv3 --kernel-trace` file: kernels on the
    serving slots' streams (every stream but the default one), the time with kernels of k distinct
    streams in flight, over the whole trace and from the first window of `window_s` seconds that
    is busy more than `dense` of the time (the saturated replay, which submits every request at
    once)."""
    ev = []
    for r in _rows(trace_csv):
        if r["Stream_Id"] == "0":
            continue
        ev.append((int(r["Start_Timestamp"]), 1, r["Stream_Id"]))
        ev.append((int(r["End_Timestamp"]), -1, r["Stream_Id"]))
    ev.sort()
    active, last, spans = {}, None, []
    for t, d, st in ev:
        if last is not None and t > last:
            spans.append((last, t, sum(1 for v in active.values() if v > 0)))
        active[st] = active.get(st, 0) + d
        last = t

    def dist(t_from):
        out = {}
        for a, b, k in spans:
            if b > t_from:
                out[k] = out.get(k, 0) + (b - max(a, t_from))
        return out

    w = int(window_s * 1e9)
    busy_by_window = {}
    for a, b, k in spans:
        t = a
        while t < b:
            e = min(b, (t // w + 1) * w)
            if k >= 1:
                busy_by_window[t // w] = busy_by_window.get(t // w, 0) + (e - t)
            t = e
    dense_w = sorted(x for x, v in busy_by_window.items() if v > dense * w)
    res = {"all": dist(spans[0][0]) if spans else {}}
    if dense_w:
        res["saturated"] = dist(dense_w[0] * w)
        res["saturated_from_s"] = (dense_w[0] * w - spans[0][0]) / 1e9
    return res


def overlap_table(res):
    lines = ["| part | busy s | idle s | 1 request | 2 | 3 | 4 or more |", "|---|---:|---:|---:|---:|---:|---:|"]
    for part in ("all", "saturated"):
        d = res.get(part)
        if not d:
            continue
        busy = sum(v for k, v in d.items() if k >= 1)
        frac = lambda lo, hi=None: sum(v for k, v in d.items() if k >= lo and (hi is None or k <= hi)) / busy
        lines.append(f"| {part} | {busy / 1e9:.3f} | {d.get(0, 0) / 1e9:.3f} | {frac(1, 1):.3f} | {frac(2, 2):.3f} | "
                     f"{frac(3, 3):.3f} | {frac(4):.3f} |")
    return "\n".join(lines)


def main(argv):
    for a in [a for a in argv if a.startswith("--n=")]:
        set_grid_size(int(a[4:]))
        argv = [x for x in argv if x != a]
    if len(argv) >= 2 and argv[0] == "trace":
        table = trace_table(argv[1])
        if len(argv) > 2:
            with open(argv[2], "a") as fh:
                fh.write(table + "\n")
        print(table)
    elif len(argv) >= 3 and argv[0] == "issue":
        t = issue(argv[1])
        with open(argv[2], "w") as fh:
            json.dump(t, fh, indent=1)
            fh.write("\n")
        table = issue_table(t)
        if len(argv) > 3:
            with open(argv[3], "a") as fh:
                fh.write(table + "\n")
        print(table)
    elif len(argv) >= 2 and argv[0] == "overlap":
        print(overlap_table(overlap(argv[1])))
    elif len(argv) >= 4 and argv[0] == "traffic":
        t = traffic(argv[1], argv[2])
        with open(argv[3], "w") as fh:
            json.dump(t, fh, indent=1)
            fh.write("\n")
        table = traffic_table(t)
        if len(argv) > 4:
            with open(argv[4], "a") as fh:
                fh.write(table + "\n")
        print(table)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
