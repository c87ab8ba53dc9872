"""Summaries of rocprofv3 result databases (kernel trace and PMC counters).

  python -m paper_2006_05874_amd.profsum trace RESULTS.db [--kernel NAME]
  python -m paper_2006_05874_amd.profsum traffic FETCH.db WRITE.db --kernel NAME

``trace``: per-kernel dispatch count, total and mean duration.  For the kernel
named by --kernel it also reports the mean over the dispatches that did their
work: launches queued behind a raised status flag return at once (a few
microseconds) and are excluded by dropping dispatches shorter than 10% of that
kernel's longest one.

``--last N`` keeps only the kernel's last N dispatches (those of the timed region
when the program tunes or warms up before it).

``traffic``: FETCH_SIZE and WRITE_SIZE per dispatch (KiB), scaled by what the
same counters read for a plain device-to-device copy of 256 MiB recorded in the
same process (the rocclr copyBuffer dispatch with the largest WRITE_SIZE), for
the dispatches of --kernel that did their work (FETCH above 10% of the
kernel's maximum).
"""
import argparse
import collections
import re
import sqlite3

COPY_BYTES = 256 * 1024 * 1024


def short_name(name):
    m = re.match(r"(?:void )?(?:rs::)?([A-Za-z_0-9:]+)", name)
    s = m.group(1) if m else name
    t = re.search(r"<(.*)>", name)
    if t and "rs::" in name:
        s += "<" + t.group(1) + ">"
    return s


def trace_summary(db, kernel=None, last=None):
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end from kernels order by start").fetchall()
    agg = collections.defaultdict(list)
    for name, st, en in rows:
        agg[short_name(name)].append((en - st) / 1e3)  # us
    total = sum(sum(v) for v in agg.values())
    lines = [f"{'total_ms':>10s} {'share':>6s} {'calls':>7s} {'mean_us':>9s}  kernel"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{sum(v) / 1e3:10.3f} {100 * sum(v) / total:5.1f}% {len(v):7d} "
                     f"{sum(v) / len(v):9.2f}  {k}")
    out = {"lines": lines, "busy_ms": total / 1e3}
    if kernel:
        ds = [(en - st) / 1e3 for name, st, en in rows if short_name(name).startswith(kernel)]
        if last:
            ds = ds[-last:]
        if ds:
            cut = 0.1 * max(ds)
            work = [d for d in ds if d >= cut]
            out["kernel"] = {"name": kernel, "dispatches": len(ds), "working": len(work),
                             "mean_us_working": sum(work) / len(work)}
    return out


def _pmc(db, counter):
    c = sqlite3.connect(db)
    rows = c.execute("select name, counter_name, counter_value from pmc_events "
                     "where counter_name = ? order by dispatch_id", (counter,)).fetchall()
    return [(short_name(n), v) for n, _, v in rows]


def traffic_summary(fetch_db, write_db, kernel, last=None):
    f = _pmc(fetch_db, "FETCH_SIZE")
    w = _pmc(write_db, "WRITE_SIZE")
    copy_w = max(v for n, v in w if n.startswith("__amd_rocclr_copyBuffer"))
    # the copy dispatch with the largest write is the 256 MiB calibration copy
    copy_f = max(v for n, v in f if n.startswith("__amd_rocclr_copyBuffer"))
    f_scale = COPY_BYTES / (copy_f * 1024.0)
    w_scale = COPY_BYTES / (copy_w * 1024.0)
    kf = [v for n, v in f if n.startswith(kernel)]
    kw = [v for n, v in w if n.startswith(kernel)]
    if last:
        kf, kw = kf[-last:], kw[-last:]
    kf_work = [v for v in kf if v >= 0.1 * max(kf)]
    kw_work = sorted(kw)[-len(kf_work):] if kf_work else []
    fetch_b = sum(kf_work) / len(kf_work) * 1024.0 * f_scale
    write_b = sum(kw_work) / len(kw_work) * 1024.0 * w_scale
    return {"kernel": kernel, "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
            "fetch_scale": f_scale, "write_scale": w_scale, "working_dispatches": len(kf_work),
            "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
            "traffic_bytes_per_launch": fetch_b + write_b}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--kernel")
    t.add_argument("--last", type=int, default=None)
    tr = sub.add_parser("traffic")
    tr.add_argument("fetch_db")
    tr.add_argument("write_db")
    tr.add_argument("--kernel", required=True)
    tr.add_argument("--last", type=int, default=None)
    a = ap.parse_args()
    if a.cmd == "trace":
        out = trace_summary(a.db, a.kernel, a.last)
        print(f"busy_ms {out['busy_ms']:.3f}")
        if "kernel" in out:
            k = out["kernel"]
            print(f"kernel {k['name']}: dispatches {k['dispatches']}, working {k['working']}, "
                  f"mean_us_working {k['mean_us_working']:.2f}")
        print("\n".join(out["lines"]))
    else:
        out = traffic_summary(a.fetch_db, a.write_db, a.kernel, a.last)
        for k, v in out.items():
            print(f"{k}: {v}")


if __name__ == "__main__":
    main()
