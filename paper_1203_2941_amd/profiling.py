"""rocprofv3 summaries for the profiles folder, and the measured HBM traffic
that bench.py reports beside its roofline.

Two summaries are written from rocprofv3 databases (``*_results.db``):

* ``trace``: per-kernel call count and durations from a ``--kernel-trace``
  run;
* ``traffic``: bytes that one transport launch moves between L2 and memory,
  from a ``--pmc FETCH_SIZE`` run and a ``--pmc WRITE_SIZE`` run of the same
  command. Each counter is scaled by what it reads for a plain elementwise
  copy of known size run first in the same process (``bench.py
  --calib-copy-mib``), so that the figure is in bytes whatever the counter's
  unit. The summary records a digest of the transport sources; bench.py
  reports the traffic only while the sources still match it.

Usage (from the repository root)::

    python -m paper_1203_2941_amd.profiling trace DB TITLE COMMAND > profiles/x.md
    python -m paper_1203_2941_amd.profiling traffic FETCH_DB WRITE_DB CALIB_MIB COMMAND > profiles/y.md
    python -m paper_1203_2941_amd.profiling rt-traffic FETCH_DB WRITE_DB CALIB_MIB COMMAND > profiles/z.md
"""
from __future__ import annotations

import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TRANSPORT_SOURCES = ("csrc/mcrt_transport.hip", "csrc/mcrt_internal.h", "csrc/mcrt_api.hip",
                     "csrc/mcrt_scatter.h")
RT_SOURCES = ("csrc/mcrt_raytrace.hip", "csrc/mcrt_rtargs.h", "csrc/mcrt_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_wf_walk_torus256_1e8_traffic.md")
RT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "raytrace_torus256_512px_traffic.md")
RT_KERNELS = ("k_build_S", "k_rt_fwd", "k_rt_adj")
TRANSPORT_KERNEL = "k_wf_walk<float, false, true, false, false>"
CALIB_KERNEL = "MulFunctor"


def source_digest(sources=TRANSPORT_SOURCES) -> str:
    """sha256 over the sources of the transport kernels and their round loop
    (or of another kernel group)."""
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_table(db: str):
    """(name, calls, total ns, mean ns) per kernel, longest total first."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end - start), avg(end - start) "
                       "from kernels group by name order by sum(end - start) desc").fetchall()
    con.close()
    return rows


def counter_values(db: str, counter: str, kernel_like: str):
    """Per-dispatch values of one counter for kernels whose name contains kernel_like."""
    con = sqlite3.connect(db)
    rows = con.execute("select value from counters_collection where counter_name = ? and "
                       "kernel_name like ? order by dispatch_id",
                       (counter, f"%{kernel_like}%")).fetchall()
    con.close()
    return [float(r[0]) for r in rows]


def trace_md(db: str, title: str, cmd: str) -> str:
    rows = kernel_table(db)
    tot = sum(r[2] for r in rows) or 1
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", cmd,
           "```", "", "| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, n, s, a in rows:
        short = name if len(name) < 90 else name[:87] + "..."
        out.append(f"| `{short}` | {n} | {s / 1e6:.3f} | {a / 1e6:.3f} | {100 * s / tot:.2f} |")
    return "\n".join(out) + "\n"


def traffic_md(fetch_db: str, write_db: str, calib_mib: int, cmd: str) -> str:
    cal_f = counter_values(fetch_db, "FETCH_SIZE", CALIB_KERNEL)
    cal_w = counter_values(write_db, "WRITE_SIZE", CALIB_KERNEL)
    fetch = counter_values(fetch_db, "FETCH_SIZE", TRANSPORT_KERNEL)
    write = counter_values(write_db, "WRITE_SIZE", TRANSPORT_KERNEL)
    if not (cal_f and cal_w and fetch and write):
        raise SystemExit("counters missing from the databases")
    nbytes = calib_mib * (1 << 20)
    sf = nbytes / cal_f[0]   # bytes per counter unit, read side
    sw = nbytes / cal_w[0]   # write side
    # the two runs are separate processes and need not take the same number
    # of rounds: each side is summed over its own run's launches
    rd, wr = sum(fetch) * sf, sum(write) * sw
    per_launch = rd / len(fetch) + wr / len(write)
    launches = 0.5 * (len(fetch) + len(write))
    lines = [
        "# HBM traffic of the walk kernel: 256^3 clumpy torus, 1e8 packets, FP32",
        "",
        "Two counter runs of one bench step each (all walk launches of the source",
        "and PAH runs), FETCH_SIZE and WRITE_SIZE in separate runs. A",
        f"{calib_mib} MiB elementwise copy in the same process calibrates each counter:",
        f"it read {cal_f[0]:.6g} FETCH_SIZE units and wrote {cal_w[0]:.6g} WRITE_SIZE",
        f"units, so one unit is {sf:.6g} B read / {sw:.6g} B written.",
        "",
        "Commands (from the repository root, one MI355X; R = repository root):",
        "",
        "```",
        cmd,
        "```",
        "",
        "| run | walk launches | counter sum | bytes | bytes per launch |",
        "|---|---:|---:|---:|---:|",
        f"| FETCH_SIZE | {len(fetch)} | {sum(fetch):.6g} | {rd:.6g} | {rd / len(fetch):.6g} |",
        f"| WRITE_SIZE | {len(write)} | {sum(write):.6g} | {wr:.6g} | {wr / len(write):.6g} |",
        "",
        f"traffic_bytes_per_launch: {per_launch:.6g}",
        f"traffic_bytes_per_step: {per_launch * launches:.6g}",
        f"launches_per_step: {launches:g}",
        f"source_sha256: {source_digest()}",
        "",
    ]
    return "\n".join(lines)


def read_traffic(path: str = TRAFFIC_FILE):
    """Measured bytes of the walk kernel, {"per_launch": B, "per_step": B}
    (a step being all launches of one bench step), or None when the summary
    is missing or was taken from other transport sources."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    pl = re.search(r"^traffic_bytes_per_launch: (\S+)$", text, re.M)
    ps = re.search(r"^traffic_bytes_per_step: (\S+)$", text, re.M)
    d = re.search(r"^source_sha256: (\S+)$", text, re.M)
    if not pl or not ps or not d or d.group(1) != source_digest():
        return None
    return {"per_launch": float(pl.group(1)), "per_step": float(ps.group(1))}


def rt_traffic_md(fetch_db: str, write_db: str, calib_mib: int, cmd: str) -> str:
    """Bytes per launch of the ray-tracer kernels (source functions, forward,
    adjoint) from a FETCH_SIZE run and a WRITE_SIZE run, calibrated as in
    traffic_md."""
    cal_f = counter_values(fetch_db, "FETCH_SIZE", CALIB_KERNEL)
    cal_w = counter_values(write_db, "WRITE_SIZE", CALIB_KERNEL)
    if not (cal_f and cal_w):
        raise SystemExit("calibration counters missing from the databases")
    nbytes = calib_mib * (1 << 20)
    sf, sw = nbytes / cal_f[0], nbytes / cal_w[0]
    lines = [
        "# HBM traffic of the ray-tracer kernels: 256^3 torus, 512^2 px, 16 wavelengths, 8 views, FP32",
        "",
        "FETCH_SIZE and WRITE_SIZE in separate runs of one bench step each; a",
        f"{calib_mib} MiB elementwise copy in the same process calibrates each counter",
        f"(one unit = {sf:.6g} B read / {sw:.6g} B written).",
        "",
        "Commands (from the repository root, one MI355X; R = repository root):",
        "",
        "```",
        cmd,
        "```",
        "",
        "| kernel | launches | read bytes per launch | written bytes per launch | total per launch |",
        "|---|---:|---:|---:|---:|",
    ]
    vals = {}
    for k in RT_KERNELS:
        f = counter_values(fetch_db, "FETCH_SIZE", k + "<")
        w = counter_values(write_db, "WRITE_SIZE", k + "<")
        if not f or not w:
            continue
        rd, wr = sum(f) * sf / len(f), sum(w) * sw / len(w)
        vals[k] = rd + wr
        lines.append(f"| `{k}` | {len(f)} | {rd:.6g} | {wr:.6g} | {rd + wr:.6g} |")
    lines.append("")
    for k, v in vals.items():
        lines.append(f"traffic_{k}: {v:.6g}")
    lines.append(f"source_sha256: {source_digest(RT_SOURCES)}")
    lines.append("")
    return "\n".join(lines)


def read_rt_traffic(path: str = RT_TRAFFIC_FILE):
    """{kernel: measured bytes per launch} of the ray-tracer kernels, or None
    when the summary is missing or was taken from other sources."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    d = re.search(r"^source_sha256: (\S+)$", text, re.M)
    if not d or d.group(1) != source_digest(RT_SOURCES):
        return None
    return {m.group(1): float(m.group(2))
            for m in re.finditer(r"^traffic_(\w+): (\S+)$", text, re.M)}


def main(argv):
    if len(argv) >= 4 and argv[0] == "trace":
        sys.stdout.write(trace_md(argv[1], argv[2], argv[3]))
    elif len(argv) >= 5 and argv[0] == "traffic":
        sys.stdout.write(traffic_md(argv[1], argv[2], int(argv[3]), argv[4]))
    elif len(argv) >= 5 and argv[0] == "rt-traffic":
        sys.stdout.write(rt_traffic_md(argv[1], argv[2], int(argv[3]), argv[4]))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
