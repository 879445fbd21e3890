"""Summaries of rocprofv3 runs for the profiles/ folder.

    python -m paper_2406_15632_amd.profile_report copy-probe [MiB]
        a plain device-to-device copy of a known size (calibrates FETCH_SIZE and
        WRITE_SIZE, which count in KiB of the memory side, against bytes moved);

    python -m paper_2406_15632_amd.profile_report trace DIR LAUNCHES OUT.md "COMMAND"
        per-kernel durations of a --kernel-trace --stats run, summed per
        transport launch (LAUNCHES = qrt_run calls in the profiled command);

    python -m paper_2406_15632_amd.profile_report traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR
        COPY_WRITE_DIR COPY_MIB LAUNCHES OUT.txt "COMMANDS"
        HBM bytes per transport launch from FETCH_SIZE and WRITE_SIZE, each
        scaled by the factor the same counter shows for the copy probe;

    python -m paper_2406_15632_amd.profile_report counters OUT.md "COMMANDS" DIR...
        L2 hit rate, VALU busy, VALU lane utilization, the share of wave
        time spent waiting and texture address / data busy, per transport
        kernel, from --pmc runs of TCC_HIT_sum TCC_MISS_sum, of
        SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAIT_INST_ANY
        SQ_WAVE_CYCLES GRBM_GUI_ACTIVE and of TA_TA_BUSY_sum TD_TD_BUSY_sum
        GRBM_GUI_ACTIVE;

    python -m paper_2406_15632_amd.profile_report trace-batch DIR RUNS OUT.md "COMMAND"
        per-kernel durations of the batched kernels (k_b*, sort steps of the
        batch) per batch run.
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import sqlite3
import sys


def _pmc_totals(d):
    tot = collections.defaultdict(lambda: collections.defaultdict(float))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            tot[r["Kernel_Name"].split("(")[0]][r["Counter_Name"]] += float(r["Counter_Value"])
    return tot


def _transport(name: str) -> bool:
    return "qrt::" in name


def copy_probe(mib: int = 1024):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB")


def _batch_kernel(name: str) -> bool:
    return "qrt::k_b" in name


def trace_summary(d: str, launches: int, out: str, command: str, select=_transport,
                  title: str = "transport kernels", unit: str = "transport launch (qrt_run calls)"):
    db = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)[0]
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average from top_kernels"))
    lines = [f"# rocprofv3 kernel trace: {title}", "", "Command:", "", "```", command, "```", "",
             f"Units of work ({unit}) in the run: {launches}", "",
             "| kernel | calls | total ms | avg us | ms per unit |", "|---|---|---|---|---|"]
    per_launch = 0.0
    for name, calls, total, avg in rows:   # the view reports microseconds
        if not select(name):
            continue
        short = name.split("(")[0].replace("void ", "")
        per = total / 1e3 / launches
        per_launch += per
        lines.append(f"| `{short}` | {calls} | {total / 1e3:.3f} | {avg:.2f} | {per:.3f} |")
    lines += ["", f"Sum of kernel time per unit: {per_launch:.3f} ms", ""]
    open(out, "w").write("\n".join(lines))
    print("\n".join(lines))


def _agent(d):
    """(XCDs, CUs) of the profiled GPU, from rocprofv3's agent table."""
    for f in glob.glob(os.path.join(d, "**", "*agent_info.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r.get("Name", "").startswith("gfx") and int(r.get("Cu_Count") or 0) > 0:
                return int(r["Num_Xcc"]), int(r["Cu_Count"])
    raise RuntimeError(f"no GPU agent in {d}")


def counters(out: str, commands: str, *dirs):
    """Per transport kernel, summed over its dispatches: L2 hit rate
    TCC_HIT / (TCC_HIT + TCC_MISS); VALU busy 100 SQ_ACTIVE_INST_VALU / (CUs
    cycles), the rocprofv3 VALUBusy definition; VALU lane utilization
    100 SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU); the share of wave
    cycles spent waiting on an instruction's inputs, SQ_WAIT_INST_ANY /
    SQ_WAVE_CYCLES; texture address (TA) and texture data (TD) busy,
    100 TA_TA_BUSY / (CUs cycles) and the same for TD_TD_BUSY.  The cycles of a
    dispatch are GRBM_GUI_ACTIVE of one XCD: the counter is reported summed
    over the XCDs, each of which counts the whole dispatch, so it is divided by
    their number.  Each ratio uses the cycles of the run that took its
    counters."""
    metrics = collections.defaultdict(dict)
    for d in dirs:
        n_xcc, cus = _agent(d)
        for k, v in _pmc_totals(d).items():
            if not _transport(k):
                continue
            cycles = max(1.0, v.get("GRBM_GUI_ACTIVE", 0.0) / n_xcc)
            m = metrics[k]
            if "TCC_HIT_sum" in v:
                m["hit"] = 100 * v["TCC_HIT_sum"] / max(1.0, v["TCC_HIT_sum"] + v["TCC_MISS_sum"])
            if "SQ_ACTIVE_INST_VALU" in v:
                m["busy"] = 100 * v["SQ_ACTIVE_INST_VALU"] / cus / cycles
                m["lanes"] = 100 * v["SQ_THREAD_CYCLES_VALU"] / max(1.0, 64 * v["SQ_ACTIVE_INST_VALU"])
                m["wait"] = 100 * v["SQ_WAIT_INST_ANY"] / max(1.0, v["SQ_WAVE_CYCLES"])
            if "TA_TA_BUSY_sum" in v:
                m["ta"] = 100 * v["TA_TA_BUSY_sum"] / cus / cycles
                m["td"] = 100 * v["TD_TD_BUSY_sum"] / cus / cycles
    lines = ["# rocprofv3 counters of the transport kernels (disk128)", "", "Commands:", "", "```", commands, "```",
             "", "| kernel | L2 hit % | VALU busy % | VALU lanes active % | wave cycles waiting % | TA busy % "
             "| TD busy % |", "|---|---|---|---|---|---|---|"]

    def f(m, key):
        return f"{m[key]:.1f}" if key in m else "-"
    for k in sorted(metrics):
        m = metrics[k]
        lines.append(f"| `{k.replace('void ', '')}` | {f(m, 'hit')} | {f(m, 'busy')} | {f(m, 'lanes')} | "
                     f"{f(m, 'wait')} | {f(m, 'ta')} | {f(m, 'td')} |")
    lines.append("")
    open(out, "w").write("\n".join(lines))
    print("\n".join(lines))


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib, launches, out, commands):
    from bench import transport_source_hash
    fetch = _pmc_totals(fetch_dir)
    write = _pmc_totals(write_dir)
    cf = _pmc_totals(cfetch_dir)
    cw = _pmc_totals(cwrite_dir)
    copy_bytes = float(copy_mib) * (1 << 20)

    def copy_counter(t, name):
        vals = [v[name] for k, v in t.items() if "copy" in k.lower() or "elementwise" in k.lower()]
        return max(vals) if vals else 0.0

    f_copy = copy_counter(cf, "FETCH_SIZE")
    w_copy = copy_counter(cw, "WRITE_SIZE")
    f_scale = copy_bytes / f_copy if f_copy else 0.0
    w_scale = copy_bytes / w_copy if w_copy else 0.0
    f_raw = sum(v["FETCH_SIZE"] for k, v in fetch.items() if _transport(k))
    w_raw = sum(v["WRITE_SIZE"] for k, v in write.items() if _transport(k))
    fetch_b = f_raw * f_scale / launches
    write_b = w_raw * w_scale / launches
    # the dominant kernels on their own, as the bench times them: every walk dispatch of a launch
    # (k_walk, k_walk_peel_lds) and the late-order launch k_tail
    walk = lambda k: "qrt::k_walk" in k or "qrt::k_tail<" in k   # noqa: E731
    wf = sum(v["FETCH_SIZE"] for k, v in fetch.items() if walk(k)) * f_scale / launches
    ww = sum(v["WRITE_SIZE"] for k, v in write.items() if walk(k)) * w_scale / launches
    lines = ["# HBM traffic of the transport step (disk128, 2^22 packets per launch)", "",
             "Commands:", "", "```", commands, "```", "",
             f"source_hash: {transport_source_hash()}",
             f"copy_probe_bytes: {copy_bytes:.0f}",
             f"copy_FETCH_SIZE: {f_copy:.6g}",
             f"copy_WRITE_SIZE: {w_copy:.6g}",
             f"fetch_scale_bytes_per_unit: {f_scale:.6g}",
             f"write_scale_bytes_per_unit: {w_scale:.6g}",
             f"launches: {launches}",
             f"transport_FETCH_SIZE_total: {f_raw:.6g}",
             f"transport_WRITE_SIZE_total: {w_raw:.6g}",
             f"fetch_bytes_per_launch: {fetch_b:.6g}",
             f"write_bytes_per_launch: {write_b:.6g}",
             f"bytes_per_step_launch: {fetch_b + write_b:.6g}",
             f"walk_fetch_bytes_per_launch: {wf:.6g}",
             f"walk_write_bytes_per_launch: {ww:.6g}",
             f"walk_bytes_per_launch: {wf + ww:.6g}", ""]
    lines += ["Per kernel (FETCH_SIZE, WRITE_SIZE raw totals):", ""]
    for k in sorted(set(fetch) | set(write)):
        if _transport(k):
            lines.append(f"- `{k}`: {fetch[k]['FETCH_SIZE']:.6g}, {write[k]['WRITE_SIZE']:.6g}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(path: str):
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "-", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    cmd = sys.argv[1]
    if cmd == "copy-probe":
        copy_probe(int(sys.argv[2]) if len(sys.argv) > 2 else 1024)
    elif cmd == "trace":
        trace_summary(sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5])
    elif cmd == "traffic":
        traffic(*sys.argv[2:6], float(sys.argv[6]), int(sys.argv[7]), sys.argv[8], sys.argv[9])
    elif cmd == "counters":
        counters(sys.argv[2], sys.argv[3], *sys.argv[4:])
    elif cmd == "trace-batch":
        trace_summary(sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5], select=_batch_kernel,
                      title="batched transport kernels (64 uneven scenes)", unit="batch runs (qrt_batch_run calls)")
