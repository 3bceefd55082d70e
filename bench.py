"""Benchmark: phase-space cell-updates per second per split step on one GPU.

Default workload: the 4096 x 4096 large-grid case (FP32 delta f, degree 17,
dt = 0.02), the configuration the metric is quoted on.  One "step" is one
full Strang step: v-sweep (dt/2), x-sweep (dt) on the v-fastest layout with
the velocity row sums of rho, FP64 field solve, v-sweep (dt/2).  The timed
region holds exactly --steps steps, bracketed by device synchronisation.  A
second pass of the same number of steps records HIP events on the sim's
stream around every kernel launch; they give each kernel's average duration
for the roofline.

Prints one JSON line with the headline FP32 delta-f rate, the FP64 plain
rate on the same GPU, the roofline of the dominant kernel (with the HBM bytes
rocprofv3 counted, when the committed measurement matches the current kernel
sources), the achievable device-copy bandwidth, a batch of 16 large-grid sims
(1 GiB of f, larger than the 256 MB Infinity Cache), the CPU-oracle baseline
and (unless --no-serving) the serving-mix latency summary.

`--summarize-rocprof DIR` instead turns the CSV output of the three rocprofv3
runs listed in PROFILE_COMMANDS into the text summaries under profiles/ and
the per-launch HBM traffic table profiles/traffic.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, 8 TB/s
FP32_VALU_PEAK_TFLOPS = 78.6    # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, no packed FP32
FP64_VALU_PEAK_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="large_grid")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-fp64-deltaf", action="store_true",
                   help="skip the FP64 delta-f leg (it shares kernels with FP64 plain, so the "
                        "profiling runs leave it out)")
    p.add_argument("--no-keen", action="store_true",
                   help="skip the KEEN 4096x4096 leg (the paper's timed workload)")
    p.add_argument("--no-merged", action="store_true",
                   help="skip the merged-v-half-step FP32 leg")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="oracle time on the headline workload (all threads); the one-thread "
                        "and other-workload samples take about 0.8 of that again")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--serving-requests", type=int, default=512)
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one plain 256 MiB device-to-device copy first (a known-size "
                        "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    p.add_argument("--dram-sims", type=int, default=16,
                   help="sims of the workload stepped together through vog_step_batch "
                        "(16 large-grid FP32 sims hold 1 GiB of f); 0 skips this leg")
    p.add_argument("--summarize-rocprof", metavar="DIR", default=None,
                   help="write profiles/ summaries from the rocprofv3 CSV output under DIR "
                        "(subfolders kt/, fetch/, write/, valu/ and kt.log, as in PROFILE_COMMANDS)")
    return p.parse_args()


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and blank lines removed, so
    that an edit of the comments alone keeps a counter measurement valid."""
    import re
    h = hashlib.sha256()
    for name in ("addr.hpp", "fft.hpp", "pair4096.hpp", "kernels.hpp", "sweep_f32.hip", "sweep_f64.hip",
                 "xsweep.hip", "mixed.hip", "field.hip", "misc.hip", "vog_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1301_5892_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def stored_traffic(kind: str, workload: str, precision: str):
    """HBM traffic per launch measured with rocprofv3 counters, if the
    committed measurement was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    key = f"{kind}/{workload}/{precision}"
    e = rec.get(key)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def run_dram(w, nsims, steps, warmup):
    """nsims independent FP32 delta-f sims of the workload advanced together
    by vog_step_batch: a working set several times the Infinity Cache, so
    the rate has to hold from HBM."""
    import torch
    from paper_1301_5892_amd import vog

    sims = [vog.Sim(w, precision="fp32_deltaf").init() for _ in range(nsims)]
    vog.step_batch(sims, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vog.step_batch(sims, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    finite = True
    for sm in sims:
        d = sm.diag()
        finite = finite and bool(d.size == 0 or d["finite"][-1] == 1)
    out = {"sims": nsims, "f_bytes": nsims * w.cells * 4, "steps": steps,
           "value": nsims * w.cells * steps / el, "unit": "cell-updates/s",
           "ms_per_step": el / steps * 1e3, "finite": finite}
    out["algorithmic_gbs"] = out["value"] * 24 / 1e9
    for sm in sims:
        sm.close()
    return out


def copy_bandwidth(nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth: a plain device-to-device copy of nbytes
    (read + write counted), best of reps."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    del src, dst
    return 2 * nbytes / best / 1e9


def run_gpu(w, precision, steps, warmup):
    """Times `steps` Strang steps twice on one sim: first plain (the headline
    rate), then with HIP events recorded around every launch (per-kernel
    average durations for the roofline)."""
    import torch
    from paper_1301_5892_amd import vog

    sim = vog.Sim(w, precision=precision).init()
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    prof = sim.profile_read()
    sim.profile(False)
    d = sim.diag()
    finite = bool(d.size == 0 or d["finite"][-1] == 1)
    sim.close()
    return elapsed, prof, finite, elapsed_prof


def roofline_for(w, precision, prof, steps):
    """Dominant kernel: the kernel kind with the largest summed time."""
    es = 4 if precision == "fp32_deltaf" else 8
    kind = max(prof, key=lambda k: prof[k][0])
    ms, n = prof[kind]
    avg_s = ms / 1e3 / max(n, 1)
    cells = w.nx * w.nv
    line = {"sweep_v": w.nv, "sweep_vv": w.nv, "sweep_x": w.nx}.get(kind)
    # Algorithmic bytes: a sweep reads and writes f once (a transpose also
    # moves f once each way: not algorithmic for the method, reported as is).
    # A sweep_vv launch carries two v half-steps (the closing one of a step
    # and the opening one of the next), so two sweeps' worth, while it moves
    # f once each way itself.
    sweeps = 2 if kind == "sweep_vv" else 1
    bytes_per_launch = sweeps * 2 * es * cells
    hbm = {"bound": "hbm", "achieved": bytes_per_launch / avg_s / 1e9, "peak": HBM_PEAK_GBS,
           "unit": "GB/s"}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    hbm["traffic"] = stored_traffic(kind, w.name, precision)
    hbm["kernel"] = kind
    hbm["avg_launch_ms"] = avg_s * 1e3
    hbm["launches"] = n
    hbm["bytes_per_launch"] = bytes_per_launch
    hbm["sweeps_per_launch"] = sweeps
    if line:
        # The paper's real-data operation count per advected element,
        # 5 log2(N) + 3 (FFT pair plus complex multiply).
        flops = sweeps * (5 * math.log2(line) + 3) * cells
        peak = FP32_VALU_PEAK_TFLOPS if es == 4 else FP64_VALU_PEAK_TFLOPS
        ach = flops / avg_s / 1e12
        hbm["alu_view"] = {"achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                           "flops_per_launch": flops}
    return hbm


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, seconds, max_steps=1000):
    """Cell-updates/s of the FP64 oracle on w (delta-f form for delta-f
    precisions): whole Strang steps from f0 until `seconds` have passed."""
    import oracle
    o = oracle.Oracle(w, deltaf=w.precision.endswith("deltaf")).init()
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= max_steps:
            break
    return w.cells * steps / el, steps, el, o.deltaf


def cpu_baseline(w, seconds):
    """The oracle (plain C, FP64, OpenMP over lines) timed on the host: the
    headline workload on all threads for about `seconds`, the same on one
    thread, and the strong-Landau and bump-on-tail workloads truncated to a
    few seconds each (per-step cost is constant, so a truncated run gives the
    rate)."""
    import oracle
    import workloads
    threads = oracle.num_threads()
    rate, steps, el, df = _oracle_rate(w, seconds)
    out = {"value": rate, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{w.name}, {'delta-f' if df else 'plain'} FP64 direct-stencil oracle, "
                     f"{steps} Strang steps from f0 ({el:.1f} s, {threads} threads)"}
    oracle.set_num_threads(1)
    try:
        r1, s1, e1, _ = _oracle_rate(w, seconds / 3)
    finally:
        oracle.set_num_threads(threads)
    out["one_thread"] = {"value": r1, "sample": f"{w.name}, {s1} steps ({e1:.1f} s, 1 thread)"}
    other = {}
    for wo in (workloads.landau_strong(), workloads.bump_on_tail()):
        ro, so, eo, _ = _oracle_rate(wo, seconds / 5)
        other[wo.name] = {"value": ro, "sample": f"{so} of {wo.nsteps} steps ({eo:.1f} s, {threads} threads)"}
    out["other_workloads"] = other
    return out


# ---------------------------------------------------------------- rocprofv3 summaries
# The three profiling runs the committed summaries come from, run from /tmp
# with TMPDIR=/tmp ({out}: output folder, {root}: repository root).  The
# kernel trace times the same bench command as the headline (fewer steps, the
# batched leg off so that every launch of a kernel has the workload's shape);
# the two counter runs add one 256 MiB device copy as the known-size kernel
# that scales FETCH_SIZE and WRITE_SIZE to bytes.
PROFILE_COMMANDS = {
    "kt": "rocprofv3 --kernel-trace --stats -f csv -d {out}/kt -o kt -- python3 {root}/bench.py "
          "--steps 100 --warmup 10 --no-serving --no-cpu-baseline --dram-sims 0 --no-merged --no-keen --no-fp64-deltaf > {out}/kt.log",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d {out}/fetch -o fetch -- python3 {root}/bench.py "
             "--steps 2 --warmup 1 --no-serving --no-cpu-baseline --dram-sims 0 --no-merged --no-keen --no-fp64-deltaf --copy-calibration",
    "write": "rocprofv3 --pmc WRITE_SIZE -f csv -d {out}/write -o write -- python3 {root}/bench.py "
             "--steps 2 --warmup 1 --no-serving --no-cpu-baseline --dram-sims 0 --no-merged --no-keen --no-fp64-deltaf --copy-calibration",
    "valu": "rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CU_CYCLES SQ_WAVE_CYCLES "
            "SQ_INSTS_LDS SQ_WAIT_INST_LDS -f csv -d {out}/valu -o valu -- python3 {root}/bench.py "
            "--steps 2 --warmup 1 --no-serving --no-cpu-baseline --dram-sims 0 --no-merged --no-keen --no-fp64-deltaf --copy-calibration",
}
COPY_CALIBRATION_BYTES = 256 << 20


def classify_kernel(name):
    """(kind, precision) of a libvog kernel name as the bench labels them;
    ("copy", None) for the runtime's copy kernel; None for anything else."""
    if "copyBuffer" in name:
        return ("copy", None)
    if "vog::" not in name:
        return None
    prec = "fp32_deltaf" if "<float" in name else ("fp64_plain" if "<double" in name else None)
    if "xsweep_fused_kernel" in name:
        return ("sweep_x", prec)
    if "sweep_kernel" in name:
        tail = name.split("(")[0].rstrip()
        return ({", 1>": "sweep_x", ", 2>": "sweep_vv", ", 3>": "sweep_vv"}.get(tail[-4:], "sweep_v"), prec)
    if "transpose_kernel" in name:
        return ("transpose", prec)
    if "rho_reduce_kernel" in name:
        return ("rho_reduce", prec)
    if "rho_v_kernel" in name:  # rho straight from f: initial state, vog_sweep field recompute
        return ("rho_v", prec)
    if "field_kernel" in name:
        return ("field", None)
    if "moments" in name:
        return ("moments", prec)
    return None


def _csv_rows(folder, suffix):
    import csv
    import glob
    paths = sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {folder}")
    rows = []
    for pth in paths:
        with open(pth, newline="") as fh:
            rows.extend({k.strip().lower(): v for k, v in r.items()} for r in csv.DictReader(fh))
    return rows


def _labelled(rows):
    """(row, kind, precision) for the libvog and copy dispatches among rows,
    in dispatch order.  Kernels whose name does not carry the storage
    precision (the partial-row reduce, the field solve) take that of the
    sweep launched before them: the bench runs one sim at a time."""
    out, last = [], None
    for r in sorted(rows, key=lambda r: int(r["dispatch_id"])):
        c = classify_kernel(r["kernel_name"])
        if c is None:
            continue
        kind, prec = c
        if kind != "copy":
            if prec in ("fp32_deltaf", "fp64_plain"):
                last = prec
            else:
                prec = last
        out.append((r, kind, prec))
    return out


def _counter_per_kernel(folder, counter=None):
    """(kernel name, kind, precision) -> list of per-dispatch values of one
    counter (all rows when the file holds a single counter)."""
    rows = [r for r in _csv_rows(folder, "counter_collection.csv")
            if counter is None or r["counter_name"] == counter]
    out = {}
    for r, kind, prec in _labelled(rows):
        out.setdefault((r["kernel_name"], kind, prec), []).append(float(r["counter_value"]))
    return out


def _last_json(path):
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{"):
                try:
                    rec = json.loads(line)
                except ValueError:
                    pass
    return rec


def summarize_rocprof(folder, wname):
    """Write profiles/kernel_trace_<workload>.md, profiles/hbm_traffic_<workload>.md
    and profiles/traffic.json from the output of PROFILE_COMMANDS."""
    prof_dir = os.path.join(ROOT, "profiles")
    os.makedirs(prof_dir, exist_ok=True)
    cmds = {k: v.format(out="$OUT", root="$REPO") for k, v in PROFILE_COMMANDS.items()}
    bench_rec = _last_json(os.path.join(folder, "kt.log"))

    # kernel trace statistics, per kernel and storage precision of the sim
    trace = _labelled(_csv_rows(os.path.join(folder, "kt"), "kernel_trace.csv"))
    lines = [f"# Kernel trace, {wname}", "",
             "Command (from /tmp, TMPDIR=/tmp; $REPO is the repository root, $OUT the output "
             "folder):", "", "```", cmds["kt"], "```", "",
             "Per-dispatch durations from the trace; precision is that of the sim (the field "
             "solve computes in FP64 for both).", "",
             "| kernel | kind | precision | calls | avg us | min us | max us | % time |",
             "|---|---|---|---|---|---|---|---|"]
    groups = {}
    for r, kind, prec in trace:
        dur = (int(r["end_timestamp"]) - int(r["start_timestamp"])) / 1e3
        groups.setdefault((r["kernel_name"].split("(")[0], kind, prec), []).append(dur)
    total = sum(sum(v) for v in groups.values()) or 1.0
    trace_avg = {}
    for (name, kind, prec), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        avg = sum(d) / len(d)
        if kind != "copy":
            trace_avg[(kind, prec)] = avg
        lines.append(f"| `{name}` | {kind} | {prec or '-'} | {len(d)} | {avg:.2f} | {min(d):.2f} | "
                     f"{max(d):.2f} | {100 * sum(d) / total:.1f} |")
    if bench_rec:
        lines += ["", "HIP-event averages the bench printed in the same run (ms per launch):", ""]
        for label, rf in (("fp32_deltaf", bench_rec.get("roofline")),
                          ("fp64_plain", (bench_rec.get("fp64_plain") or {}).get("roofline"))):
            if rf:
                tr = trace_avg.get((rf["kernel"], label))
                lines.append(f"- {label} {rf['kernel']}: events {rf['avg_launch_ms'] * 1e3:.2f} us, "
                             f"trace {tr:.2f} us" if tr else
                             f"- {label} {rf['kernel']}: events {rf['avg_launch_ms'] * 1e3:.2f} us")
        lines.append(f"- headline ms/step (no events): {bench_rec['ms_per_step']:.4f}")
    with open(os.path.join(prof_dir, f"kernel_trace_{wname}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    # HBM traffic from FETCH_SIZE / WRITE_SIZE, scaled by the copy kernel
    fetch = _counter_per_kernel(os.path.join(folder, "fetch"))
    write = _counter_per_kernel(os.path.join(folder, "write"))
    cal_kib = COPY_CALIBRATION_BYTES / 1024.0
    copy_f = max((max(v) for k, v in fetch.items() if k[1] == "copy"), default=None)
    copy_w = max((max(v) for k, v in write.items() if k[1] == "copy"), default=None)
    if not copy_f or not copy_w:
        raise SystemExit("no copy kernel in the counter output")
    kf, kw = cal_kib / copy_f, cal_kib / copy_w
    src_hash = kernel_source_hash()
    table_path = os.path.join(prof_dir, "traffic.json")
    table = {}
    if os.path.exists(table_path):
        with open(table_path) as fh:
            table = json.load(fh)
    lines = [f"# HBM traffic per launch, {wname}", "",
             "Commands (from /tmp, TMPDIR=/tmp; $REPO is the repository root, $OUT the output "
             "folder):", "", "```", cmds["fetch"], cmds["write"], "```", "",
             f"Calibration: one {COPY_CALIBRATION_BYTES >> 20} MiB device-to-device copy "
             f"(`__amd_rocclr_copyBuffer`) reads FETCH_SIZE = {copy_f:.0f} KiB and "
             f"WRITE_SIZE = {copy_w:.0f} KiB against {cal_kib:.0f} KiB moved each way, so the "
             f"counters are scaled by {kf:.4f} (fetch) and {kw:.4f} (write).  FETCH_SIZE counts "
             f"L2 misses sent to the fabric, so Infinity Cache hits are included.", "",
             f"Kernel sources hash: `{src_hash}`", "",
             "| kernel | kind | precision | dispatches | FETCH KiB | WRITE KiB | scaled MB read | "
             "scaled MB written | algorithmic MB |", "|---|---|---|---|---|---|---|---|---|"]
    es = {"fp32_deltaf": 4, "fp64_plain": 8}
    import workloads
    wl = {x.name: x for x in workloads.all_named()}.get(wname)
    per_launch = {}
    for key in sorted(set(fetch) & set(write), key=lambda k: (str(k[2]), k[1], k[0])):
        name, kind, prec = key
        if kind == "copy":
            continue
        f_avg = sum(fetch[key]) / len(fetch[key])
        w_avg = sum(write[key]) / len(write[key])
        rd, wr = f_avg * 1024 * kf, w_avg * 1024 * kw
        alg = None
        if wl and prec in es:
            # a sweep reads and writes f once; the other kernels' bytes are
            # overhead on top of the step's algorithmic traffic
            alg = {"sweep_v": 2, "sweep_x": 2, "sweep_vv": 4}.get(kind, 0) * es[prec] * wl.cells or None
        lines.append(f"| `{name.split('(')[0]}` | {kind} | {prec or '-'} | {len(fetch[key])} | "
                     f"{f_avg:.0f} | {w_avg:.0f} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | "
                     f"{'-' if alg is None else f'{alg / 1e6:.2f}'} |")
        if prec in es:
            per_launch[(kind, prec)] = rd + wr
            table[f"{kind}/{wname}/{prec}"] = {
                "kernel": name.split("(")[0], "kernel_source_hash": src_hash,
                "fetch_bytes": rd, "write_bytes": wr, "bytes_per_launch": rd + wr,
                "fetch_scale": kf, "write_scale": kw}
    if wl:
        lines += ["", "Per Strang step inside a multi-step call (steady state: the two v half-steps "
                  "between steps in one launch where there is one, else two v-sweeps; one x-sweep, "
                  "the partial-row reduce and the field solve) against the algorithmic "
                  "3 x (read + write of f):", ""]
        for prec, e in es.items():
            kinds = {k: v for (k, p), v in per_launch.items() if p == prec}
            if "sweep_x" not in kinds or not ({"sweep_v", "sweep_vv"} & set(kinds)):
                continue
            per_step = {"sweep_x": 1, "transpose": 2, "rho_reduce": 1, "field": 1}
            per_step.update({"sweep_vv": 1} if "sweep_vv" in kinds else {"sweep_v": 2})
            step = sum(per_step.get(k, 0) * v for k, v in kinds.items())
            alg = 6 * e * wl.cells
            lines.append(f"- {prec}: {step / 1e6:.1f} MB measured, {alg / 1e6:.1f} MB algorithmic "
                         f"({6 * e} B per cell): {step / alg:.3f}x")
    with open(os.path.join(prof_dir, f"hbm_traffic_{wname}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(table_path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)

    # VALU issue: SQ_ACTIVE_INST_VALU counts one per wave64 VALU instruction
    # (4 cycles of a 16-lane SIMD) and SQ_BUSY_CU_CYCLES counts cycles summed
    # over CUs; a CU's 4 SIMDs issue at most one wave instruction per cycle
    # between them, so ACTIVE_INST_VALU / BUSY_CU_CYCLES is the VALU busy
    # fraction.
    vdir = os.path.join(folder, "valu")
    if os.path.isdir(vdir):
        names = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CU_CYCLES", "SQ_WAVE_CYCLES",
                 "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS")
        per = {n: _counter_per_kernel(vdir, n) for n in names}
        lines = [f"# VALU issue per kernel, {wname}", "",
                 "Command (from /tmp, TMPDIR=/tmp; $REPO is the repository root, $OUT the output "
                 "folder):", "",
                 "```", cmds["valu"], "```", "",
                 "Averages per dispatch.  VALU busy = SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES: one "
                 "count per wave64 VALU instruction (4 cycles of a 16-lane SIMD) against CU cycles, "
                 "4 SIMDs per CU.", "",
                 "| kernel | kind | precision | VALU instr (wave) | VALU busy | LDS instr (wave) | "
                 "LDS wait / wave-cycles |", "|---|---|---|---|---|---|---|"]
        for key in sorted(per["SQ_INSTS_VALU"], key=lambda k: (str(k[2]), k[1], k[0])):
            name, kind, prec = key
            if kind == "copy":
                continue
            avg = {n: (sum(per[n].get(key, [0])) / max(len(per[n].get(key, [])), 1)) for n in names}
            busy = avg["SQ_ACTIVE_INST_VALU"] / max(avg["SQ_BUSY_CU_CYCLES"], 1)
            ldsw = avg["SQ_WAIT_INST_LDS"] / max(avg["SQ_WAVE_CYCLES"], 1)
            lines.append(f"| `{name.split('(')[0]}` | {kind} | {prec or '-'} | "
                         f"{avg['SQ_INSTS_VALU']:.3g} | {busy:.2f} | {avg['SQ_INSTS_LDS']:.3g} | "
                         f"{ldsw:.3f} |")
        with open(os.path.join(prof_dir, f"valu_{wname}.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print(f"wrote profiles/kernel_trace_{wname}.md, profiles/hbm_traffic_{wname}.md, "
          f"profiles/traffic.json and (with valu/) profiles/valu_{wname}.md")


def main():
    args = parse()
    if args.summarize_rocprof:
        import workloads
        summarize_rocprof(args.summarize_rocprof, getattr(workloads, args.workload)().name)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): a simulation runs on one "
              f"GPU, and independent simulations shard one per GPU", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_1301_5892_amd import vog

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    vog.load()
    w = getattr(workloads, args.workload)()
    K, W = args.steps, args.warmup
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    el32, prof32, fin32, el32p = run_gpu(w, "fp32_deltaf", K, W)
    value = w.cells * K / el32
    out = {
        "metric": "phase-space cell-updates/s per split step, FP32-δf vs FP64; p99 req latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el32 / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "nv": w.nv, "precision": "fp32_deltaf",
                   "degree": w.degree, "dt": w.dt, "L": w.L, "vmin": w.vmin, "vmax": w.vmax},
        "finite": fin32,
        "ms_per_step_with_kernel_events": el32p / K * 1e3,
        "kernels_ms_per_step": {k: v[0] / K for k, v in prof32.items()},
        "roofline": roofline_for(w, "fp32_deltaf", prof32, K),
        "paper_context": {"value": 2.047e8, "unit": "cell-updates/s",
                          "hardware": "NVIDIA Tesla C2070 (Fermi)",
                          "note": "Table 1, N = 4096, FP32 delta f, KEEN workload; context only"},
        "build": vog.build_info(),
    }
    if not args.copy_calibration:
        # (counter runs keep the calibration copy the only large copy kernel)
        out["roofline"]["achievable_copy_gbs"] = copy_bandwidth()
    if not args.no_fp64:
        el64, prof64, fin64, el64p = run_gpu(w, "fp64_plain", K, W)
        out["fp64_plain"] = {"value": w.cells * K / el64, "ms_per_step": el64 / K * 1e3,
                             "ms_per_step_with_kernel_events": el64p / K * 1e3,
                             "finite": fin64,
                             "kernels_ms_per_step": {k: v[0] / K for k, v in prof64.items()},
                             "roofline": roofline_for(w, "fp64_plain", prof64, K)}
        out["fp32_over_fp64"] = out["value"] / out["fp64_plain"]["value"]
    if not args.no_fp64 and not args.no_fp64_deltaf:
        # FP64 delta f (optional in the comparison): the same grid, f - f_eq
        # stored in FP64
        el64d, _, fin64d, _ = run_gpu(w, "fp64_deltaf", K, W)
        out["fp64_deltaf"] = {"value": w.cells * K / el64d, "ms_per_step": el64d / K * 1e3,
                              "finite": fin64d}
    if not args.no_keen:
        # The paper's timed workload (Section 4.3, Table 1): KEEN waves at
        # N = 4096, FP32 delta f, drive on; its C2070 figure is quoted as is.
        wk = workloads.keen(4096, 0.05, K)
        elk, _, fink, _ = run_gpu(wk, "fp32_deltaf", K, W)
        out["keen_4096"] = {"value": wk.cells * K / elk, "unit": "cell-updates/s",
                            "ms_per_step": elk / K * 1e3, "finite": fink,
                            "paper_c2070": 2.047e8,
                            "vs_paper_c2070": wk.cells * K / elk / 2.047e8}
    if not args.no_merged:
        # Opt-in variant: v half-steps of consecutive steps merged (2 sweeps per
        # step), all --steps steps in one call.  Not the headline scheme.
        elm, _, finm, _ = run_gpu(w.replace(merge_v=True), "fp32_deltaf", K, W)
        out["fp32_deltaf_merged_v"] = {"value": w.cells * K / elm, "ms_per_step": elm / K * 1e3,
                                       "finite": finm}
    if args.dram_sims > 0:
        out["dram_batch"] = run_dram(w, args.dram_sims, K, W)
    if not args.no_serving:
        try:
            from paper_1301_5892_amd import serving
            out["serving"] = serving.bench(n_requests=args.serving_requests)
        except ImportError:
            out["serving"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
