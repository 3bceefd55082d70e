"""Benchmark: phase-space cell-updates per second per split step on one GPU.

Default workload: the 4096 x 4096 large-grid case (FP32 delta f, degree 17,
dt = 0.02), the configuration the metric is quoted on.  One "step" is one
full Strang step (v-sweep, transpose, x-sweep, transpose + rho, field solve,
v-sweep).  The timed region holds exactly --steps steps, bracketed by device
synchronisation.  A second pass of the same number of steps records HIP events
on the sim's stream around every kernel launch; they give each kernel's
average duration for the roofline.

Prints one JSON line with the headline FP32 delta-f rate, the FP64 plain
rate on the same GPU, the roofline of the dominant kernel, the CPU-oracle
baseline and (unless --no-serving) the serving-mix latency summary.
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
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--serving-requests", type=int, default=512)
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one plain 256 MiB device-to-device copy first (a known-size "
                        "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return p.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("fft.hpp", "kernels.hip", "vog_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1301_5892_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
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
    line = {"sweep_v": w.nv, "sweep_x": w.nx}.get(kind)
    # Algorithmic bytes: the sweep reads and writes f once; a transpose also
    # moves f once each way (not algorithmic for the method, reported as is).
    bytes_per_launch = 2 * es * cells
    hbm = {"bound": "hbm", "achieved": bytes_per_launch / avg_s / 1e9, "peak": HBM_PEAK_GBS,
           "unit": "GB/s"}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    hbm["traffic"] = stored_traffic(kind, w.name, precision)
    hbm["kernel"] = kind
    hbm["avg_launch_ms"] = avg_s * 1e3
    hbm["launches"] = n
    hbm["bytes_per_launch"] = bytes_per_launch
    if line:
        # The paper's real-data operation count per advected element,
        # 5 log2(N) + 3 (FFT pair plus complex multiply).
        flops = (5 * math.log2(line) + 3) * cells
        peak = FP32_VALU_PEAK_TFLOPS if es == 4 else FP64_VALU_PEAK_TFLOPS
        ach = flops / avg_s / 1e12
        hbm["alu_view"] = {"achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                           "flops_per_launch": flops}
    return hbm


def cpu_baseline(w, seconds):
    import oracle
    o = oracle.Oracle(w, deltaf=w.precision.endswith("deltaf")).init()
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 1000:
            break
    return {"value": w.cells * steps / el, "unit": "cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{w.name}, {'delta-f' if o.deltaf else 'plain'} FP64 direct-stencil oracle, "
                      f"{steps} Strang steps from f0 ({el:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              f"independent simulations shard one per GPU, see DESIGN.md", file=sys.stderr)
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
    if not args.no_fp64:
        el64, prof64, fin64, el64p = run_gpu(w, "fp64_plain", K, W)
        out["fp64_plain"] = {"value": w.cells * K / el64, "ms_per_step": el64 / K * 1e3,
                             "ms_per_step_with_kernel_events": el64p / K * 1e3,
                             "finite": fin64,
                             "kernels_ms_per_step": {k: v[0] / K for k, v in prof64.items()},
                             "roofline": roofline_for(w, "fp64_plain", prof64, K)}
        out["fp32_over_fp64"] = out["value"] / out["fp64_plain"]["value"]
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
