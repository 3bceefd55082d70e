"""Long-horizon precision report (Sections 4.1 and 4.2 of the paper).

Runs on a machine with the GPU:

    python tests/precision_report.py --out REPORT.md

and writes a Markdown section with
  * the strong-Landau case (256 x 512, dt = 0.05, 1000 steps): the drift of
    the mass rho_hat_0, of L2 = dx dv sum f^2 and of the energy relative to
    t = 0, every 100 steps, for the GPU in FP32 delta f and in FP64 plain and
    for the FP64 oracle (delta-f and plain forms), and the error of each GPU
    run against the oracle of the same form; plus the step up to which an
    oracle run from f0 rounded to FP32 stays within 1e-5 of the FP64 oracle;
  * the bump-on-tail case (1024 x 2048, dt = 0.05, 10000 steps): the same
    drifts every 1000 steps over the whole run on the GPU (FP32 delta f and
    FP64 plain), and the error of the FP32 delta-f run against the FP64
    oracle every 25 steps up to step 300 (the oracle is stepped that far),
    beside the oracle-vs-oracle divergence from f0 rounded to FP32.

    python tests/precision_report.py --splice REPORT.md --into DOC.md

puts that section into the Markdown file DOC.md between its precision-report
markers.
Only the oracle and the C ABI of libvog are used.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

BEGIN = "<!-- precision-report:begin -->"
END = "<!-- precision-report:end -->"


def rel(a, b):
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _oracle_moments(o):
    """(rho_hat_0, L2, energy) of an oracle state."""
    l2, en = o.diag_moments()
    return o.diag_field()[1], l2, en


def _gpu_records(sim, store):
    for r in sim.diag():
        store[int(r["step"])] = r


def _drift_rows(steps, series):
    """series: name -> {step: (rho0, l2, energy)}; rows of drifts against step 0."""
    rows = []
    for n in steps:
        row = [str(n)]
        for name, d in series.items():
            m0, l0, e0 = d[0]
            m, l, e = d[n]
            row += [f"{m - m0:+.2e}", f"{l / l0 - 1:+.2e}", f"{e / e0 - 1:+.2e}"]
        rows.append(row)
    return rows


def _table(head, rows):
    out = ["| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    out += ["| " + " | ".join(r) + " |" for r in rows]
    return "\n".join(out)


def strong_landau(lines):
    import numpy as np

    import oracle
    import workloads
    from paper_1301_5892_amd import vog
    w = workloads.landau_strong()
    n_total, every = 1000, 100
    g32 = vog.Sim(w, moments_every=every, precision="fp32_deltaf").init()
    g64 = vog.Sim(w, moments_every=every, precision="fp64_plain").init()
    odf = oracle.Oracle(w.replace(precision="fp32_deltaf")).init()
    opl = oracle.Oracle(w.replace(precision="fp64_plain")).init()
    rnd = oracle.Oracle(w.replace(precision="fp32_deltaf")).init()
    rnd.f = np.ascontiguousarray(odf.f.astype(np.float32).astype(np.float64))
    rnd.update_field()
    series = {"GPU FP32 δf": {}, "GPU FP64 plain": {}, "oracle FP64 δf": {}, "oracle FP64 plain": {}}
    rec32, rec64 = {}, {}
    series["oracle FP64 δf"][0] = _oracle_moments(odf)
    series["oracle FP64 plain"][0] = _oracle_moments(opl)
    # the GPU runs start from the same f0: their drifts are taken against the
    # oracle's t = 0 values of the same form
    series["GPU FP32 δf"][0] = series["oracle FP64 δf"][0]
    series["GPU FP64 plain"][0] = series["oracle FP64 plain"][0]
    errs, horizon = [], None
    for n in range(every, n_total + 1, every):
        for _ in range(every // 10):   # the oracle-vs-oracle horizon to 10 steps
            odf.step(10)
            rnd.step(10)
            if horizon is None and (rel(rnd.f, odf.f) > 1e-5 or rel(rnd.E, odf.E) > 1e-5):
                horizon = odf.step_count - 10
        opl.step(every)
        g32.step(every)
        g64.step(every)
        _gpu_records(g32, rec32)
        _gpu_records(g64, rec64)
        series["oracle FP64 δf"][n] = _oracle_moments(odf)
        series["oracle FP64 plain"][n] = _oracle_moments(opl)
        errs.append([str(n), f"{rel(g32.get_raw(), odf.f):.2e}", f"{rel(g32.get_E(), odf.E):.2e}",
                     f"{rel(g64.get_f(), opl.f):.2e}", f"{rel(g64.get_E(), opl.E):.2e}",
                     f"{rel(rnd.f, odf.f):.2e}"])
    for name, rec in (("GPU FP32 δf", rec32), ("GPU FP64 plain", rec64)):
        for n, r in rec.items():
            if n % every == 0 and n > 0:
                series[name][n] = (float(r["rho0"]), float(r["l2"]), float(r["energy"]))
    steps = list(range(every, n_total + 1, every))
    lines.append(f"**Strong Landau damping, {w.nx}×{w.nv}, Δt = {w.dt}, {n_total} steps.** "
                 "Drift against t = 0 of the mass ρ̂₀ (difference), of L2 and of the energy "
                 "(relative):\n")
    head = ["step"] + [f"{nm}: {q}" for nm in series for q in ("ρ̂₀", "L2", "energy")]
    lines.append(_table(head, _drift_rows(steps, series)))
    lines.append("\nError against the FP64 oracle of the same form (max-norm, relative), and the "
                 "oracle run from f0 rounded to FP32 against the exact one:\n")
    lines.append(_table(["step", "FP32 δf: δf", "FP32 δf: E", "FP64 plain: f", "FP64 plain: E",
                         "oracle, f0 in FP32: δf"], errs))
    first = next((int(r[0]) for r in errs if float(r[1]) > 1e-5), None)
    lines.append(f"\nThe oracle run from f0 rounded to FP32 leaves the 1e-5 band "
                 f"{f'at step {horizon}' if horizon is not None else f'at no step up to {n_total}'}: "
                 "rounding the initial state is not what limits the FP32 path; its per-sweep "
                 "rounding is (first checkpoint above 1e-5: step "
                 f"{first if first is not None else f'> {n_total}'}). `tests/test_gpu_parity.py` "
                 "gates the FP32 run at 1e-5 up to step 20 and on this curve beyond.\n")


def bump_on_tail(lines):
    import numpy as np

    import oracle
    import workloads
    from paper_1301_5892_amd import vog
    w = workloads.bump_on_tail()
    n_total, every, n_orc, every_orc = 10000, 1000, 300, 25
    g32 = vog.Sim(w, moments_every=every, precision="fp32_deltaf").init()
    g64 = vog.Sim(w, moments_every=every, precision="fp64_plain").init()
    odf = oracle.Oracle(w.replace(precision="fp32_deltaf")).init()
    rnd = oracle.Oracle(w.replace(precision="fp32_deltaf")).init()
    rnd.f = np.ascontiguousarray(odf.f.astype(np.float32).astype(np.float64))
    rnd.update_field()
    o64 = oracle.Oracle(w.replace(precision="fp64_plain")).init()
    series = {"GPU FP32 δf": {0: _oracle_moments(odf)}, "GPU FP64 plain": {0: _oracle_moments(o64)}}
    curve = []
    for n in range(every_orc, n_orc + 1, every_orc):
        odf.step(every_orc)
        rnd.step(every_orc)
        g32.step(every_orc)
        curve.append([str(n), f"{rel(g32.get_raw(), odf.f):.2e}", f"{rel(g32.get_E(), odf.E):.2e}",
                      f"{rel(rnd.f, odf.f):.2e}", f"{rel(rnd.E, odf.E):.2e}"])
    rec32, rec64 = {}, {}
    _gpu_records(g32, rec32)
    done = n_orc
    while done < n_total:   # (the diagnostics ring holds 4096 records)
        k = min(500, n_total - done)
        g32.step(k)
        _gpu_records(g32, rec32)
        done += k
    for _ in range(n_total // 500):
        g64.step(500)
        _gpu_records(g64, rec64)
    for name, rec in (("GPU FP32 δf", rec32), ("GPU FP64 plain", rec64)):
        for n, r in rec.items():
            if n % every == 0 and n > 0:
                series[name][n] = (float(r["rho0"]), float(r["l2"]), float(r["energy"]))
    steps = list(range(every, n_total + 1, every))
    lines.append(f"\n**Bump-on-tail, {w.nx}×{w.nv}, Δt = {w.dt}, {n_total} steps on the GPU.** "
                 "Drift against t = 0 (the t = 0 values from the oracle):\n")
    head = ["step"] + [f"{nm}: {q}" for nm in series for q in ("ρ̂₀", "L2", "energy")]
    lines.append(_table(head, _drift_rows(steps, series)))
    lines.append(f"\nError of the FP32 δf run against the FP64 oracle (stepped to {n_orc}), beside "
                 "the oracle run from f0 rounded to FP32:\n")
    lines.append(_table(["step", "GPU FP32 δf: δf", "GPU FP32 δf: E", "oracle, f0 in FP32: δf",
                         "oracle, f0 in FP32: E"], curve))


def splice(src, doc):
    with open(src) as fh:
        body = fh.read().strip()
    with open(doc) as fh:
        text = fh.read()
    a, b = text.index(BEGIN) + len(BEGIN), text.index(END)
    with open(doc, "w") as fh:
        fh.write(text[:a] + "\n" + body + "\n" + text[b:])


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--out", default="precision_report.md")
    p.add_argument("--splice", metavar="FILE", default=None,
                   help="put FILE (a report written with --out) into the file given by --into")
    p.add_argument("--into", metavar="DOC", default=None,
                   help="Markdown file with the precision-report markers (with --splice)")
    a = p.parse_args()
    if a.splice:
        if not a.into:
            p.error("--splice needs --into")
        splice(a.splice, a.into)
        return
    import torch
    assert torch.cuda.is_available(), "the report runs the GPU path"
    torch.cuda.set_device(0)
    lines = ["Written by `python tests/precision_report.py` (GPU through the C ABI, FP64 oracle on "
             "the host).\n"]
    strong_landau(lines)
    print("strong Landau done", flush=True)
    bump_on_tail(lines)
    print("bump-on-tail done", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
