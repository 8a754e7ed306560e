"""Benchmark: SSCN steps of the 3D Gross-Pitaevskii equation on a 256^3 grid.

Workload (the headline configuration): 256^3 grid, dx = 0.05, V = (x^2 + 4y^2
+ 9z^2)/2, g = 1000, dt = 2e-4, starting from a Gaussian with 1e-3 seeded
complex noise; imaginary-time steps followed by real-time steps from the
imaginary-time result.  One benchmark step = one full SSCN time step of the
grid (potential/nonlinear substep, three Crank-Nicolson sweeps, imaginary-time
norm and renormalisation).  ``--steps K`` times ceil(K/2) imaginary-time steps
then floor(K/2) real-time steps in complex128 (the reported value), after an
untimed warm-up of W steps and at least 0.3 s of stepping.

value = grid points x K / (HIP-event time of the gp_step calls on the launch
stream; inputs resident in HBM).  One JSON line is printed on stdout.

Beside the value, the line carries (each a "leg", selectable with --legs):
  fp32      the same K steps with complex64 bulk arithmetic and FP64 reductions;
  accuracy  the full-length run (2000 imaginary + 2000 real steps) in both
            precisions, each observable's error against the stored FP64-oracle
            values (tests/golden/headline_256cubed.json) and the long-run rate;
  oned      the 1D workload (N = 512, 10^4 imaginary steps, g = 0 and 62.74):
            wall time, mu, E, rms and their error against the stored oracle values;
  quench    the 128^3 quench (ground state of the trap (1, 1, 4), then w_x -> 0.5
            and 1000 real-time steps): rate, per-kernel times, conservation;
  batch     64 uneven 2D problems in one autotuned call (complex64);
  adjoint   gradient of a final-state loss over 2000 real-time steps of a 256^2
            grid between imaginary-time ground states, both precisions;
  sweep     2D real-time point-updates/s against NX = NY = 20 .. 1000;
  cpu       the FP64 oracle on the host cores, all of them and one.

Profile helpers (no GPU needed): --summarize-trace DIR and
--summarize-traffic FETCH_DIR WRITE_DIR turn rocprofv3 CSV output into the
markdown summaries kept under profiles/.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s + %HBM peak, 3D 256³ SSCN, FP64 vs FP32, at stated μ error"
HBM_PEAK_GBPS = 8000.0
ALL_LEGS = ("fp32", "accuracy", "oned", "quench", "batch", "adjoint", "sweep", "cpu")
GOLDEN = os.path.join(ROOT, "tests", "golden")
FIELDS = ("norm", "mu", "energy", "rms_x", "rms_y", "rms_z")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="comma-separated subset of: " + ",".join(ALL_LEGS) + " (or 'none')")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--out", help="summary file written by the --summarize-* modes")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="", help="the command that produced the profile (recorded)")
    ap.add_argument("--traffic-kernel", default="k_sweep_xy_reg<double",
                    help="kernel-name prefix whose bytes per launch the traffic summary records")
    ap.add_argument("--step-kernels", default="",
                    help="semicolon-separated kernel-name prefixes (optionally @grid-size) launched once per step: the traffic summary "
                         "also records their summed bytes per launch as bytes_per_step")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1709_04423_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def golden(name):
    path = os.path.join(GOLDEN, name)
    return json.load(open(path)) if os.path.exists(path) else None


def rel_errors(got, ref, fields=FIELDS):
    out = {}
    for k in fields:
        if ref.get(k, 0.0) != 0.0:
            out[k] = abs(got[k] - ref[k]) / abs(ref[k])
    return out


class Timer:
    """HIP-event timing on the current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


# ------------------------------------------------------------------ headline

def headline_pass(torch, binding, w, psi, imag_steps, real_steps, prec, warmup, instrument):
    """Untimed warm-up (W steps, then more until 0.3 s have passed), then the timed
    imaginary + real phases from psi.  Returns (ms, observables after the run,
    per-kernel (launches, total ms) or None, warm-up steps taken)."""
    pi = binding.Plan(w.n, w.dx, w.dt, binding.GP_IMAG, w.omega, w.g, prec)
    pr = binding.Plan(w.n, w.dx, w.dt, binding.GP_REAL, w.omega, w.g, prec)
    work = psi.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm = 0
    while warm < max(warmup, 2) or time.perf_counter() - t0 < 0.3:
        pi.step(work, 1)
        pr.step(work, 1)
        torch.cuda.synchronize()
        warm += 2
    work.copy_(psi)
    pi.set_step(0)
    pr.set_step(0)
    if instrument:
        pi.timing_enable(3 * imag_steps + 4)
        pr.timing_enable(3 * real_steps + 4)
    with Timer(torch) as t:
        pi.step(work, imag_steps)
        pr.step(work, real_steps)
    kt = None
    if instrument:
        kt = {}
        for p in (pi, pr):
            for name, (cnt, tot) in p.timing_read().items():
                c0, t0_ = kt.get(name, (0, 0.0))
                kt[name] = (c0 + cnt, t0_ + tot)
    obs = pr.observables(work)
    return t.ms, obs, kt, warm


def roofline_of(w, kt, bytes_per_point):
    """Roofline of the dominant kernel (largest total time among the sweeps).
    Algorithmic bytes of a launch: one read and one write of every grid value
    it takes in and gives out -- 2 x 16 B per point in complex128 for every sweep
    kernel, the fused x+y sweep included (its x result stays on chip)."""
    sweeps = {k: v for k, v in kt.items() if k.startswith("sweep")}
    dom = max(sweeps, key=lambda k: sweeps[k][1])
    cnt, tot = sweeps[dom]
    avg_ms = tot / cnt
    alg = 2 * bytes_per_point * w.points
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = None
    tf = read_traffic_summary(os.path.join(ROOT, "profiles", f"traffic_{dom}_256cubed_c128.md"))
    if tf and tf.get("kernel_source_hash") == kernel_source_hash():
        traffic = tf.get("bytes_per_launch")
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "launches": cnt, "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": alg,
            "sweeps_per_launch": 2 if dom == "sweep_xy" else 1,
            "traffic_GBps": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1)}


def full_length(torch, binding, w, psi0, prec):
    """2000 imaginary then 2000 real steps from psi0, observables after each phase."""
    pi = binding.Plan(w.n, w.dx, w.dt, binding.GP_IMAG, w.omega, w.g, prec)
    pr = binding.Plan(w.n, w.dx, w.dt, binding.GP_REAL, w.omega, w.g, prec)
    psi = psi0.clone()
    with Timer(torch) as t1:
        pi.step(psi, w.steps)
    oi = pi.observables(psi)
    with Timer(torch) as t2:
        pr.step(psi, w.steps)
    orr = pr.observables(psi)
    return oi, orr, (t1.ms + t2.ms) / (2 * w.steps)


def accuracy_leg(torch, binding, inputs, w, psi_np):
    ref = golden("headline_256cubed.json")
    out = {"reference": "FP64 oracle, tests/golden/headline_256cubed.json" if ref else None,
           "steps": {"imag": w.steps, "real": w.steps}}
    for name, dtype, prec in (("c128", torch.complex128, binding.GP_C128), ("c64", torch.complex64, binding.GP_C64)):
        psi = torch.from_numpy(psi_np).to("cuda").to(dtype)
        oi, orr, ms = full_length(torch, binding, w, psi, prec)
        d = {"ms_per_step": ms, "point_updates_per_s": w.points / (ms * 1e-3),
             "after_imag": {k: oi[k] for k in ("norm", "mu", "energy")},
             "after_real": {k: orr[k] for k in ("norm", "mu", "energy")}}
        if ref:
            ei = rel_errors(oi, ref["imag"][str(w.steps)])
            er = rel_errors(orr, ref["real"][str(w.steps)])
            d["rel_err_after_imag"] = ei
            d["rel_err_after_real"] = er
            d["max_rel_err_norm_mu_energy"] = max(max(e[k] for k in ("norm", "mu", "energy")) for e in (ei, er))
        out[name] = d
        log(f"full length {name}: {ms * 1e3:.1f} us/step, mu {oi['mu']:.12f}"
            + (f", max rel err {d['max_rel_err_norm_mu_energy']:.2e}" if ref else ""))
        del psi
        torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ other legs

def gpu_ground_state(torch, binding, n, dx, dt, omega, g, prec=0, tol=1e-12, block=100, max_steps=200_000,
                     psi=None):
    """Imaginary-time SSCN on the GPU from the g = 0 Gaussian until mu changes by
    less than tol over `block` steps (a benchmark input, not a reference)."""
    from paper_1709_04423_amd import inputs
    plan = binding.Plan(n, dx, dt, binding.GP_IMAG, omega, g, prec)
    if psi is None:
        psi = torch.from_numpy(inputs.gaussian(n, dx, omega)).to("cuda")
    prev, steps = None, 0
    while steps < max_steps:
        plan.step(psi, block)
        steps += block
        mu = plan.observables(psi)["mu"]
        if prev is not None and abs(mu - prev) < tol:
            break
        prev = mu
    return psi, steps, mu


def oned_leg(torch, binding, inputs):
    w = inputs.ONE_D
    ref = golden("oned_512.json")
    out = {"workload": "1d_imag_512", "steps": w.steps, "dt": w.dt, "dx": w.dx}
    for g in w.extra["g_values"]:
        plan = binding.Plan(w.n, w.dx, w.dt, binding.GP_IMAG, w.omega, g)
        psi0 = torch.from_numpy(inputs.gaussian(w.n, w.dx, w.omega)).to("cuda")
        psi = psi0.clone()
        plan.step(psi, 100)  # warm-up
        psi.copy_(psi0)
        plan.set_step(0)
        with Timer(torch) as t:
            plan.step(psi, w.steps)
        o = plan.observables(psi)
        d = {"wall_ms": t.ms, "us_per_step": 1e3 * t.ms / w.steps, "mu": o["mu"], "energy": o["energy"],
             "rms_x": o["rms_x"]}
        if ref and str(g) in ref:
            d["rel_err_vs_oracle"] = rel_errors(o, ref[str(g)], ("norm", "mu", "energy", "rms_x"))
        out[f"g={g}"] = d
        log(f"1d g={g}: {t.ms:.1f} ms for {w.steps} steps, mu {o['mu']:.12f}")
    return out


def quench_leg(torch, binding, inputs):
    w = inputs.QUENCH_3D
    before = w.extra["omega_before"]
    psi, gs_steps, mu0 = gpu_ground_state(torch, binding, w.n, w.dx, 1e-2, before, w.g)
    plan = binding.Plan(w.n, w.dx, w.dt, binding.GP_REAL, w.omega, w.g)
    o0 = plan.observables(psi)
    work = psi.clone()
    plan.step(work, 20)  # warm-up
    work.copy_(psi)
    plan.set_step(0)
    with Timer(torch) as t:
        plan.step(work, w.steps)
    o1 = plan.observables(work)
    # per-kernel times of the same run, from events around every launch
    work.copy_(psi)
    plan.set_step(0)
    plan.timing_enable(4 * w.steps + 4)
    plan.step(work, w.steps)
    kt = plan.timing_read()
    plan.timing_enable(0)
    value = w.points * w.steps / (t.ms * 1e-3)
    out = {"workload": "3d_128cubed_real_quench", "grid": list(w.n), "steps": w.steps,
           "ground_state": {"imag_steps": gs_steps, "dt": 1e-2, "mu": mu0},
           "value": value, "unit": "grid-point updates/s", "ms_per_step": t.ms / w.steps,
           "hbm_frac_at_96B": 96 * value / 1e9 / HBM_PEAK_GBPS,
           "per_kernel": {k: {"launches": c, "avg_ms": round(m / c, 5)} for k, (c, m) in kt.items()},
           "norm_drift": o1["norm"] - o0["norm"], "energy_rel_change": (o1["energy"] - o0["energy"]) / o0["energy"],
           "rms_x": [o0["rms_x"], o1["rms_x"]]}
    ref = golden("quench_128cubed.json")
    if ref:
        out["rel_err_vs_oracle_after_1000"] = rel_errors(o1, ref["real"]["1000"], ("norm", "mu", "energy", "rms_x"))
        out["reference_note"] = ("oracle run from the oracle's own ground state; this run starts from the GPU's, "
                                 "which agrees to rounding")
    dram = read_traffic_summary(os.path.join(ROOT, "profiles", "traffic_quench_128cubed_c128.md"))
    if dram and dram.get("kernel_source_hash") == kernel_source_hash():
        out["dram_bytes_per_step"] = dram.get("bytes_per_step")
    log(f"quench 128^3: {value:.3e} point-updates/s, {t.ms / w.steps * 1e3:.1f} us/step")
    return out


def batch_leg(torch, binding, inputs, steps=1000):
    import tempfile
    probs = inputs.batch_problems()
    b = binding.Batch([p.n for p in probs], 0.05, 1e-3, binding.GP_REAL, [p.omega for p in probs],
                      [p.g for p in probs], binding.GP_C64)
    cache = os.path.join(tempfile.gettempdir(), f"sscn_batch_tune_{kernel_source_hash()}.txt")
    cfg = b.autotune(cache)
    # lines per item and y segments as tuned per line length (x lines: nx, y lines: ny)
    cfg["per_side"] = {str(n): b.side_config(n) for n in sorted({m for p in probs for m in p.n})}
    psis = [torch.from_numpy(inputs.gaussian(p.n, p.dx, p.omega).astype("complex64")).to("cuda") for p in probs]
    b.step(psis, 10)
    with Timer(torch) as t:
        b.step(psis, steps)
    pts = sum(p.points for p in probs)
    v = pts * steps / (t.ms * 1e-3)
    log(f"batch: {v:.3e} point-updates/s ({t.ms / steps:.3f} ms/step, config {cfg})")
    out = {"value": v, "unit": "grid-point updates/s", "problems": len(probs), "points": pts, "steps": steps,
           "ms_per_step": t.ms / steps, "dtype": "c64 bulk, f64 reductions", "config": cfg,
           "hbm_frac_at_32B": 32 * v / 1e9 / HBM_PEAK_GBPS,
           "note": "2D: 32 B per point-step (one complex64 read and write per sweep, two sweeps)"}
    # bytes through the L2 (FETCH_SIZE / WRITE_SIZE counters) of one step's two launches,
    # measured for the tuned configuration the profile recorded
    dram = read_traffic_summary(os.path.join(ROOT, "profiles", "traffic_batch_form_c64.md"))
    if dram and dram.get("kernel_source_hash") == kernel_source_hash() and dram.get("bytes_per_step"):
        out["dram_bytes_per_step"] = dram["bytes_per_step"]
        out["dram_GBps"] = dram["bytes_per_step"] / (t.ms / steps * 1e-3) / 1e9
    return out


def adjoint_leg(torch, binding, inputs):
    from paper_1709_04423_amd import adjoint
    w = inputs.ADJOINT_2D
    sched = inputs.gamma_schedule(w.steps)
    psi0, s0, mu0 = gpu_ground_state(torch, binding, w.n, w.dx, w.dt, (1.0, 1.0), w.g)
    tgt, s1, mu1 = gpu_ground_state(torch, binding, w.n, w.dx, w.dt, (w.extra["gamma_target"], 1.0), w.g)
    out = {"workload": "2d_256sq_T2000_real_adjoint",
           "inputs": {"psi0": f"ground state at gamma = 1 ({s0} imaginary steps, mu {mu0:.12f})",
                      "target": f"ground state at gamma = 1.5 ({s1} imaginary steps, mu {mu1:.12f})"}}
    ref = golden("adjoint_256sq.json")
    for name, dt_ in (("c128", torch.complex128), ("c64", torch.complex64)):
        pw = psi0.to(dt_).clone().requires_grad_(True)  # warm-up: loads the kernels this form launches
        sw = torch.tensor(sched[:20], dtype=torch.float64, device="cuda", requires_grad=True)
        adjoint.overlap_loss(adjoint.evolve(pw, sw, w.g, w.n, w.dx, w.dt, (1.0, 1.0)), tgt.to(dt_), w.dx).backward()
        psi = psi0.to(dt_).clone().requires_grad_(True)
        s = torch.tensor(sched, dtype=torch.float64, device="cuda", requires_grad=True)
        g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
        tg = tgt.to(dt_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = adjoint.overlap_loss(adjoint.evolve(psi, s, g, w.n, w.dx, w.dt, (1.0, 1.0)), tg, w.dx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pts = w.points * w.steps
        d = {"forward_s": t1 - t0, "backward_s": t2 - t1, "gradient_s": t2 - t0,
             "point_updates_per_s": 3 * pts / (t2 - t0), "loss": float(loss.item()), "dg": float(g.grad.item())}
        if ref:
            import numpy as np
            gr = ref["gradient"]
            ds = s.grad.cpu().numpy()
            d["loss_rel_err_vs_oracle"] = abs(d["loss"] - gr["loss"]) / abs(gr["loss"])
            d["dg_rel_err_vs_oracle"] = abs(d["dg"] - gr["dg"]) / abs(gr["dg"])
            dsr = np.array(gr["dsched"])
            d["dsched_max_rel_err_vs_oracle"] = float(np.max(np.abs(ds - dsr)) / np.max(np.abs(dsr)))
            d["reference_note"] = "oracle gradient from the oracle's own ground states"
        out[name] = d
        log(f"adjoint {name}: gradient {t2 - t0:.3f} s")
    out["note"] = ("wall time of loss.backward() after a checkpointed forward; point updates count the forward, "
                   "the recomputed and the adjoint steps")
    return out


def sweep_leg(torch, binding, inputs, sizes=(20, 50, 100, 200, 300, 500, 700, 1000)):
    """2D real-time SSCN rate against grid size (NX = NY), complex128, the
    counterpart of the paper's real2d grid-size study (Fig. 2)."""
    pts = []
    dx = 0.05  # the 2D workloads' spacing: the box grows with n, the per-point work stays the same
    for n in sizes:
        plan = binding.Plan((n, n), dx, 1e-3, binding.GP_REAL, (1.0, 1.0), 50.0)
        psi = torch.from_numpy(inputs.gaussian((n, n), dx, (1.0, 1.0))).to("cuda")
        plan.step(psi, 20)
        steps = max(100, min(4000, int(2e8 / (n * n))))
        with Timer(torch) as t:
            plan.step(psi, steps)
        us = 1e3 * t.ms / steps
        v = n * n / (us * 1e-6)
        pts.append({"n": n, "us_per_step": round(us, 3), "point_updates_per_s": v,
                    "hbm_frac_at_64B": 64 * v / 1e9 / HBM_PEAK_GBPS})
        log(f"sweep 2d n={n}: {us:.2f} us/step, {v:.3e} point-updates/s")
    return {"workload": "2d real time, NX = NY, dx 0.05 (box [-NX dx/2, NX dx/2)^2), trap (1, 1), g 50, dt 1e-3, "
                        "complex128; one sample per size", "points": pts}


def cpu_leg(w, psi0_np, budget_s):
    """The FP64 oracle on the host: alternating imaginary/real steps of the same
    256^3 input for about budget_s seconds on all cores, then on one core for
    about budget_s / 2 seconds (at least 2 steps each)."""
    import oracle
    res = {}
    default = oracle.num_threads()  # OMP_NUM_THREADS, else every core the runtime sees
    for label, threads, budget in (("all", default, budget_s), ("one", 1, budget_s / 2)):
        oracle.set_threads(threads)
        psi = psi0_np
        steps = 0
        t0 = time.perf_counter()
        while True:
            mode = oracle.IMAG if steps % 2 == 0 else oracle.REAL
            psi = oracle.step(psi, w.dx, w.dt, mode, w.omega, w.g, 1)
            steps += 1
            el = time.perf_counter() - t0
            if steps >= 2 and el >= budget:
                break
        res[label] = (w.points * steps / el, steps, el, oracle.num_threads())
    oracle.set_threads(default)
    v, steps, el, cores = res["all"]
    v1, steps1, el1, _ = res["one"]
    return {"value": v, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} SSCN steps (alternating imaginary/real time) of the 256^3 headline grid, "
                      f"complex128, {el:.1f} s on {cores} OpenMP threads ({cpu_model()})",
            "one_thread": {"value": v1, "cores": 1,
                           "sample": f"{steps1} steps of the same grid, {el1:.1f} s on one thread"}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def copy_probe(torch, binding, nbytes=1 << 30, reps=10):
    src = torch.empty(nbytes // 16, dtype=torch.complex128, device="cuda")
    src.real.fill_(1.0)
    dst = torch.empty_like(src)
    binding.copy_probe(dst, src)
    with Timer(torch) as t:
        for _ in range(reps):
            binding.copy_probe(dst, src)
    del src, dst
    return 2.0 * nbytes * reps / (t.ms * 1e-3) / 1e9


# ------------------------------------------------------------------ profile summaries

def _csv_rows(directory, suffix):
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name):
    name = name.replace("gp::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*$", "", name).replace("gp::", "").strip()


def summarize_trace(directory, out, title, command):
    rows = _csv_rows(directory, "kernel_stats.csv")
    if not rows:
        raise SystemExit(f"no kernel_stats.csv under {directory}")
    lines = [f"# Kernel trace: {title}", "", "Command (REPO = repository root, OUT = any output directory):", "",
             f"    {command}", "", "| kernel | calls | avg us | min us | max us | % time |",
             "|---|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")
    print(f"wrote {out}")


def _counter_means(directory, counter):
    """Mean counter value per dispatch, keyed by (kernel name, grid size): the same
    kernel launched on different grids (workloads) is kept apart."""
    per = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Kernel_Name"], int(r["Grid_Size"]))
        per.setdefault(key, {}).setdefault(r["Dispatch_Id"], 0.0)
        per[key][r["Dispatch_Id"]] += float(r["Counter_Value"])  # summed over dimensions of one dispatch
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in per.items()}


def _selects(key, selector):
    """selector 'name-prefix' or 'name-prefix@grid-size'."""
    prefix, _, grid = selector.partition("@")
    return _short(key[0]).startswith(prefix) and (not grid or key[1] == int(grid))


def summarize_traffic(fetch_dir, write_dir, out, title, command, kernel_prefix, step_kernels=""):
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if _short(k[0]).startswith("k_copy")]
    if not copy:
        raise SystemExit("the profiled run must include the 1 GiB copy probe (k_copy) for calibration")
    kib = float(1 << 20)  # 1 GiB copied = 2^20 KiB each way
    fscale = kib / fetch[copy[0]][1]
    wscale = kib / write[[k for k in write if _short(k[0]).startswith("k_copy")][0]][1]
    lines = [f"# HBM traffic per launch: {title}", "", "Commands (one counter per run; REPO = repository root, "
             "OUT = any output directory):", ""] + [f"    {c}" for c in command.split(" ;; ")] + [
        "", f"Calibration: the copy kernel `k_copy` moves exactly 1 GiB each way per launch; its counters read "
            f"FETCH_SIZE = {fetch[copy[0]][1]:.1f} KiB and WRITE_SIZE = {kib / wscale:.1f} KiB, so read bytes = "
            f"FETCH_SIZE x {fscale:.4f} KiB and write bytes = WRITE_SIZE x {wscale:.4f} KiB.", "",
        "| kernel | grid size | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB |",
        "|---|---|---|---|---|---|---|"]
    chosen = None
    step_prefixes = [p for p in step_kernels.split(";") if p]
    step_bytes = {}
    for key in sorted(fetch, key=lambda k: -fetch[k][1]):
        n, f = fetch[key]
        wv = write.get(key, (0, 0.0))[1]
        rb, wb = f * fscale * 1024, wv * wscale * 1024
        lines.append(f"| `{_short(key[0])}` | {key[1]} | {n} | {f:.1f} | {wv:.1f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} |")
        if chosen is None and _selects(key, kernel_prefix):
            chosen = (f"{_short(key[0])} (grid {key[1]})", rb, wb)
        for p in step_prefixes:
            if _selects(key, p):
                # instantiations of one kernel kind: launch-weighted mean
                c, tot = step_bytes.get(p, (0, 0.0))
                step_bytes[p] = (c + n, tot + n * (rb + wb))
    lines += ["", "Recorded for the benchmark (dominant kernel, read by bench.py while the source hash matches):", ""]
    if chosen:
        lines += [f"- kernel: `{chosen[0]}`", f"- kernel_source_hash: {kernel_source_hash()}",
                  f"- read_bytes: {int(chosen[1])}", f"- write_bytes: {int(chosen[2])}",
                  f"- bytes_per_launch: {int(chosen[1] + chosen[2])}"]
    if step_prefixes and len(step_bytes) == len(step_prefixes):
        lines += [f"- step_kernels: {', '.join(step_prefixes)}",
                  f"- bytes_per_step: {int(sum(t / c for c, t in step_bytes.values()))}"]
    open(out, "w").write("\n".join(lines) + "\n")
    print(f"wrote {out}")


def read_traffic_summary(path):
    if not os.path.exists(path):
        return None
    d = {}
    for line in open(path):
        m = re.match(r"- (\w+): `?([^`\n]+)`?", line.strip())
        if m:
            v = m.group(2).strip()
            d[m.group(1)] = int(v) if v.isdigit() else v
    return d


# ------------------------------------------------------------------ main

def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.out, args.title, args.command)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.out, args.title, args.command, args.traffic_kernel,
                          args.step_kernels)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the SSCN path here is "
              "single-GPU and has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)
    legs = set() if args.legs == "none" else set(args.legs.split(","))
    unknown = legs - set(ALL_LEGS)
    if unknown:
        raise SystemExit(f"unknown legs {sorted(unknown)}")
    import torch

    from paper_1709_04423_amd import binding, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    binding.lib()
    w = inputs.HEADLINE_3D
    K, W = args.steps, args.warmup
    imag_steps, real_steps = (K + 1) // 2, K // 2
    log(f"workload {w.name}: grid {w.n}, {imag_steps} imag + {real_steps} real steps, warmup >= {W} steps and 0.3 s")
    psi_np = inputs.headline_initial()
    psi = torch.from_numpy(psi_np).to("cuda")

    # the headline pass: gp_step calls only, timed by events around the whole run
    ms, obs64, _, warm = headline_pass(torch, binding, w, psi, imag_steps, real_steps, binding.GP_C128, W, False)
    value = w.points * K / (ms * 1e-3)
    log(f"complex128: {ms:.2f} ms for {K} steps ({warm} warm-up steps) -> {value:.4e} point-updates/s")
    # a second pass with an event pair around every launch gives the per-kernel times
    ms_inst, _, kt, _ = headline_pass(torch, binding, w, psi, imag_steps, real_steps, binding.GP_C128, W, True)
    per_kernel = {k: {"launches": c, "avg_ms": round(t / c, 5)} for k, (c, t) in kt.items()}
    log(f"per-kernel: {per_kernel}")
    roof = roofline_of(w, kt, 16)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3d_256cubed_imag_then_real", "grid": list(w.n), "dx": w.dx, "dt": w.dt,
                   "omega": list(w.omega), "g": w.g, "imag_steps": imag_steps, "real_steps": real_steps,
                   "storage": "complex128", "initial": "Gaussian + 1e-3 seeded complex noise"},
        "warmup_steps_taken": warm,
        "step_hbm_frac_at_96B": round(96 * value / 1e9 / HBM_PEAK_GBPS, 4),
        "step_hbm_frac_at_64B": round(64 * value / 1e9 / HBM_PEAK_GBPS, 4),
        "ms_per_step_with_kernel_events": ms_inst / K,
        "roofline": roof,
        "per_kernel": per_kernel,
    }

    if "fp32" in legs:
        ms32, obs32, kt32, _ = headline_pass(torch, binding, w, psi.to(torch.complex64), imag_steps, real_steps,
                                             binding.GP_C64, W, False)
        v32 = w.points * K / (ms32 * 1e-3)
        out["fp32"] = {"value": v32, "ms_per_step": ms32 / K, "dtype": "c64 bulk, f64 reductions",
                       "step_hbm_frac_at_48B": 48 * v32 / 1e9 / HBM_PEAK_GBPS,
                       "step_hbm_frac_at_32B": 32 * v32 / 1e9 / HBM_PEAK_GBPS}
        log(f"complex64: {ms32:.2f} ms -> {v32:.4e} point-updates/s")
    if "accuracy" in legs:
        acc = accuracy_leg(torch, binding, inputs, w, psi_np)
        out["accuracy"] = acc
        out["long_run_value"] = acc["c128"]["point_updates_per_s"]
        if "fp32" in out:
            for k in ("rel_err_after_imag", "rel_err_after_real", "max_rel_err_norm_mu_energy"):
                if k in acc["c64"]:
                    out["fp32"][k] = acc["c64"][k]
            out["fp32"]["long_run_value"] = acc["c64"]["point_updates_per_s"]
    del psi
    torch.cuda.empty_cache()
    if "oned" in legs:
        out["oned"] = oned_leg(torch, binding, inputs)
    if "quench" in legs:
        out["quench"] = quench_leg(torch, binding, inputs)
        torch.cuda.empty_cache()
    if "batch" in legs:
        out["batch"] = batch_leg(torch, binding, inputs)
        torch.cuda.empty_cache()
    if "adjoint" in legs:
        out["adjoint"] = adjoint_leg(torch, binding, inputs)
        torch.cuda.empty_cache()
    if "sweep" in legs:
        out["grid_sweep"] = sweep_leg(torch, binding, inputs)
    out["copy_probe_GBps"] = round(copy_probe(torch, binding), 1)
    log(f"copy probe: {out['copy_probe_GBps']:.0f} GB/s")
    if "cpu" in legs:
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_leg(w, psi_np, args.cpu_seconds)
        log(f"CPU oracle: {out['cpu_baseline']['value']:.3e} point-updates/s on {out['cpu_baseline']['cores']} "
            f"threads, {out['cpu_baseline']['one_thread']['value']:.3e} on one")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
