"""Benchmark: SSCN steps of the 3D Gross-Pitaevskii equation on a 256^3 grid.

Workload (the headline configuration): 256^3 grid, dx = 0.05, V = (x^2 + 4y^2
+ 9z^2)/2, g = 1000, dt = 2e-4, starting from a Gaussian with 1e-3 seeded
complex noise; imaginary-time steps followed by real-time steps from the
imaginary-time result.  One benchmark step = one full SSCN time step of the
grid (potential/nonlinear substep, three Crank-Nicolson sweeps, imaginary-time
norm and renormalisation).  ``--steps K`` times ceil(K/2) imaginary-time steps
then floor(K/2) real-time steps in complex128 (the reported value), and the
same again with complex64 bulk arithmetic and FP64 reductions (reported beside
it with its chemical-potential error against the complex128 run).

The chosen forms are reported beside it: complex64 bulk (``fp32``), the batched
form (``batch``: 64 uneven 2D problems, 1000 real-time steps in one autotuned
call) and the adjoint form (``adjoint``: gradient of a final-state loss over
2000 real-time steps of a 256^2 grid, both precisions).

value = grid points x steps / time of the gp_step calls (inputs resident in HBM,
HIP-event timing on the launch stream).  One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s + %HBM peak, 3D 256³ SSCN, FP64 vs FP32, at stated μ error"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the complex64 run")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and adjoint forms")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1709_04423_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def timed_run(torch, binding, w, psi, imag_steps, real_steps, prec, warmup, instrument):
    """Run warmup imaginary steps (untimed), then the timed imaginary + real phases.
    Returns (ms, mu after the imaginary phase, kernel timing dict or None)."""
    stream = torch.cuda.current_stream()
    pi = binding.Plan(w.n, w.dx, w.dt, binding.GP_IMAG, w.omega, w.g, prec)
    pr = binding.Plan(w.n, w.dx, w.dt, binding.GP_REAL, w.omega, w.g, prec)
    work = psi.clone()
    if warmup:
        pi.step(work, warmup)
        pr.step(work.clone(), min(warmup, 4))
        work.copy_(psi)
        pi.set_step(0)
        pr.set_step(0)
    if instrument:
        pi.timing_enable(3 * imag_steps + 4)
        pr.timing_enable(3 * real_steps + 4)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    pi.step(work, imag_steps)
    tm = torch.cuda.Event(enable_timing=True)
    tm.record(stream)
    pr.step(work, real_steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    kt = None
    if instrument:
        kt = {}
        for p in (pi, pr):
            for name, (cnt, tot) in p.timing_read().items():
                c0, t0_ = kt.get(name, (0, 0.0))
                kt[name] = (c0 + cnt, t0_ + tot)
    # mu after the imaginary phase: rerun that phase alone (outside the timed region)
    chk = psi.clone()
    pi.set_step(0)
    pi.timing_enable(0)
    pi.step(chk, imag_steps)
    mu = pi.observables(chk)
    obs_real = pr.observables(work)
    del chk
    return ms, wall, mu, obs_real, kt


def copy_probe(torch, binding, nbytes=1 << 30, reps=10):
    src = torch.empty(nbytes // 16, dtype=torch.complex128, device="cuda")
    src.real.fill_(1.0)
    dst = torch.empty_like(src)
    binding.copy_probe(dst, src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        binding.copy_probe(dst, src)
    b.record()
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return gbps


def batch_form(torch, binding, inputs, steps=1000):
    """Batched form: the 64 uneven 2D problems (sides from {128..512}, dx = 0.05,
    dt = 1e-3, g ~ U[10, 500], nu ~ U[0.5, 2]), complex64 bulk, autotuned launch,
    `steps` real-time steps in one gp_batch_step call."""
    import tempfile
    probs = inputs.batch_problems()
    b = binding.Batch([p.n for p in probs], 0.05, 1e-3, binding.GP_REAL, [p.omega for p in probs],
                      [p.g for p in probs], binding.GP_C64)
    cache = os.path.join(tempfile.gettempdir(), "sscn_batch_tune.txt")
    cfg = b.autotune(cache)
    psis = [torch.from_numpy(inputs.gaussian(p.n, p.dx, p.omega).astype("complex64")).to("cuda") for p in probs]
    b.step(psis, 10)
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    b.step(psis, steps)
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e)
    pts = sum(p.points for p in probs)
    v = pts * steps / (ms * 1e-3)
    return {"value": v, "unit": "grid-point updates/s", "problems": len(probs), "points": pts, "steps": steps,
            "ms_per_step": ms / steps, "dtype": "c64 bulk, f64 reductions", "config": cfg,
            "hbm_frac": 32 * v / 1e9 / HBM_PEAK_GBPS,
            "note": "2D: 32 B per point-step (one complex64 read and write per sweep, two sweeps)"}


def adjoint_form(torch, binding, inputs):
    """Adjoint form: 256^2, dx = 0.05, dt = 1e-3, g = 200, T = 2000 real-time steps with a
    seeded trap schedule; forward (sqrt(T) checkpoints) and backward (recompute +
    hand-written adjoint kernels) through torch.autograd, in both precisions."""
    from paper_1709_04423_amd import adjoint
    w = inputs.ADJOINT_2D
    sched = inputs.gamma_schedule(w.steps)
    psi0 = inputs.gaussian(w.n, w.dx, (1.0, 1.0))
    tgt = inputs.gaussian(w.n, w.dx, (1.5, 1.0))
    out = {}
    for name, dt_ in (("c128", torch.complex128), ("c64", torch.complex64)):
        # untimed warm-up: loads the kernels this form launches
        pw = torch.from_numpy(psi0).to("cuda").to(dt_).requires_grad_(True)
        sw = torch.tensor(sched[:20], dtype=torch.float64, device="cuda", requires_grad=True)
        adjoint.overlap_loss(adjoint.evolve(pw, sw, w.g, w.n, w.dx, w.dt, (1.0, 1.0)),
                             torch.from_numpy(tgt).to("cuda").to(dt_), w.dx).backward()
        psi = torch.from_numpy(psi0).to("cuda").to(dt_).requires_grad_(True)
        s = torch.tensor(sched, dtype=torch.float64, device="cuda", requires_grad=True)
        g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
        tg = torch.from_numpy(tgt).to("cuda").to(dt_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = adjoint.overlap_loss(adjoint.evolve(psi, s, g, w.n, w.dx, w.dt, (1.0, 1.0)), tg, w.dx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # forward T steps, backward T recomputed steps + T adjoint steps
        pts = w.points * w.steps
        out[name] = {"forward_s": t1 - t0, "backward_s": t2 - t1, "gradient_s": t2 - t0,
                     "point_updates_per_s": 3 * pts / (t2 - t0), "loss": float(loss.item()),
                     "dg": float(g.grad.item())}
    out["workload"] = "2d_256sq_T2000_real_adjoint"
    out["note"] = ("wall time of loss.backward() after a checkpointed forward; point updates count the "
                   "forward, the recomputed and the adjoint steps")
    return out


def cpu_baseline(w, psi0_np, budget_s):
    """The FP64 oracle on the host cores: alternating imaginary/real steps of the
    same 256^3 input until about budget_s seconds have passed (at least 2 steps)."""
    import oracle
    psi = psi0_np
    steps = 0
    t0 = time.perf_counter()
    while True:
        mode = oracle.IMAG if steps % 2 == 0 else oracle.REAL
        psi = oracle.step(psi, w.dx, w.dt, mode, w.omega, w.g, 1)
        steps += 1
        el = time.perf_counter() - t0
        if steps >= 2 and el >= budget_s:
            break
    pts = w.points * steps
    return {"value": pts / el, "unit": "grid-point updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} SSCN steps (alternating imaginary/real time) of the 256^3 headline grid, "
                      f"complex128, {el:.1f} s on {oracle.num_threads()} OpenMP threads ({cpu_model()})"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the SSCN path here is "
              "single-GPU and has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1709_04423_amd import binding, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    binding.lib()
    w = inputs.HEADLINE_3D
    K, W = args.steps, args.warmup
    imag_steps, real_steps = (K + 1) // 2, K // 2
    log(f"workload {w.name}: grid {w.n}, {imag_steps} imag + {real_steps} real steps, warmup {W}")
    psi_np = inputs.headline_initial()
    psi = torch.from_numpy(psi_np).to("cuda")

    # the headline pass: gp_step calls only, timed by events around the whole run
    ms, wall, mu64, real64, _ = timed_run(torch, binding, w, psi, imag_steps, real_steps, binding.GP_C128, W,
                                          instrument=False)
    value = w.points * K / (ms * 1e-3)
    log(f"complex128: {ms:.1f} ms for {K} steps -> {value:.3e} point-updates/s")
    # a second pass with an event pair around every launch gives the per-kernel times
    # (the events themselves add a few percent to each launch)
    ms_inst, _, _, _, kt = timed_run(torch, binding, w, psi, imag_steps, real_steps, binding.GP_C128, W,
                                     instrument=True)
    log(f"complex128 with per-kernel events: {ms_inst:.1f} ms")

    # dominant kernel: largest total time among the sweeps.  Algorithmic bytes
    # are one read and one write of the grid per sweep (16 + 16 per point in
    # complex128); the fused x+y kernel performs two sweeps per launch but keeps
    # the x result on chip, so its compulsory traffic is one read and one write.
    sweeps = {k: v for k, v in kt.items() if k.startswith("sweep")}
    dom = max(sweeps, key=lambda k: sweeps[k][1])
    cnt, tot = sweeps[dom]
    avg_ms = tot / cnt
    nsweeps = 2 if dom == "sweep_xy" else 1
    alg_bytes = 32 * w.points * nsweeps
    compulsory = 32 * w.points
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = None
    tf_path = os.path.join(ROOT, "profiles", f"traffic_{dom}_256cubed_c128.json")
    if os.path.exists(tf_path):
        tf = json.load(open(tf_path))
        if tf.get("kernel_source_hash") == kernel_source_hash():
            traffic = tf.get("bytes_per_launch")
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "launches": cnt, "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": alg_bytes,
            "sweeps_per_launch": nsweeps, "compulsory_bytes_per_launch": compulsory,
            "compulsory_GBps": round(compulsory / (avg_ms * 1e-3) / 1e9, 1),
            "measured_traffic_GBps": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1)}
    step_bytes = 96 * w.points
    hbm_frac = step_bytes * K / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS
    per_kernel = {k: {"launches": c, "avg_ms": round(t / c, 5)} for k, (c, t) in kt.items()}
    log(f"per-kernel: {per_kernel}")

    fp32 = None
    if not args.no_fp32:
        ms32, _, mu32, real32, _ = timed_run(torch, binding, w, psi.to(torch.complex64), imag_steps, real_steps,
                                             binding.GP_C64, W, instrument=False)
        v32 = w.points * K / (ms32 * 1e-3)
        fp32 = {"value": v32, "ms_per_step": ms32 / K, "dtype": "c64 bulk, f64 reductions",
                "hbm_frac": 48 * w.points * K / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                "mu_rel_err_vs_c128": abs(mu32["mu"] - mu64["mu"]) / abs(mu64["mu"]),
                "energy_rel_err_vs_c128": abs(mu32["energy"] - mu64["energy"]) / abs(mu64["energy"]),
                "norm_after_real_phase": real32["norm"],
                "energy_rel_err_after_real_phase": abs(real32["energy"] - real64["energy"]) / abs(real64["energy"])}
        log(f"complex64: {ms32:.1f} ms -> {v32:.3e} point-updates/s, mu err {fp32['mu_rel_err_vs_c128']:.2e}")

    batch = None
    if not args.no_forms:
        batch = batch_form(torch, binding, inputs)
        log(f"batch form: {batch['value']:.3e} point-updates/s ({batch['ms_per_step']:.3f} ms/step, "
            f"config {batch['config']})")
    adj = None
    if not args.no_forms:
        adj = adjoint_form(torch, binding, inputs)
        log(f"adjoint form: c128 gradient {adj['c128']['gradient_s']:.3f} s, c64 {adj['c64']['gradient_s']:.3f} s")

    gbps = copy_probe(torch, binding)
    log(f"copy probe: {gbps:.0f} GB/s")
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(w, psi_np, args.cpu_seconds)
        log(f"CPU oracle: {cpu['value']:.3e} point-updates/s on {cpu['cores']} threads")

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
        "hbm_frac": round(hbm_frac, 4),
        "ms_per_step_with_kernel_events": ms_inst / K,
        "mu_after_imag": mu64["mu"],
        "roofline": roof,
        "per_kernel": per_kernel,
        "copy_probe_GBps": round(gbps, 1),
        "fp32": fp32,
        "batch": batch,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
