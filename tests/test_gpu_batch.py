"""Batched form on the GPU: many uneven 2D problems advanced together, phased
and persistent, against each problem run alone and against the FP64 oracle.
The mix has y lines for both batched y solvers: the scan solver (up to 512
points) and the windowed one (the 600-point lines)."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1709_04423_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04423_amd import binding
    binding.lib()
    return binding


SIZES = [(128, 96), (64, 200), (192, 128), (100, 37), (256, 64), (40, 300), (70, 600)]  # x first, ragged
OMEGA = [(1.0, 0.7), (1.0, 1.3), (1.0, 2.0), (1.0, 0.5), (1.0, 1.1), (1.0, 1.6), (1.0, 0.9)]
G = [30.0, 120.0, 400.0, 10.0, 250.0, 60.0, 80.0]
DX, DT = 0.1, 1e-3


def initial(k, dtype):
    n = SIZES[k]
    psi = inputs.gaussian(n, DX, OMEGA[k]) + 0.03 * inputs.random_field(n[::-1], 100 + k)
    return torch.from_numpy(psi.astype(dtype)).to("cuda")


def run_batch(gp, mode, prec, cfg, steps=7):
    dtype = np.complex128 if prec == gp.GP_C128 else np.complex64
    b = gp.Batch(SIZES, DX, DT, mode, OMEGA, G, prec)
    b.set_config(**cfg)
    psis = [initial(k, dtype) for k in range(len(SIZES))]
    b.step(psis, steps)
    torch.cuda.synchronize()
    return b, [p.cpu().numpy() for p in psis]


def run_alone(gp, mode, prec, steps=7):
    dtype = np.complex128 if prec == gp.GP_C128 else np.complex64
    out = []
    for k in range(len(SIZES)):
        plan = gp.Plan(SIZES[k], DX, DT, mode, OMEGA[k], G[k], prec)
        psi = initial(k, dtype)
        plan.step(psi, steps)
        out.append(psi.cpu().numpy())
    return out


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_phased_batch_matches_problems_run_alone(gp, mode, prec):
    say(f"batch phased mode={mode} prec={prec}")
    _, got = run_batch(gp, mode, prec, dict(persistent=0, lines=2, ysegs=4))
    ref = run_alone(gp, mode, prec)
    tol = 1e-13 if prec == 0 else 1e-5
    for k in range(len(SIZES)):
        assert max_rel(got[k], ref[k]) <= tol, k


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("grid", [3, 64, 1024])
def test_persistent_batch_equals_phased_bitwise(gp, prec, grid):
    # same items, same arithmetic per item: identical bits whatever the grid
    say(f"batch persistent grid={grid} prec={prec}")
    cfg = dict(lines=4, ysegs=2)
    _, a = run_batch(gp, 1, prec, dict(persistent=0, **cfg))
    _, b = run_batch(gp, 1, prec, dict(persistent=1, grid=grid, **cfg))
    for k in range(len(SIZES)):
        assert np.array_equal(a[k], b[k]), k


def test_batch_matches_oracle(gp):
    say("batch vs oracle")
    _, got = run_batch(gp, 1, gp.GP_C128, dict(persistent=1, grid=256, lines=4, ysegs=4), steps=5)
    for k in (0, 3, 5, 6):
        psi0 = initial(k, np.complex128).cpu().numpy()
        ref = oracle.step(psi0, DX, DT, oracle.REAL, OMEGA[k], G[k], 5)
        assert max_rel(got[k], ref) <= 1e-12, k
    _, got = run_batch(gp, 0, gp.GP_C128, dict(persistent=0, lines=1, ysegs=8), steps=5)
    for k in (1, 4, 6):
        psi0 = initial(k, np.complex128).cpu().numpy()
        ref = oracle.step(psi0, DX, DT, oracle.IMAG, OMEGA[k], G[k], 5)
        assert max_rel(got[k], ref) <= 1e-12, k


def test_persistent_wait_limit_reports_timeout(gp):
    # a wait bound of one poll: some dependency is not met at once, the launch
    # stops taking items and finishes, and the step reports GP_ETIMEOUT
    b = gp.Batch(SIZES, DX, DT, 1, OMEGA, G, gp.GP_C64)
    b.set_config(persistent=1, grid=1024, lines=1, ysegs=8)
    b.set_wait_limit(1)
    psis = [initial(k, np.complex64) for k in range(len(SIZES))]
    with pytest.raises(gp.GpError) as e:
        b.step(psis, 50)
    assert e.value.status == gp.GP_ETIMEOUT
    # the grids are undefined after a timeout and the step indices did not move:
    # reload them, and with a normal bound the batch gives what a fresh one does
    b.set_wait_limit(1 << 22)
    psis = [initial(k, np.complex64) for k in range(len(SIZES))]
    b.step(psis, 2)
    _, ref = run_batch(gp, 1, gp.GP_C64, dict(persistent=1, grid=1024, lines=1, ysegs=8), steps=2)
    for k in range(len(SIZES)):
        assert np.array_equal(psis[k].cpu().numpy(), ref[k]), k


def test_autotune_and_cache(gp, tmp_path):
    sizes = [p.n for p in inputs.batch_problems(count=12)]
    b = gp.Batch(sizes, 0.05, 1e-3, 1, [(1.0, 1.2)] * 12, [100.0] * 12, gp.GP_C64)
    cache = str(tmp_path / "tune.txt")
    cfg = b.autotune(cache)
    say(f"autotuned {cfg}")
    assert cfg["lines"] in (1, 2, 4) and cfg["ysegs"] in (1, 2, 4, 8, 16, 32)
    assert open(cache).read().count("\n") == 1
    b2 = gp.Batch(sizes, 0.05, 1e-3, 1, [(1.0, 1.2)] * 12, [100.0] * 12, gp.GP_C64)
    assert b2.autotune(cache) == cfg  # read back without timing
    assert open(cache).read().count("\n") == 1
    sides = sorted({n for s in sizes for n in s})
    assert [b2.side_config(n) for n in sides] == [b.side_config(n) for n in sides]  # per-length settings too
    say(f"per side {[(n, b.side_config(n)) for n in sides]}")
    psis = [torch.zeros(s[::-1], dtype=torch.complex64, device="cuda") for s in sizes]
    b.step(psis, 3)


def test_per_side_settings_change_grouping_not_results(gp):
    # real time: every scan-solved line is solved alone, so regrouping lines
    # into items leaves the bits unchanged; other y segments of a windowed line
    # move its results only within the window bound
    _, ref = run_batch(gp, 1, gp.GP_C64, dict(persistent=0, lines=2, ysegs=4))
    dtype = np.complex64
    b = gp.Batch(SIZES, DX, DT, 1, OMEGA, G, gp.GP_C64)
    b.set_config(persistent=0, lines=2, ysegs=4)
    b.set_side_config(128, 8, 1)   # x lines of problem 0 and y lines of problem 2
    b.set_side_config(600, 1, 16)  # the windowed y lines of problem 6
    assert b.side_config(128) == {"lines": 8, "ysegs": 1}
    assert b.side_config(96) == {"lines": 2, "ysegs": 4}  # the defaults
    psis = [initial(k, dtype) for k in range(len(SIZES))]
    b.step(psis, 7)
    for k in range(len(SIZES)):
        got = psis[k].cpu().numpy()
        assert np.array_equal(got, ref[k]) if SIZES[k][1] <= 512 else max_rel(got, ref[k]) <= 1e-6, k
    b.set_config(persistent=0, lines=4, ysegs=2)  # clears the per-length settings
    assert b.side_config(128) == {"lines": 4, "ysegs": 2}
    with pytest.raises(gp.GpError):
        b.set_side_config(0, 1, 1)
    with pytest.raises(gp.GpError):
        b.set_side_config(128, 65, 1)
