"""Host checks of the precomputed Thomas tables (no GPU): they factor the
Crank-Nicolson system correctly, the windowed back substitution the sweep
kernels perform reproduces a dense solve, and in real time the rounded tables
keep the map unitary."""
import numpy as np
import pytest

from paper_1709_04423_amd import binding

BLOCK = 4  # points per block of the strided-axis solver (16 for transposed x lines)


def cn_dense(n, dx, dt, mode, adjoint=False):
    r = dt / (4 * dx * dx)
    b, e = (1 + 2j * r, -1j * r) if mode == binding.GP_REAL else (1 + 2 * r + 0j, -r + 0j)
    if adjoint:
        b, e = np.conj(b), np.conj(e)
    A = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, e), 1) + np.diag(np.full(n - 1, e), -1)
    B = np.diag(np.full(n, 2 - b)) - np.diag(np.full(n - 1, e), 1) - np.diag(np.full(n - 1, e), -1)
    return A, B


def solve_with_table(c, beta, u):
    """Full Thomas solve of the scaled system with the table (no window)."""
    n = len(u)
    up = np.concatenate([[0], u, [0]])
    rhs = beta * u - (up[:-2] + up[2:])
    y = np.zeros(n, complex)
    prev = 0
    for p in range(n):
        y[p] = (rhs[p] - prev) * c[p]
        prev = y[p]
    v = np.zeros(n, complex)
    nxt = 0
    for p in range(n - 1, -1, -1):
        v[p] = y[p] - c[p] * nxt
        nxt = v[p]
    return v


def solve_windowed(c, beta, u, K, block=BLOCK, segs=1):
    """The kernels' streaming algorithm: blocks of `block` points, forward
    elimination as values arrive, back substitution per output block started K
    points past it with zero, rows past the line zero; optionally the line is
    split into `segs` segments, each starting its elimination D blocks before
    its first output block from y = 0."""
    n = len(u)
    D = (K + 1 + block - 1) // block
    nblocks = (n + block - 1) // block
    rows = (nblocks + D) * block + 1
    ctab = np.zeros(rows, complex)
    btab = np.zeros(rows, complex)
    ctab[1:n + 1] = c
    btab[1:n + 1] = beta
    ext = np.zeros((nblocks + D) * block + 2, complex)
    ext[:n] = u
    out = np.zeros(n, complex)
    for s in range(segs):
        o_lo, o_hi = s * nblocks // segs, (s + 1) * nblocks // segs
        j0 = max(0, o_lo - D)
        y = {}
        um1 = u0 = yprev = 0
        if j0 > 0:
            um1, u0 = ext[j0 * block - 2], ext[j0 * block - 1]
        for j in range(j0, o_hi + D):
            for k in range(block):
                q = j * block + k
                up1 = ext[q]
                rhs = btab[q] * u0 - (um1 + up1)
                d = (rhs - yprev) * ctab[q]
                y[q - 1] = d
                yprev, um1, u0 = d, u0, up1
            o = j - D
            if o_lo <= o < o_hi:
                ob = o * block
                v = 0
                for t in range(ob + (D + 1) * block - 2, ob - 1, -1):
                    v = y[t] - ctab[t + 1] * v
                    if t < ob + block and t < n:
                        out[t] = v
    return out


CASES = [(1, 0.05, 1e-3), (7, 0.1, 1e-2), (37, 0.2, 1e-2), (256, 0.05, 2e-4), (300, 0.05, 1e-3),
         (128, 0.1, 1e-3), (50, 0.05, 3e-3)]


@pytest.mark.parametrize("mode", [binding.GP_IMAG, binding.GP_REAL])
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_table_factorises_cn_fp64(mode, adjoint, case):
    n, dx, dt = case
    if adjoint and mode == binding.GP_IMAG:
        pytest.skip("the adjoint is defined for real time")
    c, beta, K, rho = binding.thomas_table(n, dx, dt, mode, binding.GP_C128, adjoint)
    A, B = cn_dense(n, dx, dt, mode, adjoint)
    u = np.random.default_rng(n).standard_normal(n) + 1j * np.random.default_rng(n + 1).standard_normal(n)
    ref = np.linalg.solve(A, B @ u)
    got = solve_with_table(c, beta, u)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert K >= 0
    for block, segs in ((4, 1), (4, 3), (16, 1)):
        win = solve_windowed(c, beta, u, K, block, segs)
        assert np.max(np.abs(win - ref)) <= 1e-14 * np.max(np.abs(ref)), (block, segs)


@pytest.mark.parametrize("mode", [binding.GP_IMAG, binding.GP_REAL])
def test_table_fp32_rounding(mode):
    n, dx, dt = 256, 0.05, 2e-4
    c, beta, K, rho = binding.thomas_table(n, dx, dt, mode, binding.GP_C64)
    assert np.all(c.real.astype(np.float32) == c.real) and np.all(c.imag.astype(np.float32) == c.imag)
    A, B = cn_dense(n, dx, dt, mode)
    u = np.random.default_rng(3).standard_normal(n) + 0j
    ref = np.linalg.solve(A, B @ u)
    got = solve_windowed(c, beta, u, K)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_real_time_fp32_table_is_unitary_in_the_interior():
    # delta_p = 1/c'_p + c'_{p-1} of the rounded table: Im beta_p must equal Im delta_p
    # to far better than FP32 precision, so that the map's Hermitian parts agree
    n, dx, dt = 256, 0.05, 2e-4
    c, beta, K, rho = binding.thomas_table(n, dx, dt, binding.GP_REAL, binding.GP_C64)
    cl = c.astype(np.clongdouble)
    delta = 1 / cl + np.concatenate([[0], cl[:-1]])
    assert np.max(np.abs(beta.imag - delta.imag.astype(np.float64)) / np.abs(delta.imag)) < 1e-14
    # plain rounding of Im beta to FP32 would leave ~1e-8; the map built from the
    # FP32 values stays norm-preserving on a smooth interior mode to ~1e-13
    A_eff = np.diag(delta.astype(complex)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    B_eff = np.diag(beta) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    x = np.arange(n) - n / 2
    u = np.exp(-(x / 30.0) ** 2) + 0j
    v = np.linalg.solve(A_eff, B_eff @ u)
    assert abs(np.linalg.norm(v) / np.linalg.norm(u) - 1) < 1e-13


@pytest.mark.parametrize("mode", [binding.GP_IMAG, binding.GP_REAL])
@pytest.mark.parametrize("prec", [binding.GP_C128, binding.GP_C64])
def test_windowed_solve_with_one_window_per_segment(mode, prec):
    # small grids are split down to segments of D + 1 blocks; each still matches
    # the dense solve to the window bound
    n, dx, dt = 256, 0.05, 1e-3
    c, beta, K, rho = binding.thomas_table(n, dx, dt, mode, prec)
    A, B = cn_dense(n, dx, dt, mode)
    u = np.random.default_rng(11).standard_normal(n) + 1j * np.random.default_rng(12).standard_normal(n)
    ref = np.linalg.solve(A, B @ u) if prec == binding.GP_C128 else solve_with_table(c, beta, u)
    D = (K + 1 + BLOCK - 1) // BLOCK
    segs = ((n + BLOCK - 1) // BLOCK) // (D + 1)
    got = solve_windowed(c, beta, u, K, BLOCK, segs)
    tol = 1e-14 if prec == binding.GP_C128 else 1e-12
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def test_window_depth_and_exact_fallback():
    # K = D*4 - 1 for the smallest D whose window meets the bound
    _, _, K, rho = binding.thomas_table(256, 0.05, 2e-4, binding.GP_REAL, binding.GP_C128)
    assert 0.019 < rho < 0.021 and rho ** (K + 1) <= 2.0 ** -60 and (K + 1) % 4 == 0
    assert rho ** (K + 1 - 4) > 2.0 ** -60
    _, _, K32, rho32 = binding.thomas_table(256, 0.05, 2e-4, binding.GP_REAL, binding.GP_C64)
    assert rho32 ** (K32 + 1) <= 2.0 ** -44 and (K32 + 1) % 4 == 0 and K32 <= K
    _, _, K2, rho2 = binding.thomas_table(256, 0.05, 1e-3, binding.GP_REAL, binding.GP_C128)
    assert K2 == 19 and rho2 ** 16 > 2.0 ** -60
    _, _, Kx, rho_x = binding.thomas_table(64, 0.05, 0.2, binding.GP_REAL, binding.GP_C128)
    assert Kx == -1 and rho_x > 0.8


def solve_scan(c, beta, u, lanes=64, steps=None):
    """The x kernel's algorithm: Q points per lane, per-lane affine maps,
    Hillis-Steele scans of `steps` steps (default: full), then local apply."""
    n = len(u)
    Q = 1
    while Q * lanes < n:
        Q *= 2
    S = 6 if steps is None else steps
    N = Q * lanes
    up = np.zeros(N + 2, complex)
    up[1:n + 1] = u
    cz = np.zeros(N, complex)
    bz = np.zeros(N, complex)
    cz[:n], bz[:n] = c, beta
    rhs = bz * up[1:N + 1] - (up[0:N] + up[2:N + 2])
    a, f = -cz, cz * rhs
    A = np.ones(lanes, complex)
    F = np.zeros(lanes, complex)
    for L in range(lanes):
        Ai, Fi = 1.0 + 0j, 0j
        for i in range(Q):
            p = L * Q + i
            Fi = a[p] * Fi + f[p]
            Ai = a[p] * Ai
        A[L], F[L] = Ai, Fi
    for s in range(S):
        d = 1 << s
        A2, F2 = A.copy(), F.copy()
        for L in range(d, lanes):
            F2[L] = A[L] * F[L - d] + F[L]
            A2[L] = A[L] * A[L - d]
        A, F = A2, F2
    y = np.zeros(N, complex)
    for L in range(lanes):
        yy = F[L - 1] if L > 0 else 0
        for i in range(Q):
            p = L * Q + i
            yy = a[p] * yy + f[p]
            y[p] = yy
    B = np.ones(lanes, complex)
    G = np.zeros(lanes, complex)
    for L in range(lanes):
        Bi, Gi = 1.0 + 0j, 0j
        for i in range(Q - 1, -1, -1):
            p = L * Q + i
            Gi = a[p] * Gi + y[p]
            Bi = a[p] * Bi
        B[L], G[L] = Bi, Gi
    for s in range(S):
        d = 1 << s
        B2, G2 = B.copy(), G.copy()
        for L in range(lanes - d):
            G2[L] = B[L] * G[L + d] + G[L]
            B2[L] = B[L] * B[L + d]
        B, G = B2, G2
    v = np.zeros(N, complex)
    for L in range(lanes):
        vv = G[L + 1] if L + 1 < lanes else 0
        for i in range(Q - 1, -1, -1):
            p = L * Q + i
            vv = a[p] * vv + y[p]
            v[p] = vv
    return v[:n]


@pytest.mark.parametrize("mode", [binding.GP_IMAG, binding.GP_REAL])
@pytest.mark.parametrize("case", [(1, 0.05, 1e-3), (37, 0.2, 1e-2), (256, 0.05, 2e-4), (300, 0.05, 1e-3),
                                  (512, 0.05, 5e-4), (64, 0.05, 0.2)])
def test_x_scan_algorithm(mode, case):
    n, dx, dt = case
    c, beta, K, rho = binding.thomas_table(n, dx, dt, mode, binding.GP_C128)
    A, B = cn_dense(n, dx, dt, mode)
    u = np.random.default_rng(n + 7).standard_normal(n) + 1j * np.random.default_rng(n + 8).standard_normal(n)
    ref = np.linalg.solve(A, B @ u)
    assert np.max(np.abs(solve_scan(c, beta, u) - ref)) <= 1e-14 * np.max(np.abs(ref))
    # truncated scan: the plan's step count reaches Kmin + 1 points back
    kmin = 0
    while rho > 0 and rho ** (kmin + 1) > 2.0 ** -60:
        kmin += 1
    Q = 1
    while Q * 64 < n:
        Q *= 2
    S = 0
    while S < 6 and Q * (1 << S) <= kmin:
        S += 1
    got = solve_scan(c, beta, u, steps=S)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
