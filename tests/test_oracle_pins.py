"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: textbook rational weights, exact
polynomial reproduction, the closed-form discrete dispersion relation, the analytic Green's
function, exact conservation and reversal identities, the adjoint identity, finite differences and
brute force.  A dropped term, a wrong sign or a swapped axis anywhere in the oracle fails at least
one of them.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle


def _load_textbook():
    """Centred second-derivative weights, the published table (Fornberg 1988, Table 1), from
    tests/golden/fornberg_second_derivative.txt: {R: [c_0, ..., c_R]} as exact fractions."""
    path = os.path.join(os.path.dirname(__file__), "golden", "fornberg_second_derivative.txt")
    table = {}
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r, *cs = line.split()
                table[int(r)] = [Fr(c) for c in cs]
    return table


TEXTBOOK = _load_textbook()


def test_textbook_table_complete():
    assert sorted(TEXTBOOK) == [1, 2, 3, 4]
    assert all(len(TEXTBOOK[r]) == r + 1 for r in TEXTBOOK)


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
def test_coefficients_match_textbook(radius):
    c = oracle.fd_coefficients(radius)
    ref = np.array([float(x) for x in TEXTBOOK[radius]])
    np.testing.assert_allclose(c, ref, rtol=2e-15, atol=1e-16)


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6])
def test_coefficients_taylor_moments(radius):
    """sum_k c_k k^(2j) over the full stencil is 0, 2, 0, ..., 0 for j < R+1 and nonzero at j = R+1."""
    c = oracle.fd_coefficients(radius)
    for j in range(radius + 2):
        mom = c[0] * (1.0 if j == 0 else 0.0) + 2.0 * sum(c[m] * float(m) ** (2 * j) for m in range(1, radius + 1))
        expect = 2.0 if j == 1 else 0.0
        if j <= radius:
            assert abs(mom - expect) < 1e-11 * max(1.0, float(radius) ** (2 * j)), (j, mom)
        else:
            assert abs(mom) > 1.0, (j, mom)


def test_radius4_next_moment_exact():
    """The first non-vanishing moment of the 8th-order weights (exact rationals): the truncation error
    of the 1-D operator is (2 * sum c_m m^10 / 10!) h^8 f^(10) = -(h^8/3150) f^(10)."""
    c = TEXTBOOK[4]
    mom = 2 * sum(c[m] * m**10 for m in range(1, 5))
    assert mom / math.factorial(10) == Fr(-1, 3150)
    np.testing.assert_allclose(2 * sum(oracle.fd_coefficients(4)[m] * m**10 for m in range(1, 5)), float(mom),
                               rtol=1e-12)


def test_stability_limit_closed_form():
    # S = sum |c| over the full stencil: 2048/315 (R=4), 16/3 (R=2); C* = 2/sqrt(3S).
    assert abs(oracle.stability_limit(4) - 2.0 / math.sqrt(3.0 * 2048.0 / 315.0)) < 1e-14
    assert abs(oracle.stability_limit(2) - 0.5) < 1e-14
    assert abs(oracle.stable_dt(4, 10.0, 2000.0) - 1.132139e-3) < 1e-9
    assert abs(oracle.stable_dt(4, 10.0, 4500.0) - 0.503173e-3) < 1e-9


@pytest.mark.parametrize("radius", [2, 4])
def test_laplacian_exact_on_polynomials(radius, oracle_threads):
    """A radius-R centred stencil differentiates polynomials of degree <= 2R+1 exactly, so away from
    the boundary L u / h^2 equals the analytic Laplacian (distinct polynomial on each axis and a
    mixed term, on a non-cubic grid)."""
    nx, ny, nz = 23, 19, 17
    h = 0.5
    deg = 2 * radius + 1
    x = (np.arange(nx) - 11) * h
    y = (np.arange(ny) - 9) * h
    z = (np.arange(nz) - 8) * h
    X, Y, Z = x[None, None, :], y[None, :, None], z[:, None, None]
    rng = np.random.default_rng(7)
    a, b, cz = rng.standard_normal((3, deg + 1)) / 50.0
    poly = lambda co, t: sum(co[p] * t**p for p in range(deg + 1))
    dpoly2 = lambda co, t: sum(co[p] * p * (p - 1) * t ** (p - 2) for p in range(2, deg + 1))
    u = poly(a, X) + poly(b, Y) + poly(cz, Z) + 0.1 * X**2 * Y**3 * Z
    exact = dpoly2(a, X) + dpoly2(b, Y) + dpoly2(cz, Z) + 0.1 * (2 * Y**3 * Z + 6 * X**2 * Y * Z)
    exact = np.broadcast_to(exact, u.shape)
    num = oracle.laplacian(u, radius, False, oracle_threads) / h**2
    r = radius
    inner = (slice(r, nz - r), slice(r, ny - r), slice(r, nx - r))
    np.testing.assert_allclose(num[inner], exact[inner], rtol=1e-8, atol=1e-8 * np.max(np.abs(exact)))


@pytest.mark.parametrize("radius,order", [(4, 8), (2, 4)])
def test_laplacian_convergence_order(radius, order, oracle_threads):
    errs = []
    for h in (0.5, 0.25, 0.125):
        n = int(round(16 / h)) + 1
        x = (np.arange(n) - (n - 1) / 2) * h
        X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
        r2 = X**2 + Y**2 + Z**2
        f = np.exp(-r2 / 2.0)
        exact = f * (r2 - 3.0)
        num = oracle.laplacian(f, radius, False, oracle_threads) / h**2
        errs.append(np.max(np.abs(num - exact)[r2 < 9.0]))
    slope = math.log2(errs[1] / errs[2])
    assert abs(slope - order) < 0.4, (errs, slope)


def _textbook_symbol(kd_h, radius=4):
    c = [float(v) for v in TEXTBOOK[radius]]
    return c[0] + 2.0 * sum(c[m] * math.cos(m * kd_h) for m in range(1, radius + 1))


def test_discrete_dispersion_relation():
    """On a periodic box the standing wave cos(k.x) with p^{-1} = p^0 cos(w dt) evolves exactly as
    cos(k.x) cos(w n dt), where sin(w dt / 2) = (v dt / 2h) sqrt(-sum_d symbol(k_d h))."""
    nx, ny, nz = 16, 12, 20
    h, v = 10.0, 2000.0
    dt = 0.5 * 0.4528555233184200 * h / v
    mx, my, mz = 3, 2, 5
    kx, ky, kz = (2 * math.pi * m / (n * h) for m, n in ((mx, nx), (my, ny), (mz, nz)))
    lam = sum(_textbook_symbol(kd * h) for kd in (kx, ky, kz))
    w = 2.0 / dt * math.asin(v * dt / (2 * h) * math.sqrt(-lam))
    x, y, z = np.arange(nx) * h, np.arange(ny) * h, np.arange(nz) * h
    phase = kx * x[None, None, :] + ky * y[None, :, None] + kz * z[:, None, None]
    p0 = np.cos(phase)
    kap = np.full((nz, ny, nx), (v * dt / h) ** 2)
    nsteps = 200
    out = oracle.forward(kap, None, nsteps, u_cur=p0, u_prv=p0 * math.cos(w * dt), periodic=True)
    assert np.max(np.abs(out["u_cur"] - p0 * math.cos(w * nsteps * dt))) < 1e-12
    assert np.max(np.abs(out["u_prv"] - p0 * math.cos(w * (nsteps - 1) * dt))) < 1e-12


def test_sponge_scalar_recurrence_closed_form(oracle_threads):
    """With kappa = 0 every cell obeys u^{n+1} = g (2 u^n - g u^{n-1}), whose characteristic
    polynomial (r - g)^2 has the double root g, so u^n = (A + B n) g^n with A = u^0 and
    B = u^0 - g u^{-1}.  Pins where the sponge enters both time levels, cell by cell, for
    different per-axis factors."""
    rng = np.random.default_rng(21)
    nz, ny, nx = 6, 7, 9
    gx, gy, gz = rng.uniform(0.6, 1.0, nx), rng.uniform(0.6, 1.0, ny), rng.uniform(0.6, 1.0, nz)
    gx[0] = 1.0
    g = gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    u0 = rng.standard_normal((nz, ny, nx))
    um = rng.standard_normal((nz, ny, nx))
    nsteps = 40
    out = oracle.forward(np.zeros((nz, ny, nx)), (gx, gy, gz), nsteps, u_cur=u0, u_prv=um, nthreads=oracle_threads)
    A, B = u0, u0 - g * um
    for n, key in ((nsteps, "u_cur"), (nsteps - 1, "u_prv")):
        ref = (A + B * n) * g ** n
        assert np.max(np.abs(out[key] - ref)) <= 1e-13 * np.max(np.abs(A) + np.abs(B) * n)


def test_adjoint_sponge_scalar_recurrence_closed_form():
    """With kappa = 0 the transposed recursion is mu^m = 2 g mu^{m+1} - g^2 mu^{m+2}: the same double
    root g, so mu^{N+1-j} = (A + B j) g^j with A = mu^{N+1} and B = mu^{N+1} - g mu^{N+2}.  Pins the
    -g^2 mu term and the 2 g factor of the adjoint step."""
    rng = np.random.default_rng(22)
    nz, ny, nx = 5, 6, 8
    gx, gy, gz = rng.uniform(0.6, 1.0, nx), rng.uniform(0.6, 1.0, ny), rng.uniform(0.6, 1.0, nz)
    g = gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    a0 = rng.standard_normal((nz, ny, nx))      # mu one level later
    b0 = rng.standard_normal((nz, ny, nx))      # mu two levels later
    mu_a, mu_b = a0, b0
    kap = np.zeros((nz, ny, nx))
    A, B = a0, a0 - g * b0
    for j in range(1, 31):
        mu = oracle.adjoint_step(mu_a, mu_b, kap, (gx, gy, gz))
        mu_b, mu_a = mu_a, mu
        ref = (A + B * j) * g ** j
        assert np.max(np.abs(mu - ref)) <= 1e-13 * np.max(np.abs(A) + np.abs(B) * j), j


def _damped_mode(a0, am1, g, c, n):
    """n-th term of a^{n+1} = g (2 + q) a^n - g^2 a^{n-1} with q = kappa lambda: a^n = g^n (A cos n t
    + B sin n t), cos t = 1 + q / 2 (an oscillating mode, |1 + q/2| < 1)."""
    t = math.acos(c)
    A = a0
    B = (A * math.cos(t) - g * am1) / math.sin(t)
    return g ** n * (A * math.cos(n * t) + B * math.sin(n * t))


@pytest.mark.parametrize("adjoint", [False, True])
def test_damped_standing_wave_closed_form(adjoint):
    """A standing wave on a periodic box with constant sponge factor g and constant kappa: L p = lambda p
    with the exact discrete symbol, so the forward update (and the transposed one, which for constant
    g and kappa is the same map) multiplies the mode amplitude by the scalar recurrence
    a^{n+1} = g (2 + kappa lambda) a^n - g^2 a^{n-1}, solved in closed form.  Pins where g sits
    relative to kappa L (outside both), in both directions of time."""
    nx, ny, nz = 16, 12, 10
    h, v = 10.0, 2500.0
    dt = oracle.stable_dt(4, h, v)
    modes = (3, 2, 1)
    kx, ky, kz = (2 * math.pi * m / (n * h) for m, n in zip(modes, (nx, ny, nz)))
    lam = sum(_textbook_symbol(kd * h) for kd in (kx, ky, kz))
    kap = oracle.kappa_field(np.full((nz, ny, nx), v), dt, h)
    q = kap[0, 0, 0] * lam
    x, y, z = np.arange(nx) * h, np.arange(ny) * h, np.arange(nz) * h
    p = np.cos(kx * x[None, None, :] + ky * y[None, :, None] + kz * z[:, None, None])
    gxv, gyv, gzv = 0.99, 0.985, 0.995
    sponge = (np.full(nx, gxv), np.full(ny, gyv), np.full(nz, gzv))
    g = gxv * gyv * gzv
    a0, am1 = 1.0, 0.7
    nsteps = 120
    if not adjoint:
        out = oracle.forward(kap, sponge, nsteps, u_cur=a0 * p, u_prv=am1 * p, periodic=True)
        got = out["u_cur"]
    else:
        mu_a, mu_b = a0 * p, am1 * p
        for _ in range(nsteps):
            mu = oracle.adjoint_step(mu_a, mu_b, kap, sponge, periodic=True)
            mu_b, mu_a = mu_a, mu
        got = mu_a
    ref = _damped_mode(a0, am1, g, 1.0 + q / 2.0, nsteps) * p
    assert np.max(np.abs(got - ref)) <= 1e-12
    # the damping really acts: the undamped amplitude differs
    assert np.max(np.abs(got - _damped_mode(a0, am1, 1.0, 1.0 + q / 2.0, nsteps) * p)) > 1e-3


def test_kappa_field_values():
    """kappa = (v dt / h)^2: exact values, and at v_max with dt at half the stability limit
    kappa = (C*/2)^2 = 1 / (3 S) with S = 2048/315 (radius 4), the squared Courant number."""
    assert oracle.kappa_field(np.array([2000.0]), 1e-3, 10.0)[0] == pytest.approx(0.04, rel=1e-15)
    assert oracle.kappa_field(np.array([1500.0]), 2e-3, 20.0)[0] == pytest.approx(0.0225, rel=1e-15)
    v = np.array([[[3000.0, 1500.0], [4500.0, 2250.0]]])
    dt = oracle.stable_dt(4, 10.0, 4500.0)
    kap = oracle.kappa_field(v, dt, 10.0)
    assert kap.shape == v.shape
    assert kap[0, 1, 0] == pytest.approx(315.0 / 6144.0, rel=1e-14)
    np.testing.assert_allclose(kap, (v / 4500.0) ** 2 * 315.0 / 6144.0, rtol=1e-14)


def test_stability_threshold():
    """The checkerboard mode grows above the limit and stays bounded just below it."""
    n = 8
    ii = np.indices((n, n, n)).sum(axis=0)
    mode = np.where(ii % 2 == 0, 1.0, -1.0)
    cstar = 2.0 / math.sqrt(3.0 * 2048.0 / 315.0)
    peaks = {}
    for frac in (0.99, 1.01):
        kap = np.full((n, n, n), (frac * cstar) ** 2)
        out = oracle.forward(kap, None, 400, u_cur=mode, u_prv=mode, periodic=True)
        peaks[frac] = np.max(np.abs(out["u_cur"]))
    assert peaks[0.99] < 2.0
    assert peaks[1.01] > 1e3


def test_energy_conservation(oracle_threads):
    """With g = 1 and no source, E^{n+1/2} = <du, du/kappa> - <u^{n+1}, L u^n> is an exact invariant
    of leapfrog with a symmetric L (Dirichlet ghosts), for any variable kappa."""
    rng = np.random.default_rng(11)
    shape = (10, 12, 14)
    cstar = oracle.stability_limit(4)
    kap = (cstar * rng.uniform(0.3, 0.9, shape)) ** 2
    u0 = rng.standard_normal(shape)
    um = u0 + 0.05 * rng.standard_normal(shape)
    energies = []
    u_prv, u_cur = um, u0
    for n in range(1000):
        u_nxt = oracle.step(u_cur, u_prv, kap, None, 4, False, 1)
        du = u_nxt - u_cur
        e = np.sum(du * du / kap) - np.sum(u_nxt * oracle.laplacian(u_cur, 4, False, 1))
        energies.append(e)
        u_prv, u_cur = u_cur, u_nxt
    energies = np.array(energies)
    assert np.max(np.abs(energies - energies[0])) / abs(energies[0]) < 1e-12


def test_energy_not_conserved_with_wrong_kappa_placement():
    """Control for the energy pin: putting kappa inside L (L(kappa u)) breaks the invariant, so the
    pin does see where kappa sits."""
    rng = np.random.default_rng(12)
    shape = (8, 9, 10)
    kap = (oracle.stability_limit(4) * rng.uniform(0.3, 0.9, shape)) ** 2
    u0 = rng.standard_normal(shape)
    u_prv, u_cur = u0.copy(), u0
    es = []
    for _ in range(50):
        u_nxt = 2 * u_cur - u_prv + oracle.laplacian(kap * u_cur, 4, False, 1)
        du = u_nxt - u_cur
        es.append(np.sum(du * du / kap) - np.sum(u_nxt * oracle.laplacian(u_cur, 4, False, 1)))
        u_prv, u_cur = u_cur, u_nxt
    assert np.max(np.abs(np.array(es) - es[0])) / abs(es[0]) > 1e-6


def test_time_reversal():
    """With g = 1 and no source the update is its own inverse: step(u^n, u^{n+1}) = u^{n-1}."""
    rng = np.random.default_rng(13)
    shape = (12, 10, 14)
    kap = (oracle.stability_limit(4) * rng.uniform(0.4, 0.9, shape)) ** 2
    u0 = rng.standard_normal(shape)
    um = rng.standard_normal(shape)
    fwd = oracle.forward(kap, None, 100, u_cur=u0, u_prv=um)
    back = oracle.forward(kap, None, 100, u_cur=fwd["u_prv"], u_prv=fwd["u_cur"])
    np.testing.assert_allclose(back["u_cur"], um, atol=1e-10 * np.max(np.abs(um)))
    np.testing.assert_allclose(back["u_prv"], u0, atol=1e-10 * np.max(np.abs(u0)))


def test_threads_bitwise(oracle_threads):
    rng = np.random.default_rng(14)
    shape = (20, 18, 22)
    kap = (oracle.stability_limit(4) * rng.uniform(0.2, 0.9, shape)) ** 2
    u, up = rng.standard_normal((2,) + shape)
    g = [oracle.sponge_profile(n, 4) for n in (22, 18, 20)]
    a = oracle.step(u, up, kap, g, 4, False, 1)
    b = oracle.step(u, up, kap, g, 4, False, oracle_threads)
    assert np.array_equal(a, b)


def test_axis_permutation_symmetry(oracle_threads):
    """A cube with a centred source, constant velocity and the same sponge on every axis is invariant
    under permutations of x, y and z."""
    n, h, v = 32, 10.0, 2000.0
    dt = oracle.stable_dt(4, h, v)
    kap = oracle.kappa_field(np.full((n, n, n), v), dt, h)
    g = oracle.sponge_profile(n, 8)
    amp = oracle.ricker(np.arange(60) * dt, 15.0)[:, None]
    out = oracle.forward(kap, (g, g, g), 60, src_ijk=[(16, 16, 16)], src_w=[oracle.injection_weight(v, dt, h)],
                         src_amp=amp, nthreads=oracle_threads)
    u = out["u_cur"]
    scale = np.max(np.abs(u))
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        assert np.max(np.abs(np.transpose(u, perm) - u)) <= 1e-13 * scale


def test_sponge_profile_properties():
    n, w, alpha = 64, 16, 0.015
    g = oracle.sponge_profile(n, w, alpha)
    assert np.all(g[w:n - w] == 1.0)
    assert np.array_equal(g, g[::-1])
    assert np.all(np.diff(g[: w + 1]) > 0)
    # at the outermost cell the taper depth is w cells: exp(-(alpha w)^2)
    assert abs(g[0] - math.exp(-((alpha * w) ** 2))) < 1e-15
    assert np.array_equal(oracle.sponge_profile(10, 0), np.ones(10))


def test_ricker_properties():
    fp = 15.0
    t0 = 1.5 / fp
    assert abs(oracle.ricker(t0, fp) - 1.0) < 1e-15
    # zero crossings at tau = +-1/(sqrt(2) pi fp); the wavelet integrates to zero
    tz = 1.0 / (math.sqrt(2.0) * math.pi * fp)
    assert abs(oracle.ricker(t0 + tz, fp)) < 1e-14 and abs(oracle.ricker(t0 - tz, fp)) < 1e-14
    t = np.linspace(0.0, 2 * t0, 200001)
    assert abs(np.trapezoid(oracle.ricker(t, fp), t)) < 1e-8
    # starts from (nearly) zero, as the Green's-function tests need
    assert abs(oracle.ricker(0.0, fp)) < 1e-8


def _plane_wave_error(h, v=2000.0, fp=15.0, xr=200.0, T=0.33, D=700.0):
    """1-D reduction (ny = nz = 1, periodic): a plane source f(t) delta(x) in
    (1/v^2) p_tt - p_xx = f(t) delta(x) gives p = (v/2) F(t - |x|/v), F' = f.  For the Ricker
    wavelet F(t) = tau exp(-(pi fp tau)^2)."""
    a = math.pi * fp
    t0 = 1.5 / fp
    n = int(round(2 * D / h)) + 1
    isrc = n // 2
    dt = oracle.stable_dt(4, h, v)
    nsteps = int(round(T / dt))
    kap = np.full((1, 1, n), (v * dt / h) ** 2)
    amp = oracle.ricker(np.arange(nsteps) * dt, fp, t0)[:, None]
    w = oracle.injection_weight(v, dt, h) * h * h        # point weight times the cell's face area
    ir = isrc + int(round(xr / h))
    out = oracle.forward(kap, None, nsteps, src_ijk=[(isrc, 0, 0)], src_w=[w], src_amp=amp, rec_ijk=[(ir, 0, 0)],
                         periodic=True)
    ts = (np.arange(nsteps) + 1) * dt
    tau = ts - xr / v - t0
    exact = (v / 2.0) * tau * np.exp(-((a * tau) ** 2))
    return oracle.rel_l2(out["traces"][:, 0], exact)


def test_plane_wave_green_function_second_order():
    errs = [_plane_wave_error(h) for h in (10.0, 5.0, 2.5)]
    assert errs[0] < 1e-2
    slope = math.log2(errs[1] / errs[2])
    assert 1.9 <= slope <= 2.1, (errs, slope)


def _point_source_errors(h, nthreads, v=2000.0, fp=10.0, r=150.0, T=0.36, D=430.0):
    """3-D point source: p = f(t - r/v) / (4 pi r) for (1/v^2) p_tt - lap p = f(t) delta(x)."""
    a = math.pi * fp
    t0 = 1.5 / fp
    n = int(round(2 * D / h)) + 1
    c = n // 2
    dt = oracle.stable_dt(4, h, v)
    nsteps = int(round(T / dt))
    kap = np.full((n, n, n), (v * dt / h) ** 2)
    amp = oracle.ricker(np.arange(nsteps) * dt, fp, t0)[:, None]
    ir = int(round(r / h))
    rec = [(c + ir, c, c), (c, c - ir, c), (c, c, c + ir)]
    out = oracle.forward(kap, None, nsteps, src_ijk=[(c, c, c)], src_w=[oracle.injection_weight(v, dt, h)],
                         src_amp=amp, rec_ijk=rec, nthreads=nthreads)
    tau = (np.arange(nsteps) + 1) * dt - r / v - t0
    exact = (1 - 2 * (a * tau) ** 2) * np.exp(-((a * tau) ** 2)) / (4 * math.pi * r)
    return [oracle.rel_l2(out["traces"][:, i], exact) for i in range(3)]


def test_point_source_green_function(oracle_threads):
    e = _point_source_errors(10.0, oracle_threads)
    assert max(e) < 5e-3, e
    assert max(e) - min(e) < 1e-12      # the three axis directions agree


@pytest.mark.slow
def test_point_source_green_function_converges(oracle_threads):
    e10 = max(_point_source_errors(10.0, oracle_threads))
    e5 = max(_point_source_errors(5.0, oracle_threads))
    slope = math.log2(e10 / e5)
    assert 1.8 <= slope <= 2.2, (e10, e5, slope)


def _random_problem(seed, shape=(24, 24, 24), nsteps=60, nsrc=3, nrec=7, width=4):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    cstar = oracle.stability_limit(4)
    kap = (cstar * rng.uniform(0.3, 0.8, shape)) ** 2
    sponge = (oracle.sponge_profile(nx, width), oracle.sponge_profile(ny, width), oracle.sponge_profile(nz, width))
    pick = lambda m: np.stack([rng.integers(0, nx, m), rng.integers(0, ny, m), rng.integers(0, nz, m)], axis=1)
    return rng, kap, sponge, pick(nsrc), rng.uniform(0.5, 2.0, nsrc), pick(nrec)


def test_adjoint_dot_product():
    """<F x, y> = <x, F^T y> for the map (source series -> traces), sponge on, variable kappa."""
    rng, kap, sponge, src, w, rec = _random_problem(21)
    nsteps = 60
    x = rng.standard_normal((nsteps, len(w)))
    y = rng.standard_normal((nsteps, len(rec)))
    fx = oracle.forward(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=x, rec_ijk=rec)["traces"]
    fty = oracle.adjoint_sources(kap, sponge, nsteps, src_ijk=src, src_w=w, rec_ijk=rec, y=y)
    lhs = float(np.sum(fx * y))
    rhs = float(np.sum(x * fty))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_gradient_matches_finite_differences():
    rng, kap, sponge, src, w, rec = _random_problem(31, shape=(20, 18, 22), nsteps=80, nrec=12)
    nsteps = 80
    amp = rng.standard_normal((nsteps, len(w)))
    kap_true = kap * (1.0 + 0.05 * rng.standard_normal(kap.shape))
    obs = oracle.forward(kap_true, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, rec_ijk=rec)["traces"]
    J, grad = oracle.gradient_kappa(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, rec_ijk=rec, observed=obs)
    # directional derivative along a random direction, and single-cell derivatives
    cells = [tuple(int(rng.integers(0, s)) for s in kap.shape) for _ in range(3)]
    top = np.argsort(np.abs(grad * kap).ravel())[-3:]
    cells += [tuple(int(i) for i in np.unravel_index(t, kap.shape)) for t in top]
    for direction in ["random"] + cells:
        if direction == "random":
            e = rng.standard_normal(kap.shape) * kap
        else:
            e = np.zeros_like(kap)
            e[direction] = kap[direction]
        # central differences are O(eps^2); eps is chosen so that truncation sits below 1e-7
        eps = 1e-5 if direction == "random" else 1e-4
        jp = oracle.misfit(oracle.forward(kap + eps * e, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp,
                                          rec_ijk=rec)["traces"], obs)
        jm = oracle.misfit(oracle.forward(kap - eps * e, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp,
                                          rec_ijk=rec)["traces"], obs)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(grad * e))
        # the FD quotient carries a rounding error of about 1e-15 J / eps
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-14 * J / eps, (direction, fd, an)


def test_image_matches_brute_force_and_is_linear():
    rng, kap, sponge, src, w, rec = _random_problem(41, shape=(16, 16, 16), nsteps=40, nsrc=1, nrec=9)
    nsteps, s = 40, 4
    amp = oracle.ricker(np.arange(nsteps) * 2e-3, 25.0)[:, None]
    data = rng.standard_normal((nsteps, len(rec)))
    rw = rng.uniform(0.5, 1.5, len(rec))
    img = oracle.migrate(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, rec_ijk=rec, rec_w=rw, data=data,
                         image_every=s)
    # brute force: keep every level of both wavefields, then correlate u^k with r^{N+1-k}
    fw = oracle.forward(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, snap_every=1)["snaps"]
    bw = oracle.forward(kap, sponge, nsteps, src_ijk=rec, src_w=rw, src_amp=data[::-1], snap_every=1)["snaps"]
    brute = np.zeros_like(kap)
    for k in range(1, nsteps + 1):
        if k % s == 0:
            brute += fw[k - 1] * bw[nsteps + 1 - k - 1]
    np.testing.assert_allclose(img, brute, rtol=0, atol=1e-13 * np.max(np.abs(brute)))
    img3 = oracle.migrate(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, rec_ijk=rec, rec_w=rw,
                          data=-2.5 * data, image_every=s)
    np.testing.assert_allclose(img3, -2.5 * img, rtol=0, atol=1e-13 * np.max(np.abs(img)))


def test_image_focuses_on_reflector(oracle_threads):
    """A flat interface below a surface shot: the RTM image of the reflection data (true minus
    background) peaks at the interface depth below the source."""
    n, nzr, h = 48, 30, 10.0
    v_bg = np.full((n, n, n), 2000.0)
    v_true = v_bg.copy()
    v_true[nzr:] = 2800.0
    dt = oracle.stable_dt(4, h, 2800.0)
    nsteps = 420
    g = oracle.sponge_profile(n, 10, 0.03)
    sponge = (g, g, g)
    src = [(24, 24, 12)]
    amp = oracle.ricker(np.arange(nsteps) * dt, 20.0)[:, None]
    rec = [(i, j, 12) for i in range(14, 35, 2) for j in range(14, 35, 2)]
    traces = {}
    for name, v in (("true", v_true), ("bg", v_bg)):
        kap = oracle.kappa_field(v, dt, h)
        w = oracle.injection_weight([2000.0], dt, h)
        traces[name] = oracle.forward(kap, sponge, nsteps, src_ijk=src, src_w=w, src_amp=amp, rec_ijk=rec,
                                      nthreads=oracle_threads)["traces"]
    data = traces["true"] - traces["bg"]
    kap_bg = oracle.kappa_field(v_bg, dt, h)
    img = oracle.migrate(kap_bg, sponge, nsteps, src_ijk=src, src_w=oracle.injection_weight([2000.0], dt, h),
                         src_amp=amp, rec_ijk=rec, rec_w=np.full(len(rec), 1.0), data=data, image_every=2,
                         nthreads=oracle_threads)
    column = np.abs(img[16:40, 22:27, 22:27]).sum(axis=(1, 2))
    zpeak = 16 + int(np.argmax(column))
    assert abs(zpeak - nzr) <= 2, zpeak


def test_pack_faces_layout():
    u = np.arange(5 * 6 * 7, dtype=np.float64).reshape(5, 6, 7)
    f = oracle.pack_faces(u, radius=2)
    sizes = [2 * 6 * 5, 2 * 6 * 5, 7 * 2 * 5, 7 * 2 * 5, 7 * 6 * 2, 7 * 6 * 2]
    assert [len(x) for x in f] == sizes
    # -X: x fastest within the 2-wide layer, then y, then z
    assert list(f[0][:4]) == [u[0, 0, 0], u[0, 0, 1], u[0, 1, 0], u[0, 1, 1]]
    assert list(f[1][:2]) == [u[0, 0, 5], u[0, 0, 6]]
    assert f[5][0] == u[3, 0, 0]


def test_bf16_rounding_is_nearest_even():
    """Brute force: the oracle's BF16 code is the nearest BF16 value, ties to the even pattern."""
    rng = np.random.default_rng(51)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        np.array([1.0, -1.0, 1.00390625, 1.01171875, 0.0, 3.0e-39], dtype=np.float32)])
    codes = oracle.bf16_rne(x)
    for xi, c in zip(x, codes):
        sign, mag = int(c) & 0x8000, int(c) & 0x7FFF
        cands = [sign | m for m in (max(mag - 1, 0), mag, mag + 1)]      # neighbours of the same sign
        vals = [oracle.bf16_to_f32(np.array([cc], dtype=np.uint16))[0].astype(np.float64) for cc in cands]
        d = [abs(v - float(xi)) for v in vals]
        assert d[1] <= d[0] and d[1] <= d[2], (xi, c)
        if (d[1] == d[0] and cands[0] != cands[1]) or d[1] == d[2]:
            assert mag % 2 == 0, (xi, c)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even pattern 0x3F80
    assert oracle.bf16_rne(np.array([1.00390625], dtype=np.float32))[0] == 0x3F80
    assert oracle.bf16_rne(np.array([1.01171875], dtype=np.float32))[0] == 0x3F82


def test_snapshot_codec_roundtrip_bounds():
    """Per-slab scaling: |decode(encode(u)) - u| <= unit roundoff x slab max (BF16 2^-9, FP16 2^-11
    in the normal range); all-zero slabs stay zero; FP16 codes equal numpy's RNE conversion."""
    rng = np.random.default_rng(52)
    u = rng.standard_normal((6, 9, 11)).astype(np.float32) * np.array([1e-3, 1.0, 50.0, 0.0, 1e-20, 7.0],
                                                                      dtype=np.float32)[:, None, None]
    for fmt, ur in (("bf16", 2.0 ** -9), ("f16", 2.0 ** -11)):
        codes, scales = oracle.snapshot_encode(u, fmt)
        np.testing.assert_array_equal(scales, np.max(np.abs(u), axis=(1, 2)))
        rec = oracle.snapshot_decode(codes, scales, fmt)
        err = np.abs(rec.astype(np.float64) - u.astype(np.float64))
        tol = scales.astype(np.float64)[:, None, None] * (ur * 1.0001 if fmt == "bf16" else 2.0 ** -14)
        tol = np.maximum(tol, np.abs(u) * ur * 1.0001)
        assert np.all(err <= tol + 1e-45), fmt
        assert np.all(rec[3] == 0)
    codes, scales = oracle.snapshot_encode(u, "f16")
    q = (u / np.where(scales > 0, scales, np.float32(1))[:, None, None]).astype(np.float32)
    q[scales == 0] = 0.0                         # a zero slab is coded as +0
    np.testing.assert_array_equal(codes, q.astype(np.float16).view(np.uint16))


def test_cnn_conv3d_matches_direct_definition():
    """The oracle's convolution equals the definition written as explicit loops (tiny volume)."""
    from oracle import cnn

    rng = np.random.default_rng(61)
    x = rng.standard_normal((3, 4, 5, 2))
    w = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(3)
    y = cnn.conv3d(x, w, b)
    nz, ny, nx = x.shape[:3]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for co in range(3):
                    s = b[co]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                kk, jj, ii = k + dz, j + dy, i + dx
                                if 0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx:
                                    t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                                    s += sum(w[t, co, ci] * x[kk, jj, ii, ci] for ci in range(2))
                    assert abs(y[k, j, i, co] - s) < 1e-12


@pytest.mark.parametrize("relu", [True, False])
@pytest.mark.parametrize("masked", [False, True])
def test_cnn_gradients_match_finite_differences(relu, masked):
    """Every parameter group's gradient against central differences of the loss, for the ReLU and
    the linear network, with and without a per-voxel mask and a loss weight."""
    from oracle import cnn

    rng = np.random.default_rng(62)
    x = rng.standard_normal((4, 5, 6, 3))
    tgt = rng.standard_normal((4, 5, 6, 2))
    params = [(rng.standard_normal((27, 4, 3)) * 0.3, rng.standard_normal(4) * 0.1),
              (rng.standard_normal((27, 4, 4)) * 0.3, rng.standard_normal(4) * 0.1),
              (rng.standard_normal((27, 2, 4)) * 0.3, rng.standard_normal(2) * 0.1)]
    kw = dict(relu=relu)
    if masked:
        mask = rng.uniform(0.0, 1.0, (4, 5, 6))
        mask[rng.uniform(size=mask.shape) < 0.3] = 0.0
        kw.update(mask=mask, weight=0.37)
    loss, grads = cnn.loss_and_grads(x, tgt, params, **kw)
    eps = 1e-6
    for li in range(3):
        for which in (0, 1):
            p = params[li][which]
            for _ in range(4):
                idx = tuple(int(rng.integers(0, s)) for s in p.shape)
                old = p[idx]
                p[idx] = old + eps
                lp = cnn.loss_and_grads(x, tgt, params, **kw)[0]
                p[idx] = old - eps
                lm = cnn.loss_and_grads(x, tgt, params, **kw)[0]
                p[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = grads[li][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (li, which, idx, fd, an)


def test_cnn_masked_loss_brute_force_and_linearity():
    """The masked, weighted loss equals its definition summed voxel by voxel; a voxel with mask 0
    does not count; the linear network without biases is linear in its input, the ReLU one is not."""
    from oracle import cnn

    rng = np.random.default_rng(63)
    shape = (3, 4, 5)
    x = rng.standard_normal(shape + (3,))
    tgt = rng.standard_normal(shape + (2,))
    params = [(rng.standard_normal((27, 4, 3)) * 0.3, np.zeros(4)),
              (rng.standard_normal((27, 4, 4)) * 0.3, np.zeros(4)),
              (rng.standard_normal((27, 3, 4)) * 0.3, np.zeros(3))]
    mask = rng.uniform(0.0, 1.0, shape)
    mask[1, 2, 3] = 0.0
    for relu in (True, False):
        out, _ = cnn.forward(x, params, relu)
        loss, _ = cnn.loss_and_grads(x, tgt, params, relu=relu, mask=mask, weight=2.5)
        brute = 0.0
        for k in range(shape[0]):
            for j in range(shape[1]):
                for i in range(shape[2]):
                    for c in range(2):       # the third output channel is not in the loss
                        brute += 0.5 * 2.5 * mask[k, j, i] * (out[k, j, i, c] - tgt[k, j, i, c]) ** 2
        assert abs(loss - brute) <= 1e-13 * brute
        t2 = tgt.copy()
        t2[1, 2, 3] += 10.0
        l2, g2 = cnn.loss_and_grads(x, t2, params, relu=relu, mask=mask, weight=2.5)
        _, g1 = cnn.loss_and_grads(x, tgt, params, relu=relu, mask=mask, weight=2.5)
        assert l2 == loss
        assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(g1, g2))
    lin, _ = cnn.forward(-2.0 * x, params, relu=False)
    np.testing.assert_allclose(lin, -2.0 * cnn.forward(x, params, relu=False)[0], rtol=1e-12, atol=1e-12)
    rel, _ = cnn.forward(-2.0 * x, params, relu=True)
    assert not np.allclose(rel, -2.0 * cnn.forward(x, params, relu=True)[0])
