"""Pins of the FP64 oracle's particle-in-cell routines.

Each test checks the oracle against something it does not compute itself:
numpy's Philox generator, closed forms (gyration orbit, Yee vacuum dispersion,
the 1D current of a moving CIC/TSC charge), invariants (partition of unity,
charge continuity, Gauss's law) and brute force over every node of a tiny
periodic grid with minimum-image distances.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


# ---------------------------------------------------------------------------
# Philox4x64-10 against numpy's implementation (bit-exact).

def _numpy_block(key, ctr):
    """numpy increments its 256-bit counter before each block: the block for
    counter c comes from a generator whose counter is c - 1."""
    c = [int(v) for v in ctr]
    val = sum(v << (64 * i) for i, v in enumerate(c)) - 1
    val %= 1 << 256
    prev = np.array([(val >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    return bg.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((160602862, 0), (1, 0, 0, 0)),
    ((160602863, 0), (12345678, 1, 2, 77)),
    ((2**64 - 1, 0), (2**64 - 1, 2**63, 5, 2**40)),
    ((42, 0), (0, 1, 0, 0)),
])
def test_philox_matches_numpy(key, ctr):
    got = oracle.philox4x64_10(ctr, key)
    want = _numpy_block(key, ctr)
    assert np.array_equal(got, want)


def test_u01_open_interval():
    assert oracle.u01(0) == 2.0 ** -54
    assert oracle.u01(2**64 - 1) == 1.0 - 2.0 ** -54
    assert 0.0 < oracle.u01(2**63) < 1.0


# ---------------------------------------------------------------------------
# Assignment functions.

@pytest.mark.parametrize("order", [1, 2, 3])
def test_shape_partition_and_moments(order):
    xs = workloads.rng(1).uniform(-3, 3, 400)
    for x in xs:
        nodes = np.arange(math.floor(x) - 3, math.floor(x) + 4)
        s = np.array([oracle.shape(order, x - i) for i in nodes])
        assert abs(s.sum() - 1.0) < 1e-15
        assert abs((nodes * s).sum() - x) < 1e-13
        # the B-spline of n unit boxes has discrete variance n/12 at every x
        # from n = 3 on (quadratic 1/4, cubic 1/3); the cubic's odd moments vanish
        if order == 2:
            assert abs(((nodes - x) ** 2 * s).sum() - 0.25) < 1e-13
        if order == 3:
            assert abs(((nodes - x) ** 2 * s).sum() - 1.0 / 3.0) < 1e-13
            assert abs(((nodes - x) ** 3 * s).sum()) < 1e-13


def test_shape_values():
    assert oracle.shape(1, 0.0) == 1.0 and oracle.shape(1, 0.25) == 0.75 and oracle.shape(1, 1.0) == 0.0
    assert oracle.shape(2, 0.0) == 0.75 and oracle.shape(2, 0.5) == 0.5 and oracle.shape(2, -0.5) == 0.5
    assert oracle.shape(2, 1.0) == 0.125 and oracle.shape(2, 1.5) == 0.0 and oracle.shape(2, 2.0) == 0.0
    # continuity of the two TSC pieces at |d| = 1/2 from either side
    assert abs(oracle.shape(2, 0.5 - 1e-12) - oracle.shape(2, 0.5 + 1e-12)) < 1e-11
    # cubic B-spline: 2/3 and 1/6 at the integers, 23/48 and 1/48 at the half integers
    assert abs(oracle.shape(3, 0.0) - 2 / 3) < 1e-16 and abs(oracle.shape(3, 1.0) - 1 / 6) < 1e-16
    assert oracle.shape(3, 2.0) == 0.0 and oracle.shape(3, -2.5) == 0.0
    assert abs(oracle.shape(3, 0.5) - 23 / 48) < 1e-16 and abs(oracle.shape(3, -1.5) - 1 / 48) < 1e-16
    assert abs(oracle.shape(3, 1.0 - 1e-12) - oracle.shape(3, 1.0 + 1e-12)) < 1e-11


# ---------------------------------------------------------------------------
# Field gather.

_OFF_E = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
_OFF_B = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def _min_image(d, n):
    return (d + n / 2.0) % n - n / 2.0


def _brute_interp(order, F, pos, off):
    nz, ny, nx = F.shape
    acc = 0.0
    for k in range(nz):
        sz = oracle.shape(order, _min_image(pos[2] - off[2] - k, nz))
        for j in range(ny):
            sy = oracle.shape(order, _min_image(pos[1] - off[1] - j, ny))
            for i in range(nx):
                sx = oracle.shape(order, _min_image(pos[0] - off[0] - i, nx))
                acc += sx * sy * sz * F[k, j, i]
    return acc


@pytest.mark.parametrize("order", [1, 2, 3])
def test_gather_brute_force_5cube(order):
    g = oracle.make_grid(5, 5, 5, order, b0=(0.01, -0.02, 0.1))
    E, B = workloads.random_fields(7 + order, 5, 5, 5, amp=1.0)
    r = workloads.rng(3 + order)
    pts = r.uniform(0, 5, size=(2, 3))
    Ep, Bp = oracle.gather(g, E, B, pts[:, 0], pts[:, 1], pts[:, 2])
    for p in range(2):
        for c in range(3):
            assert abs(Ep[p, c] - _brute_interp(order, E[c], pts[p], _OFF_E[c])) < 1e-14
            assert abs(Bp[p, c] - _brute_interp(order, B[c], pts[p], _OFF_B[c]) - g.b0[c]) < 1e-14


@pytest.mark.parametrize("order", [1, 2, 3])
def test_gather_uniform_and_linear_fields_exact(order):
    n = 12
    g = oracle.make_grid(n, n, n, order)
    E = np.zeros((3, n, n, n))
    B = np.zeros((3, n, n, n))
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    coef = [(0.3, -0.2, 0.1, 0.05), (-0.1, 0.4, 0.2, -0.3), (0.7, 0.1, -0.5, 0.2)]
    for c in range(3):
        a, bx, by, bz = coef[c]
        ox, oy, oz = _OFF_E[c]
        E[c] = a + bx * (ii + ox) + by * (jj + oy) + bz * (kk + oz)
        B[c] = 0.25 * (c + 1)  # uniform
    pts = workloads.rng(11).uniform(3, n - 3, size=(50, 3))
    Ep, Bp = oracle.gather(g, E, B, pts[:, 0], pts[:, 1], pts[:, 2])
    for c in range(3):
        a, bx, by, bz = coef[c]
        want = a + bx * pts[:, 0] + by * pts[:, 1] + bz * pts[:, 2]
        assert np.max(np.abs(Ep[:, c] - want)) < 1e-13
        assert np.max(np.abs(Bp[:, c] - 0.25 * (c + 1))) < 1e-15


# ---------------------------------------------------------------------------
# Galerkin gather: one order lower along a component's staggered axes.

def test_ngp_shape_order0():
    """Order 0 (nearest grid point) on the half-integer grid: weight 1 on the
    node within [-1/2, 1/2), the upper node taking a tie."""
    assert oracle.shape(0, 0.0) == 1.0 and oracle.shape(0, -0.5) == 1.0 and oracle.shape(0, 0.5) == 0.0
    assert oracle.shape(0, 0.49) == 1.0 and oracle.shape(0, -0.51) == 0.0
    for x in workloads.rng(5).uniform(-3, 3, 200):
        nodes = np.arange(math.floor(x) - 2, math.floor(x) + 3)
        assert sum(oracle.shape(0, x - i) for i in nodes) == 1.0


def _brute_interp_orders(orders, F, pos, off):
    nz, ny, nx = F.shape
    acc = 0.0
    for k in range(nz):
        sz = oracle.shape(orders[2], _min_image(pos[2] - off[2] - k, nz))
        for j in range(ny):
            sy = oracle.shape(orders[1], _min_image(pos[1] - off[1] - j, ny))
            for i in range(nx):
                sx = oracle.shape(orders[0], _min_image(pos[0] - off[0] - i, nx))
                acc += sx * sy * sz * F[k, j, i]
    return acc


@pytest.mark.parametrize("order", [1, 2, 3])
def test_galerkin_gather_brute_force_5cube(order):
    g = oracle.make_grid(5, 5, 5, order, b0=(0.01, -0.02, 0.1), galerkin=True)
    E, B = workloads.random_fields(17 + order, 5, 5, 5, amp=1.0)
    pts = workloads.rng(13 + order).uniform(0, 5, size=(3, 3))
    Ep, Bp = oracle.gather(g, E, B, pts[:, 0], pts[:, 1], pts[:, 2])
    for p in range(3):
        for c in range(3):
            oe = [order - 1 if o else order for o in _OFF_E[c]]
            ob = [order - 1 if o else order for o in _OFF_B[c]]
            assert abs(Ep[p, c] - _brute_interp_orders(oe, E[c], pts[p], _OFF_E[c])) < 1e-14
            assert abs(Bp[p, c] - _brute_interp_orders(ob, B[c], pts[p], _OFF_B[c]) - g.b0[c]) < 1e-14


@pytest.mark.parametrize("order", [1, 2, 3])
def test_galerkin_equals_standard_for_fields_uniform_along_staggered_axes(order):
    """Every shape sums to one, so a component that does not vary along its
    staggered axes is gathered identically by both schemes."""
    n = 10
    g0 = oracle.make_grid(n, n, n, order)
    g1 = oracle.make_grid(n, n, n, order, galerkin=True)
    r = workloads.rng(31)
    E = np.zeros((3, n, n, n))
    B = np.zeros((3, n, n, n))
    for c in range(3):
        base = r.uniform(-1, 1, (n, n, n))
        # E_c varies only across axis c; B_c only along axis c
        e = base.mean(axis=2 - c, keepdims=True)
        E[c] = np.broadcast_to(e, (n, n, n))
        keep = [ax for ax in (0, 1, 2) if ax != 2 - c]
        b = base.mean(axis=tuple(keep), keepdims=True)
        B[c] = np.broadcast_to(b, (n, n, n))
    pts = r.uniform(0, n, size=(40, 3))
    E0, B0 = oracle.gather(g0, E, B, *pts.T)
    E1, B1 = oracle.gather(g1, E, B, *pts.T)
    assert np.max(np.abs(E0 - E1)) < 1e-14 and np.max(np.abs(B0 - B1)) < 1e-14
    # and they differ for a generic field
    E2, B2 = workloads.random_fields(32, n, n, n, amp=1.0)
    Ea, _ = oracle.gather(g0, E2, B2, *pts.T)
    Eb, _ = oracle.gather(g1, E2, B2, *pts.T)
    assert np.max(np.abs(Ea - Eb)) > 1e-3


# ---------------------------------------------------------------------------
# Boris push.

def _circumcenter(p0, p1, p2):
    ax, ay = p0
    bx, by = p1
    cx, cy = p2
    d = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax**2 + ay**2) * (by - cy) + (bx**2 + by**2) * (cy - ay) + (cx**2 + cy**2) * (ay - by)) / d
    uy = ((ax**2 + ay**2) * (cx - bx) + (bx**2 + by**2) * (ax - cx) + (cx**2 + cy**2) * (bx - ax)) / d
    return np.array([ux, uy])


@pytest.mark.parametrize("q,m,dt,Bz,u", [(-1.0, 1.0, 0.5, 0.1, (0.3, 0.1, 0.05)),
                                          (1.0, 1836.0, 0.5, 0.1, (0.002, -0.001, 0.0)),
                                          (-1.0, 1.0, 2.0, 1.0, (0.9, 0.4, 0.2))])
def test_boris_gyration_closed_form(q, m, dt, Bz, u):
    """Uniform B, E = 0: |u| is conserved, u_perp turns by 2 atan(w_c dt / 2)
    per step with w_c = |q|B/(m gamma), and the discrete orbit is a circle of
    radius (u_perp m / |q| B) sqrt(1 + (w_c dt/2)^2)."""
    ux, uy, uz = (np.array([v]) for v in u)
    u2 = sum(v * v for v in u)
    gam = math.sqrt(1 + u2)
    wc = abs(q) * Bz / (m * gam)
    theta = 2 * math.atan(wc * dt / 2)
    uperp = math.hypot(u[0], u[1])
    R = uperp * m / (abs(q) * Bz) * math.sqrt(1 + (wc * dt / 2) ** 2)
    Ep = np.zeros((1, 3))
    Bp = np.array([[0.0, 0.0, Bz]])
    pos = [np.zeros(2)]
    phase0 = math.atan2(u[1], u[0])
    nsteps = 400
    for n in range(1, nsteps + 1):
        ux, uy, uz = oracle.boris(q / m, dt, Ep, Bp, ux, uy, uz)
        nu = math.sqrt(ux[0] ** 2 + uy[0] ** 2 + uz[0] ** 2)
        assert abs(nu * nu - u2) < 1e-15 * max(1.0, u2) * n
        ang = math.atan2(uy[0], ux[0])
        want = phase0 - math.copysign(1.0, q) * n * theta
        assert abs(math.remainder(ang - want, 2 * math.pi)) < 1e-11 * n
        pos.append(pos[-1] + dt * np.array([ux[0], uy[0]]) / gam)
    pos = np.array(pos)
    ctr = _circumcenter(pos[0], pos[1], pos[2])
    dist = np.hypot(*(pos - ctr).T)
    assert np.max(np.abs(dist / R - 1.0)) < 1e-6
    # period in steps is 2 pi / theta, which tends to 2 pi gamma m / (|q| B dt) as dt -> 0
    assert abs((2 * math.pi / theta) * dt / (2 * math.pi * gam * m / (abs(q) * Bz)) - 1) < (wc * dt) ** 2


def test_boris_small_dt_limit_textbook_larmor():
    q, m, Bz, u = -1.0, 1.0, 0.2, (0.1, 0.0, 0.0)
    gam = math.sqrt(1 + 0.01)
    rl = 0.1 * m / (abs(q) * Bz)
    dt = 1e-3
    ux, uy, uz = np.array([u[0]]), np.array([u[1]]), np.array([u[2]])
    pos = [np.zeros(2)]
    for _ in range(3):
        ux, uy, uz = oracle.boris(q / m, dt, np.zeros((1, 3)), np.array([[0, 0, Bz]]), ux, uy, uz)
        pos.append(pos[-1] + dt * np.array([ux[0], uy[0]]) / gam)
    ctr = _circumcenter(*pos[:3])
    assert abs(np.hypot(*(pos[1] - ctr)) / rl - 1) < 1e-6


def test_boris_uniform_e_exact_kick():
    q, m, dt = -1.0, 1.0, 0.5
    E = np.array([[0.013, -0.027, 0.0041]])
    ux, uy, uz = np.array([0.1]), np.array([-0.2]), np.array([0.05])
    u0 = np.array([0.1, -0.2, 0.05])
    for n in range(1, 21):
        ux, uy, uz = oracle.boris(q / m, dt, E, np.zeros((1, 3)), ux, uy, uz)
        want = u0 + n * q * E[0] * dt / m
        assert np.max(np.abs(np.array([ux[0], uy[0], uz[0]]) - want)) < 1e-15 * n


def test_boris_exb_drift():
    """E perpendicular to B, |E| << |B|: mean velocity equals E x B / B^2."""
    q, m, dt = 1.0, 1.0, 0.05
    Ey, Bz = 1e-3, 1.0
    E = np.array([[0.0, Ey, 0.0]])
    B = np.array([[0.0, 0.0, Bz]])
    # start near the drift with a small gyration on top; average over ~200 gyro-periods
    ux, uy, uz = np.array([Ey / Bz + 2e-4]), np.array([0.0]), np.array([0.0])
    nper = int(round(2 * math.pi / dt))
    vsum = np.zeros(2)
    n = 200 * nper
    for _ in range(n):
        ux, uy, uz = oracle.boris(q / m, dt, E, B, ux, uy, uz)
        g = math.sqrt(1 + ux[0] ** 2 + uy[0] ** 2 + uz[0] ** 2)
        vsum += np.array([ux[0], uy[0]]) / g
    vd = vsum / n
    assert abs(vd[0] / (Ey / Bz) - 1) < 1e-3
    assert abs(vd[1]) < 1e-3 * Ey / Bz


# ---------------------------------------------------------------------------
# Esirkepov current.

def _random_moves(seed, n, L, maxd):
    r = workloads.rng(seed)
    p0 = r.uniform(0, L, size=(n, 3))
    d = r.uniform(-maxd, maxd, size=(n, 3))
    return p0, p0 + d


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("dx", [(1.0, 1.0, 1.0), (0.7, 1.3, 0.9)])
def test_esirkepov_continuity_residual(order, dx):
    """div J + (rho1 - rho0)/dt = 0 at every node, to round-off."""
    n = 8
    g = oracle.make_grid(n, n, n, order, dx=dx[0], dy=dx[1], dz=dx[2], dt=0.37)
    p0, p1 = _random_moves(5 + order, 40, n, 0.95)
    qw = workloads.rng(9).uniform(-1.0, 1.0, 40)
    J = oracle.esirkepov(g, qw, *p0.T, *p1.T)
    r0 = oracle.deposit_rho(g, qw, *p0.T)
    r1 = oracle.deposit_rho(g, qw, *(p1 % n).T)
    res = oracle.div_nodes(g, J) + (r1 - r0) / g.dt
    scale = np.abs(qw).max() / g.dt / (g.dx * g.dy * g.dz)
    assert np.max(np.abs(res)) < 1e-14 * scale * 10


@pytest.mark.parametrize("order", [1, 2, 3])
def test_esirkepov_total_current_and_support(order):
    """sum J_d dV = q w (x1_d - x0_d) dx_d / dt; J vanishes off the window."""
    n = 10
    g = oracle.make_grid(n, n, n, order, dx=0.8, dy=1.1, dz=1.0, dt=0.5)
    p0 = np.array([[4.3, 5.7, 4.95]])
    p1 = p0 + np.array([[0.6, -0.8, 0.3]])
    qw = -0.125
    J = oracle.esirkepov(g, qw, *p0.T, *p1.T)
    dV = g.dx * g.dy * g.dz
    for d, dl in enumerate((g.dx, g.dy, g.dz)):
        tot = J[d].sum() * dV
        assert abs(tot - qw * (p1[0, d] - p0[0, d]) * dl / g.dt) < 1e-15
    nz = np.argwhere(np.any(J != 0.0, axis=0))
    lo = np.floor(np.minimum(p0, p1)[0] + (0.0 if order == 1 else -0.5)).astype(int) - (order - 1)
    hi = np.floor(np.maximum(p0, p1)[0]).astype(int) + 2
    for k, j, i in nz:
        for ax, idx in zip((0, 1, 2), (i, j, k)):
            assert lo[ax] - 1 <= idx <= hi[ax] + 1


def _cic_cdf(s):
    if s <= -1:
        return 0.0
    if s <= 0:
        return 0.5 * (1 + s) ** 2
    if s < 1:
        return 1 - 0.5 * (1 - s) ** 2
    return 1.0


def _tsc_cdf(s):
    """Integral of the quadratic B-spline from -inf to s (piecewise cubic)."""
    if s <= -1.5:
        return 0.0
    if s <= -0.5:
        return (s + 1.5) ** 3 / 6
    if s <= 0.5:
        return 1 / 6 + 0.75 * (s + 0.5) - (s**3 + 0.125) / 3
    if s < 1.5:
        return 1 - (1.5 - s) ** 3 / 6
    return 1.0


@pytest.mark.parametrize("order", [1, 2, 3])
def test_esirkepov_one_axis_reduces_to_1d_flux(order):
    """Motion along x only: J_x through face i+1/2 is the charge that crossed
    it.  For CIC that is the charge times (x1 - x0) inside one cell; for TSC it
    is the difference of the triangle's cumulative at x - (i + 1/2); for PCS
    that of the quadratic B-spline's cumulative."""
    n = 12
    g = oracle.make_grid(n, n, n, order, dt=0.5)
    qw = 0.3
    cases = [(5.2, 5.6), (5.7, 6.4), (6.1, 5.3)] if order >= 2 else [(5.2, 5.6), (5.45, 5.05)]
    for x0, x1 in cases:
        y, z = 4.3, 7.8
        J = oracle.esirkepov(g, qw, x0, y, z, x1, y, z)
        for k in range(n):
            sz = oracle.shape(order, z - k)
            for j in range(n):
                sy = oracle.shape(order, y - j)
                for i in range(n):
                    if order == 1:
                        flux = (x1 - x0) if i == math.floor(x0) else 0.0
                    elif order == 2:
                        flux = _cic_cdf(x1 - i - 0.5) - _cic_cdf(x0 - i - 0.5)
                    else:
                        flux = _tsc_cdf(x1 - i - 0.5) - _tsc_cdf(x0 - i - 0.5)
                    want = qw / g.dt * flux * sy * sz
                    assert abs(J[0, k, j, i] - want) < 1e-15
        assert np.all(J[1] == 0) and np.all(J[2] == 0)


def _brute_esirkepov(order, n, dt, qw, p0, p1):
    """Esirkepov's current from its definition as the mean over the six
    orders of moving one coordinate at a time, evaluated at every node of a
    periodic n^3 grid with minimum-image shapes; each line's running sum starts
    at a node outside the particle's reach (dx = dy = dz = 1)."""
    J = np.zeros((3, n, n, n))
    S0 = [np.array([oracle.shape(order, _min_image(p0[d] - i, n)) for i in range(n)]) for d in range(3)]
    S1 = [np.array([oracle.shape(order, _min_image(p1[d] - i, n)) for i in range(n)]) for d in range(3)]
    for d in range(3):
        e1, e2 = (d + 1) % 3, (d + 2) % 3
        a0, a1 = S0[d][:, None, None], S1[d][:, None, None]
        b0, b1 = S0[e1][None, :, None], S1[e1][None, :, None]
        c0, c1 = S0[e2][None, None, :], S1[e2][None, None, :]
        Wd = ((a1 * b1 * c1 - a0 * b1 * c1) / 3 + (a1 * b0 * c1 - a0 * b0 * c1) / 6 +
              (a1 * b1 * c0 - a0 * b1 * c0) / 6 + (a1 * b0 * c0 - a0 * b0 * c0) / 3)
        cut = next(i for i in range(n) if S0[d][i] == 0 and S1[d][i] == 0)
        Jd = np.zeros((n, n, n))  # indexed [axis d, axis e1, axis e2]
        run = np.zeros((n, n))
        for s in range(n):
            i = (cut + s) % n
            run = run - qw / dt * Wd[i]
            Jd[i] = run
        # back to [k, j, i] order
        perm = {0: (0, 1, 2), 1: (1, 2, 0), 2: (2, 0, 1)}[d]  # axes of Jd are (d, e1, e2)
        axes_xyz = np.moveaxis(Jd, [0, 1, 2], [perm[0], perm[1], perm[2]])  # -> (x, y, z)
        J[d] = np.transpose(axes_xyz, (2, 1, 0))
    return J


@pytest.mark.parametrize("order,n", [(1, 5), (2, 5), (3, 7)])
def test_esirkepov_brute_force_two_particles(order, n):
    g = oracle.make_grid(n, n, n, order, dt=0.5)
    p0, p1 = _random_moves(21 + order, 2, n, 0.9)
    qw = np.array([-0.125, 0.25])
    J = oracle.esirkepov(g, qw, *p0.T, *p1.T)
    Jb = _brute_esirkepov(order, n, g.dt, qw[0], p0[0], p1[0]) + _brute_esirkepov(order, n, g.dt, qw[1], p0[1], p1[1])
    assert np.max(np.abs(J - Jb)) < 1e-14


# ---------------------------------------------------------------------------
# Yee solver.

@pytest.mark.parametrize("dxs,dt", [((1.0, 1.0, 1.0), 0.5), ((1.0, 0.8, 1.2), 0.4)])
def test_yee_vacuum_dispersion(dxs, dt):
    """A divergence-free discrete mode with B = 0 evolves as cos(n theta) with
    sin(theta/2) = dt sqrt(sum_d sin^2(k_d dx_d / 2) / dx_d^2)."""
    n = 16
    g = oracle.make_grid(n, n, n, 1, dx=dxs[0], dy=dxs[1], dz=dxs[2], dt=dt)
    mvec = np.array([1, 2, 3])
    dl = np.array(dxs)
    k = 2 * np.pi * mvec / (n * dl)
    kt = 2 / dl * np.sin(k * dl / 2)
    e = np.cross(kt, [0.3, -0.5, 0.8])
    e /= np.linalg.norm(e)
    phi = 0.37
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    E0 = np.zeros((3, n, n, n))
    for c in range(3):
        off = np.zeros(3)
        off[c] = 0.5
        arg = k[0] * (ii + off[0]) * dl[0] + k[1] * (jj + off[1]) * dl[1] + k[2] * (kk + off[2]) * dl[2] + phi
        E0[c] = e[c] * np.cos(arg)
    E = E0.copy()
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    theta = 2 * math.asin(dt * math.sqrt(float(np.sum(np.sin(k * dl / 2) ** 2 / dl**2))))
    st = oracle.State(g, [], E, B, J)
    for nstep in range(1, 101):
        oracle.step(st, 1)
        if nstep % 25 == 0:
            assert np.max(np.abs(st.E - math.cos(nstep * theta) * E0)) < 1e-13
    assert np.max(np.abs(oracle.div_cells(g, st.B))) < 1e-13
    assert np.max(np.abs(oracle.div_nodes(g, st.E))) < 1e-13


# ---------------------------------------------------------------------------
# The whole cycle.

def test_init_structure_and_statistics():
    cfg = workloads.config(2, nx=8, ny=8, nz=8)
    cfg["species"][0]["layout"] = "shear"
    cfg["species"][0]["drift_beta"] = (0.2, 0.0, 0.0)
    st = oracle.init_state(cfg)
    e, p = st.species
    ncell = 8 ** 3
    assert e.n == 8 * ncell and p.n == 8 * ncell
    assert np.array_equal(e.id, np.arange(e.n)) and np.array_equal(p.id, np.arange(p.n) + e.n)
    # exactly ppc particles in every cell, each inside its own cell
    cell = np.floor(e.x).astype(int) + 8 * (np.floor(e.y).astype(int) + 8 * np.floor(e.z).astype(int))
    assert np.array_equal(cell, np.repeat(np.arange(ncell), 8))
    # coincident placement: protons sit exactly on the electrons
    assert np.array_equal(e.x, p.x) and np.array_equal(e.y, p.y) and np.array_equal(e.z, p.z)
    # shear layer: +u_d for 4j in [ny, 3ny), -u_d elsewhere
    ud = 0.2 / math.sqrt(1 - 0.04)
    j = np.floor(e.y).astype(int)
    inside = (4 * j >= 8) & (4 * j < 24)
    assert abs(e.ux[inside].mean() - ud) < 3e-3 and abs(e.ux[~inside].mean() + ud) < 3e-3
    assert abs(e.uy.std() / 0.02 - 1) < 0.05 and abs(p.uz.std() / 0.0005 - 1) < 0.05
    assert e.w[0] == 1.0 / 8 and p.w[0] == 1.0 / 8


def test_init_draws_follow_counter_layout():
    cfg = workloads.config(0, nx=8, ny=8, nz=4)
    st = oracle.init_state(cfg)
    e = st.species[0]
    seed = cfg["grid"]["seed"]
    for pid in (0, 17, 2047):
        w0 = oracle.philox4x64_10([pid, 0, 0, 0], [seed, 0])
        cell = pid // 8
        i, j, k = cell % 8, (cell // 8) % 8, cell // 64
        assert e.x[pid] == i + oracle.u01(w0[0]) and e.y[pid] == j + oracle.u01(w0[1])
        assert e.z[pid] == k + oracle.u01(w0[2])
        w1 = oracle.philox4x64_10([pid, 0, 1, 0], [seed, 0])
        a, b = oracle.u01(w1[0]), oracle.u01(w1[1])
        assert abs(e.ux[pid] - 0.05 * math.sqrt(-2 * math.log(a)) * math.cos(2 * math.pi * b)) < 1e-16


@pytest.mark.parametrize("idx,box", [(0, (16, 16, 16)), (2, (8, 8, 8))])
def test_cycle_gauss_invariant(idx, box):
    """G = div E - rho keeps its t = 0 value at every node over the run."""
    cfg = workloads.reduced(idx, *box)
    st = oracle.init_state(cfg)
    G0 = oracle.gauss_residual(st)
    rmax = np.abs(oracle.rho(st)).max() + 1.0
    nsteps = 30 if idx == 0 else 10
    for _ in range(3):
        oracle.step(st, nsteps // 3)
        assert np.max(np.abs(oracle.gauss_residual(st) - G0)) < 1e-12 * rmax
    assert np.max(np.abs(oracle.div_cells(st.grid, st.B))) < 1e-12


def test_cycle_trace_bookkeeping_and_immobile():
    cfg = workloads.reduced(2, 8, 8, 8)
    cfg["species"][1]["mobile"] = False
    st = oracle.init_state(cfg)
    p0 = st.species[1].copy()
    tr = oracle.step(st, 3, trace=True)
    # immobile species untouched
    assert np.array_equal(st.species[1].x, p0.x) and np.array_equal(st.species[1].ux, p0.ux)
    # K^{n+1/2} of one step is K^{(n+1)-1/2} of the next
    assert np.allclose(tr[1:, 2], tr[:-1, 3], rtol=0, atol=1e-14)
    we, wb = oracle.field_energy(st.grid, st.E, st.B)
    assert we > 0 and wb > 0


def test_threaded_cycle_matches_serial_cycle():
    """The all-cores CPU baseline (particle loop split over threads, private
    current arrays summed after the loop) computes the cycle of orc_step: only
    the order of the current sums differs, so states agree to rounding."""
    cfg = workloads.config(1, nx=16, ny=16, nz=8)   # shear layer: many crossings
    a = oracle.init_state(cfg)
    b = a.copy()
    oracle.step(a, 5)
    used = oracle.step_threads(b, 5, 4)
    assert used >= 1
    for sa, sb in zip(a.species, b.species):
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            assert np.max(np.abs(getattr(sa, k) - getattr(sb, k))) < 1e-12, k
    for fa, fb in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert np.max(np.abs(fa - fb)) <= 1e-12 * max(np.abs(fa).max(), 1e-300)
