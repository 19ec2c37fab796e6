"""The particle kernel's deposit arithmetic, run on the CPU, against the
oracle's Esirkepov deposit on the whole periodic grid.

The kernel's esirkepov_axis / deposit / deposit_cross1 (the Esirkepov
charge-conserving scheme, Comput. Phys. Commun. 135, 144 (2001), the current
solver the paper names in its Evaluation section) are compiled for the host
from the same header the kernel includes and driven through every path the
kernel takes: in line (first shape node unchanged), the general window of the
queued particles, and the single-axis window; in FP32 and FP64, for CIC, TSC
and PCS, with the degenerate moves (no displacement, faces, the tie of TSC).
The fixed-point accumulation of the FP32 tile is checked for its overflow
bound at the largest possible contributions.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from tests import host

SC = np.array([8, 8, 4])
ORIGIN = np.array([8, 8, 4])           # supercell corner in the test grid
GRID = (24, 24, 12)                    # room for every tile node without wrap


@pytest.fixture(scope="module")
def lib():
    L = C.CDLL(host.build())
    dp = C.POINTER(C.c_double)
    L.pdh_deposit.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, dp, dp, dp, C.c_double, dp, dp]
    L.pdh_deposit.restype = C.c_int
    L.pdh_layout.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def kernel_tile(L, prec, order, path, x0, x1, coef, jscale=0.0):
    dims = (C.c_int * 3)()
    lo = C.c_int()
    L.pdh_layout(dims, C.byref(lo))
    ox, oy, oz = dims
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 3)
    x1 = np.ascontiguousarray(x1, dtype=np.float64).reshape(-1, 3)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    out = np.zeros((3, oz, oy, ox))
    mx = C.c_double()
    r = L.pdh_deposit(prec, order, path, x0.shape[0], _p(x0), _p(x1), _p(coef), jscale, _p(out), C.byref(mx))
    assert r == 0, f"pdh_deposit returned {r}"
    # scatter the tile onto the test grid
    J = np.zeros((3,) + GRID[::-1])
    k0, j0, i0 = ORIGIN[2] + lo.value, ORIGIN[1] + lo.value, ORIGIN[0] + lo.value
    J[:, k0:k0 + oz, j0:j0 + oy, i0:i0 + ox] = out
    return J, mx.value


def oracle_J(order, x0, x1, qw, dl=(1.0, 1.0, 1.0), dt=0.5):
    g = oracle.make_grid(*GRID, order, dx=dl[0], dy=dl[1], dz=dl[2], dt=dt)
    a = np.asarray(x0, dtype=np.float64).reshape(-1, 3) + ORIGIN
    b = np.asarray(x1, dtype=np.float64).reshape(-1, 3) + ORIGIN
    return oracle.esirkepov(g, qw, a[:, 0], a[:, 1], a[:, 2], b[:, 0], b[:, 1], b[:, 2])


def coefs(qw, dl, dt):
    dV = dl[0] * dl[1] * dl[2]
    return np.array([-qw * d / (dV * dt) for d in dl])


def first_node(order, x):
    x = np.asarray(x)
    if order == 1:
        return np.floor(x).astype(int)
    if order == 2:
        return np.floor(x + 0.5).astype(int) - 1
    return np.floor(x).astype(int) - 1


def moves(order, kind, n, rng, prec):
    """n (x0, x1) pairs of supercell-relative positions for one path kind,
    rounded to the kernel's precision first (both sides then see the same moves)."""
    out0, out1 = [], []
    cast = np.float32 if prec == 0 else np.float64
    while len(out0) < n:
        x0 = cast(rng.uniform(0, 1, 3) * SC)
        amp = {"inline": 0.3, "general": 0.99, "single": 0.99}[kind]
        d = rng.uniform(-amp, amp, 3)
        if kind == "single":
            ax = rng.integers(3)
            d = d * 0.02
            d[ax] = rng.uniform(-0.99, 0.99)
        x1 = cast(x0 + d)
        ch = first_node(order, x0) != first_node(order, x1)
        if kind == "inline" and ch.any():
            continue
        if kind == "single" and ch.sum() != 1:
            continue
        out0.append(x0.astype(np.float64))
        out1.append(x1.astype(np.float64))
    return np.array(out0), np.array(out1)


TOL = {0: 3e-6, 1: 1e-13}


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("order", [1, 2, 3], ids=["cic", "tsc", "pcs"])
@pytest.mark.parametrize("kind,path", [("inline", 0), ("general", 1), ("single", 2), ("inline", 1),
                                       ("single", 1)])
def test_deposit_paths_match_oracle(lib, prec, order, kind, path):
    if path == 2 and order == 3:
        pytest.skip("the single-axis window serves CIC and TSC only")
    rng = np.random.default_rng(1000 * order + 10 * path + prec + (5 if kind == "single" else 0))
    dl, dt = (1.0, 0.75, 1.25), 0.4
    for trial in range(40):
        x0, x1 = moves(order, kind, 1, rng, prec)
        qw = -0.0625 * (1 + trial % 3)
        Jk, _ = kernel_tile(lib, prec, order, path, x0, x1, coefs(qw, dl, dt))
        Jo = oracle_J(order, x0, x1, qw, dl, dt)
        scale = np.abs(Jo).max()
        assert scale > 0
        err = np.abs(Jk - Jo).max() / scale
        assert err <= TOL[prec], (trial, x0, x1, err)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("order", [1, 2, 3], ids=["cic", "tsc", "pcs"])
def test_degenerate_moves(lib, prec, order):
    dl, dt, qw = (1.0, 1.0, 1.0), 0.5, -0.125
    c = coefs(qw, dl, dt)
    cases = [
        ((3.25, 4.5, 1.75), (3.25, 4.5, 1.75)),          # no displacement (also a particle kept in place)
        ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),              # on the low faces, at rest
        ((0.0, 2.0, 3.0), (0.3, 2.0, 3.0)),              # from a face, along x
        ((2.7, 5.0, 1.0), (3.0, 5.0, 1.0)),              # onto a face
        ((7.9, 7.9, 3.9), (8.2, 8.1, 4.05)),             # out through the far corner
        ((0.1, 0.1, 0.1), (-0.5, -0.6, -0.7)),           # out through the near corner
        ((2.5, 3.5, 1.5), (2.5, 3.5, 1.5)),              # TSC tie (half-integer), at rest
        ((2.5, 3.5, 1.5), (2.7, 3.2, 1.6)),              # from the tie
        ((1.4, 1.6, 2.4), (1.5, 1.5, 2.5)),              # onto the tie
    ]
    for x0, x1 in cases:
        x0 = np.array(x0, dtype=np.float32 if prec == 0 else np.float64).astype(np.float64)
        x1 = np.array(x1, dtype=np.float32 if prec == 0 else np.float64).astype(np.float64)
        Jo = oracle_J(order, x0, x1, qw, dl, dt)
        ch = first_node(order, x0) != first_node(order, x1)
        paths = [1] + ([0] if not ch.any() else []) + ([2] if ch.sum() == 1 and order != 3 else [])
        for path in paths:
            Jk, _ = kernel_tile(lib, prec, order, path, x0, x1, c)
            err = np.abs(Jk - Jo).max() / np.abs(c).max()
            assert err <= TOL[prec], (x0, x1, path, err)
            if np.array_equal(x0, x1):
                assert not Jk.any(), (x0, path)     # no displacement: exactly no current


@pytest.mark.parametrize("order", [1, 2, 3], ids=["cic", "tsc", "pcs"])
def test_fixed_point_bound_holds_at_the_largest_contributions(lib, order):
    """The FP32 tile's scale 2^30 / vmax (vmax = |q w| dx_d / (dV dt)) keeps
    every scaled contribution inside int32 at the largest Esirkepov factors
    (moves of just under one cell on every axis), and the truncated int64 sums
    of many such particles still match the oracle."""
    n = 6144
    dl, dt, qw = (1.0, 0.75, 1.25), 0.4, -1.0 / 16
    c = coefs(qw, dl, dt)
    vmax = np.abs(c).max()
    jscale = float(np.float32(2.0 ** 30) / np.float32(vmax))
    for x0, x1 in [((3.999, 3.999, 1.999), (4.998, 4.998, 2.998)), ((4.001, 4.001, 2.001), (3.002, 3.002, 1.002)),
                   ((3.5, 3.5, 1.5), (4.49, 4.49, 2.49)), ((0.001, 7.999, 0.001), (-0.998, 7.0, -0.998))]:
        a = np.tile(np.array(x0, dtype=np.float32).astype(np.float64), (n, 1))
        b = np.tile(np.array(x1, dtype=np.float32).astype(np.float64), (n, 1))
        Jk, mx = kernel_tile(lib, 0, order, 1, a, b, c, jscale)
        assert mx <= 2.0 ** 30 * (1 + 1e-6), mx
        assert mx > 0.1 * 2.0 ** 30          # these moves come within an order of magnitude of the bound
        Jo = oracle_J(order, a[:1], b[:1], qw, dl, dt) * n
        # identical particles truncate identically, so the error adds up
        # coherently: at most n units of the fixed-point scale, plus FP32
        err = np.abs(Jk - Jo).max()
        assert err <= n / jscale + 1e-6 * np.abs(Jo).max(), err
