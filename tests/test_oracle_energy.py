"""Pins of the FP64 oracle's energy diagnostics: W_E = (1/2) sum |E|^2 dV,
W_B = (1/2) sum |B|^2 dV, K = sum w m (gamma - 1) and the cycle's total-energy
trace T_n = W_E^n + W_B^n + (K^{n-1/2} + K^{n+1/2}) / 2.

The paper's benchmark is an energy-trace workload (section "Evaluation": the
Kelvin-Helmholtz run), so these are the diagnostics the 100-step parity trace
rests on.  Each is pinned by something the oracle does not compute itself:
  - the field energies of a Yee vacuum mode on a grid with dx != dy != dz,
    from the mode's closed-form solution of the discrete scheme;
  - K at rest (exactly 0) and in its non-relativistic and ultra-relativistic
    limits;
  - energy conservation of the whole cycle in a cold Langmuir oscillation with
    the Galerkin gather (the gather that is the transpose of the Esirkepov
    deposit, so the semi-discrete scheme conserves energy): the drift of T_n
    over one plasma period is pure time-discretisation error and falls 4x
    when dt halves.
The last test compiles copies of the oracle with one planted mistake each (a
dropped 1/2, dV, m or w, gamma in place of gamma - 1) and a trace without the
time-centred kinetic term, and checks that one of the pins fails for every one.
"""
import math
import os

import numpy as np
import pytest

import oracle

# ---------------------------------------------------------------------------
# Field energies of a Yee vacuum mode.
#
# With E^0 = e cos(k.r_E + phi) (k~ . e = 0, k~_d = (2/dx_d) sin(k_d dx_d / 2))
# and B^0 = 0, the B/2, E, B/2 cycle gives E^n = cos(n theta) E^0 with
# sin(theta/2) = dt |k~| / 2, and B^n = sin(n theta) cos(theta/2) / |k~|
# (k~ x e) sin(k.r_B + phi), each B component at its own Yee location.  Over
# the N nodes of the periodic grid each cos^2 / sin^2 sums to N/2 (2k is not a
# multiple of the grid's period), so W_E^n = (N dV / 4) cos^2(n theta) and
# W_B^n = (N dV / 4) sin^2(n theta) cos^2(theta/2).

_EOFF = [(0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5)]
_BOFF = [(0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]


def _yee_mode(n=16, dxs=(0.7, 1.3, 0.9), dt=0.4, mvec=(1, 2, 3), phi=0.37):
    dl = np.array(dxs)
    k = 2 * np.pi * np.array(mvec) / (n * dl)
    kt = 2 / dl * np.sin(k * dl / 2)
    e = np.cross(kt, [0.3, -0.5, 0.8])
    e /= np.linalg.norm(e)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")

    def wave(offs, amp, fn):
        F = np.zeros((3, n, n, n))
        for c in range(3):
            o = offs[c]
            arg = (k[0] * (ii + o[0]) * dl[0] + k[1] * (jj + o[1]) * dl[1] + k[2] * (kk + o[2]) * dl[2] + phi)
            F[c] = amp[c] * fn(arg)
        return F

    theta = 2 * math.asin(dt * np.linalg.norm(kt) / 2)
    return dict(n=n, dl=dl, dt=dt, kt=kt, e=e, theta=theta,
                E0=wave(_EOFF, e, np.cos), Bshape=wave(_BOFF, np.cross(kt, e) / np.linalg.norm(kt), np.sin))


def _pin_yee_field_energy():
    m = _yee_mode()
    n, dl, th = m["n"], m["dl"], m["theta"]
    g = oracle.make_grid(n, n, n, 1, dx=dl[0], dy=dl[1], dz=dl[2], dt=m["dt"])
    st = oracle.State(g, [], m["E0"].copy(), np.zeros_like(m["E0"]), np.zeros_like(m["E0"]))
    quarter = n**3 * float(np.prod(dl)) / 4
    we, wb = oracle.field_energy(g, st.E, st.B)
    assert abs(we - quarter) < 1e-12 * quarter and wb == 0.0
    for step in range(1, 41):
        oracle.step(st, 1)
        if step % 5:
            continue
        b_amp = math.sin(step * th) * math.cos(th / 2)
        assert np.max(np.abs(st.B - b_amp * m["Bshape"])) < 1e-13
        we, wb = oracle.field_energy(g, st.E, st.B)
        assert abs(we - quarter * math.cos(step * th) ** 2) < 1e-12 * quarter
        assert abs(wb - quarter * b_amp**2) < 1e-12 * quarter


def test_yee_mode_field_energies_closed_form():
    _pin_yee_field_energy()


# ---------------------------------------------------------------------------
# Kinetic energy: at rest, and its two limits.

def _species(u, w, m, q=-1.0):
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    n = u.shape[0]
    z = np.zeros(n)
    return oracle.Species(z.copy(), z.copy(), z.copy(), u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy(),
                          np.full(n, w), np.arange(n, dtype=np.int64), q=q, m=m)


def _kinetic(sp):
    g = oracle.make_grid(8, 8, 8, 1)
    return oracle.kinetic(oracle.State(g, [sp], *[oracle.zero_fields(g)] * 3))


def _pin_kinetic_limits():
    w, mass = 0.37, 5.5
    assert _kinetic(_species(np.zeros((7, 3)), w, mass)) == 0.0
    dirs = np.array([[1.0, 0.0, 0.0], [0.6, -0.8, 0.0], [0.0, 0.28, -0.96], [-0.48, 0.36, 0.8]])
    # non-relativistic: gamma - 1 = u^2/2 - u^4/8 + ..., K -> (1/2) sum w m u^2
    for s in (1e-3, 1e-2):
        u = s * dirs
        k_nr = 0.5 * w * mass * float(np.sum(u * u))
        assert abs(_kinetic(_species(u, w, mass)) / k_nr - 1.0) < 0.3 * s * s
    # ultra-relativistic: gamma - 1 = |u| - 1 + 1/(2|u|) + ..., K -> sum w m (|u| - 1)
    for s in (1e3, 1e5):
        u = s * dirs
        k_ur = w * mass * len(dirs) * (s - 1.0)
        assert abs(_kinetic(_species(u, w, mass)) / k_ur - 1.0) < 1.0 / s**2


def test_kinetic_energy_rest_and_limits():
    _pin_kinetic_limits()


# ---------------------------------------------------------------------------
# Energy conservation of the cycle: cold Langmuir oscillation.

def _langmuir_drift(dt, order=1, q=-1.0, m=3.0, ppcx=4, u0=2e-3):
    """Relative drift max_n |T_n - T_0| / max_n W_E^n over one plasma period of
    a cold plasma on a quiet lattice (ppcx particles per cell along x, one at
    each y, z cell centre), velocity perturbation u0 sin(k x) with k = 2 pi / L_x,
    immobile neutralising background, Galerkin gather, dx != dy != dz."""
    nx, ny, nz = 16, 2, 2
    dxs = (0.7, 1.3, 0.9)
    g = oracle.make_grid(nx, ny, nz, order, dx=dxs[0], dy=dxs[1], dz=dxs[2], dt=dt, rho_bg=-q, galerkin=True)
    dV = float(np.prod(dxs))
    xs = (np.arange(nx * ppcx) + 0.5) / ppcx
    X, Y, Z = (a.ravel() for a in np.meshgrid(xs, np.arange(ny) + 0.5, np.arange(nz) + 0.5, indexing="ij"))
    npart = X.size
    ux = u0 * np.sin(2 * np.pi / nx * X)
    zero = np.zeros(npart)
    sp = oracle.Species(X.copy(), Y.copy(), Z.copy(), ux, zero.copy(), zero.copy(), np.full(npart, dV / ppcx),
                        np.arange(npart, dtype=np.int64), q=q, m=m)
    st = oracle.State(g, [sp], *[oracle.zero_fields(g) for _ in range(3)])
    omega_p = abs(q) / math.sqrt(m)    # density 1: omega_p^2 = n q^2 / m
    nsteps = int(round(2 * math.pi / omega_p / dt))
    tr = oracle.step(st, nsteps, trace=True)
    T = oracle.energy_trace_total(tr)
    assert tr[:, 0].max() > 0.4 * tr[:, 2].max() > 0     # the energy does slosh between E and K
    return float(np.max(np.abs(T - T[0])) / tr[:, 0].max())


def _pin_langmuir_energy():
    for order in (1, 2):
        a, b = _langmuir_drift(0.1, order), _langmuir_drift(0.05, order)
        assert a < 3e-3, (order, a)
        assert 3.6 < a / b < 4.4, (order, a, b)


def test_cycle_energy_conserved_to_second_order_in_dt():
    _pin_langmuir_energy()


# ---------------------------------------------------------------------------
# Planted mistakes: every one must fail at least one pin above.

_MUTANTS = {
    "W_E without 1/2": ("out[0] = 0.5 * we * dV;", "out[0] = we * dV;"),
    "W_E without dV": ("out[0] = 0.5 * we * dV;", "out[0] = 0.5 * we;"),
    "W_B without 1/2": ("out[1] = 0.5 * wb * dV;", "out[1] = wb * dV;"),
    "W_B without dV": ("out[1] = 0.5 * wb * dV;", "out[1] = 0.5 * wb;"),
    "K with gamma": ("k += s->w[p] * s->m * (gm - 1.0);", "k += s->w[p] * s->m * gm;"),
    "K without m": ("k += s->w[p] * s->m * (gm - 1.0);", "k += s->w[p] * (gm - 1.0);"),
    "K without w": ("k += s->w[p] * s->m * (gm - 1.0);", "k += s->m * (gm - 1.0);"),
}


def _pins_fail() -> bool:
    for pin in (_pin_yee_field_energy, _pin_kinetic_limits, _pin_langmuir_energy):
        try:
            pin()
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_planted_mistakes_fail_a_pin(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "pic_oracle.c")).read()
    old, new = _MUTANTS[name]
    assert src.count(old) == 1
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    L = oracle.load_library(oracle.build(str(path), str(tmp_path / "libmutant.so")))
    prev = oracle.use_library(L)
    try:
        assert _pins_fail(), f"no pin caught: {name}"
    finally:
        oracle.use_library(prev)


def test_trace_without_time_centred_kinetic_term_fails_a_pin(monkeypatch):
    monkeypatch.setattr(oracle, "energy_trace_total", lambda tr: tr[:, 0] + tr[:, 1] + tr[:, 3])
    assert _pins_fail()
