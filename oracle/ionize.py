"""FP64 oracle for the Monte Carlo electron-impact ionisation step
(TEST INFRASTRUCTURE; only tests, the smoke check and the CPU-baseline leg
of the benchmark use it).

The paper's introduction adds a Monte Carlo atomic-physics step to the PIC
cycle: per ion and step, a transition probability from rates that depend on
the local electron population.  Here that step is single-shell Lotz
electron-impact ionisation:

  sigma(E) = a q ln(E/P) / (E P)            for E >= P   (Lotz 1967)
  <sigma v> = integral of sigma(E) v(E) f(E) dE over a Maxwellian f at kT
            = vbar (a q / (P kT)) e^{-P/kT} * sum_k w_k ln(1 + x_k kT / P)

with the substitution E = P + kT x and 64-point Gauss-Laguerre nodes x_k,
weights w_k (numpy's `laggauss`), vbar = c sqrt(8 kT / (pi m_e c^2)).  The
rate per ion is nu = n_e <sigma v>; over a step of dt/omega_p seconds the ion
ionises with probability p = 1 - exp(-nu dt / omega_p), decided by one Philox
uniform.  n_e and T_e come from nearest-grid-point moments of the electrons
in the ion's cell (drift removed).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.laguerre import laggauss

from . import philox4x64_10

ME_C2_EV = 510998.95            # electron rest energy (eV)
C_CM_S = 2.99792458e10          # speed of light (cm/s)
LOTZ_A = 4.5e-14                # Lotz constant (cm^2 eV^2)
E_CHARGE = 1.602176634e-19      # C
EPS0 = 8.8541878128e-12         # F/m
M_E = 9.1093837015e-31          # kg

_GL = None


def gl64():
    global _GL
    if _GL is None:
        _GL = laggauss(64)
    return _GL


def omega_p(n_ref_cm3: float) -> float:
    """Plasma frequency (1/s) of the reference density (SI)."""
    return math.sqrt(n_ref_cm3 * 1e6 * E_CHARGE**2 / (EPS0 * M_E))


def vbar(kT):
    return C_CM_S * np.sqrt(8.0 * kT / (math.pi * ME_C2_EV))


def sigma_v_exact(kT, P, q):
    """Maxwellian-averaged Lotz rate coefficient (cm^3/s) by GL-64.
    kT, P in eV (arrays broadcast); zero where kT <= 0."""
    kT = np.asarray(kT, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    x, w = gl64()
    kTs = np.where(kT > 0, kT, 1.0)
    z = P / kTs
    s = np.zeros(np.broadcast(kTs, P).shape)
    for xk, wk in zip(x, w):
        s = s + wk * np.log1p(xk / z)
    out = vbar(kTs) * (LOTZ_A * q / (P * kTs)) * np.exp(-z) * s
    return np.where(kT > 0, out, 0.0)


def ln_rate_exact(kT, ne, P, q):
    """ln nu for nu = n_e <sigma v> (1/s), evaluated without underflow."""
    kT, ne, P, q = (np.asarray(a, dtype=np.float64) for a in (kT, ne, P, q))
    x, w = gl64()
    z = P / kT
    s = np.zeros(np.broadcast(kT, P).shape)
    for xk, wk in zip(x, w):
        s = s + wk * np.log1p(xk / z)
    return np.log(ne * vbar(kT) * LOTZ_A * q / (P * kT)) - z + np.log(s)


def rate_exact(kT, ne, P, q):
    return np.asarray(ne, dtype=np.float64) * sigma_v_exact(kT, P, q)


def cell_moments(st, e_index: int):
    """Nearest-grid-point moments of one species per cell: sum w, sum w u
    (3 components) and sum w |u|^2.  Returns (ncell, 5)."""
    g = st.grid
    s = st.species[e_index]
    i = np.floor(s.x).astype(np.int64) % g.nx
    j = np.floor(s.y).astype(np.int64) % g.ny
    k = np.floor(s.z).astype(np.int64) % g.nz
    cell = i + g.nx * (j + g.ny * k)
    n = g.nx * g.ny * g.nz
    m = np.zeros((n, 5))
    m[:, 0] = np.bincount(cell, weights=s.w, minlength=n)
    m[:, 1] = np.bincount(cell, weights=s.w * s.ux, minlength=n)
    m[:, 2] = np.bincount(cell, weights=s.w * s.uy, minlength=n)
    m[:, 3] = np.bincount(cell, weights=s.w * s.uz, minlength=n)
    m[:, 4] = np.bincount(cell, weights=s.w * (s.ux**2 + s.uy**2 + s.uz**2), minlength=n)
    return m


def density_temperature(mom, dV: float, n_ref_cm3: float):
    """n_e (cm^-3) and kT_e (eV) per cell from the moments: n_e = (N/dV) n_ref,
    kT = m_e c^2 (sum w u^2 / N - |ubar|^2) / 3; zero where N = 0."""
    N = mom[:, 0]
    safe = np.where(N > 0, N, 1.0)
    ub = mom[:, 1:4] / safe[:, None]
    kT = ME_C2_EV * (mom[:, 4] / safe - np.sum(ub * ub, axis=1)) / 3.0
    ne = N / dV * n_ref_cm3
    kT = np.where(N > 0, np.maximum(kT, 0.0), 0.0)
    ne = np.where(N > 0, ne, 0.0)
    return ne, kT


def ion_uniforms(seed: int, ion_ids, ion_species: int, step: int):
    """The ionisation draw of each ion: Philox counter (id, species, 2, step)."""
    out = np.empty(len(ion_ids))
    for t, pid in enumerate(ion_ids):
        wd = philox4x64_10([int(pid), ion_species, 2, step], [seed, 0])
        out[t] = ((float(int(wd[0]) >> 11)) + 0.5) * 2.0**-53
    return out


def ionize_step(st, cfg: dict, e_index: int, ion_index: int, id_base_new: int, ion_id_offset: int,
                uniforms=None, return_details=False):
    """One Monte Carlo ionisation step on an oracle State, in place.

    Per ion with Z < z_max: cell of the ion (NGP), n_e and kT_e of that cell,
    nu = n_e <sigma v>(kT_e; P_Z, q_Z), p = 1 - exp(-nu dt/omega_p); if the
    uniform r < p then Z += 1 and an electron is born at the ion's position
    with the ion's momentum and weight.  Its id is
    id_base_new + (ion id - ion_id_offset) * z_max + (Z_new - 1), unique
    because each ion passes each charge state at most once.
    """
    g = st.grid
    gc = cfg["grid"]
    spc = cfg["species"][ion_index]
    ion = st.species[ion_index]
    el = st.species[e_index]
    dV = g.dx * g.dy * g.dz
    ne_c, kT_c = density_temperature(cell_moments(st, e_index), dV, gc["n_ref_cm3"])
    i = np.floor(ion.x).astype(np.int64) % g.nx
    j = np.floor(ion.y).astype(np.int64) % g.ny
    k = np.floor(ion.z).astype(np.int64) % g.nz
    cell = i + g.nx * (j + g.ny * k)
    Z = ion.zstate.astype(np.int64)
    active = Z < spc["z_max"]
    P = np.array(spc["ionization_ev"], dtype=np.float64)
    q = np.array(spc["lotz_q"], dtype=np.float64)
    Zc = np.minimum(Z, spc["z_max"] - 1)
    ne = ne_c[cell]
    kT = kT_c[cell]
    nu = np.where(active & (ne > 0) & (kT > 0), rate_exact(kT, ne, P[Zc], q[Zc]), 0.0)
    dtp = g.dt / omega_p(gc["n_ref_cm3"])
    prob = -np.expm1(-nu * dtp)
    if uniforms is None:
        uniforms = ion_uniforms(gc["seed"], ion.id, ion_index, st.step)
    fire = active & (uniforms < prob)
    idx = np.nonzero(fire)[0]
    ion.zstate[idx] += 1
    new_ids = id_base_new + (ion.id[idx] - ion_id_offset) * spc["z_max"] + (ion.zstate[idx] - 1)
    for name in ("x", "y", "z", "ux", "uy", "uz", "w"):
        setattr(el, name, np.ascontiguousarray(np.concatenate([getattr(el, name), getattr(ion, name)[idx]])))
    el.id = np.ascontiguousarray(np.concatenate([el.id, new_ids.astype(np.int64)]))
    if return_details:
        return dict(nu=nu, prob=prob, uniforms=uniforms, fire=fire, ne=ne, kT=kT, new_ids=new_ids)
    return int(idx.size)
