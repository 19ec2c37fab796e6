"""FP64 oracle for the Monte Carlo electron-impact ionisation step
(TEST INFRASTRUCTURE; only tests, the smoke check and the CPU-baseline leg
of the benchmark use it).

The paper's introduction adds a Monte Carlo atomic-physics step to the PIC
cycle: per ion and step, a transition probability from rates that depend on
the local electron population.  Here that step is Lotz electron-impact
ionisation.  Each charge state has one or more subshells j (the outermost
first), each with binding energy P_j, electron count q_j and constants
a_j, b_j, c_j (Lotz 1968; b = c = 0 and a = 4.5e-14 cm^2 eV^2 is the plain
single-shell form of Lotz 1967):

  sigma(E) = sum_j a_j q_j ln(E/P_j) / (E P_j) [1 - b_j e^{-c_j (E/P_j - 1)}]   (E >= P_j)
  <sigma v> = integral of sigma(E) v(E) f(E) dE over a Maxwellian f at kT
            = vbar / kT sum_j (a_j q_j / P_j) e^{-P_j/kT}
                 * sum_k w_k ln(1 + x_k r_j) (1 - b_j e^{-c_j x_k r_j}),  r_j = kT / P_j

with the substitution E = P_j + kT x per subshell and 64-point
Gauss-Laguerre nodes x_k, weights w_k (numpy's `laggauss`),
vbar = c sqrt(8 kT / (pi m_e c^2)).  The rate per ion is nu = n_e <sigma v>;
over a step of dt/omega_p seconds the ion ionises with probability
p = 1 - exp(-nu dt / omega_p), decided by one Philox uniform.  n_e and T_e
come from nearest-grid-point moments of the electrons in the ion's cell
(drift removed).

Two options widen the step (both off by default):
  - max_events > 1: successive ionisations within one step.  With n_e and
    kT frozen over the step, the ion's waiting time in state Z is exponential
    with rate nu_Z; the j-th event happens if the sum of the first j waiting
    times E_i / nu_{Z+i} (E_i = -ln(1 - u_i), unit exponentials) is below
    the step, for at most max_events events.
  - energy_loss: the electrons of the ion's cell pay the ionisation energy.
    Their momenta about the cell's mean momentum are scaled by
    f = sqrt(max(0, 1 - dE / (3/2 N kT))), dE the sum of w P_Z over the
    cell's events and N kT the cell's weight times temperature, which lowers
    the cell's kT (as the moments define it) by exactly dE / (3/2 N).
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


def shell_sum(r, b=0.0, c=0.0):
    """sum_k w_k ln(1 + x_k r) (1 - b e^{-c x_k r}): GL-64 for the integral
    over x >= 0 of ln(1 + x r) (1 - b e^{-c x r}) e^{-x}."""
    r = np.asarray(r, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x, w = gl64()
    s = np.zeros(np.broadcast(r, b, c).shape)
    for xk, wk in zip(x, w):
        s = s + wk * np.log1p(xk * r) * (1.0 - b * np.exp(-c * xk * r))
    return s


def sigma_v_exact(kT, P, q, a=LOTZ_A, b=0.0, c=0.0):
    """Maxwellian-averaged Lotz rate coefficient (cm^3/s) of one subshell by
    GL-64.  kT, P in eV (arrays broadcast); zero where kT <= 0."""
    kT = np.asarray(kT, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    kTs = np.where(kT > 0, kT, 1.0)
    z = P / kTs
    out = vbar(kTs) * (a * q / (P * kTs)) * np.exp(-z) * shell_sum(kTs / P, b, c)
    return np.where(kT > 0, out, 0.0)


def sigma_v_shells(kT, shells):
    """<sigma v> of a charge state: the sum over its subshells (P, a, b, c, q)."""
    return sum(sigma_v_exact(kT, P, q, a, b, c) for (P, a, b, c, q) in shells)


def ln_rate_exact(kT, ne, P, q, a=LOTZ_A, b=0.0, c=0.0):
    """ln nu for nu = n_e <sigma v> of one subshell (1/s), without underflow."""
    kT, ne, P, q = (np.asarray(v, dtype=np.float64) for v in (kT, ne, P, q))
    z = P / kT
    return np.log(ne * vbar(kT) * a * q / (P * kT)) - z + np.log(shell_sum(kT / P, b, c))


def ln_rate_shells(kT, ne, shells):
    """ln nu of a charge state with several subshells, without underflow:
    the factor e^{-P_0/kT} of the outermost subshell (the smallest P) is
    taken out of the sum."""
    kT = np.asarray(kT, dtype=np.float64)
    ne = np.asarray(ne, dtype=np.float64)
    P0 = min(sh[0] for sh in shells)
    acc = np.zeros(np.broadcast(kT, ne).shape)
    for (P, a, b, c, q) in shells:
        acc = acc + (a * q / P) * np.exp(-(P - P0) / kT) * shell_sum(kT / P, b, c)
    return np.log(ne * vbar(kT) / kT) - P0 / kT + np.log(acc)


def rate_exact(kT, ne, P, q):
    return np.asarray(ne, dtype=np.float64) * sigma_v_exact(kT, P, q)


def rate_shells(kT, ne, shells):
    return np.asarray(ne, dtype=np.float64) * sigma_v_shells(kT, shells)


def lotz_shells(spc: dict) -> list:
    """The subshells (P, a, b, c, q) of each charge state Z < z_max: the
    species' "lotz_shells"[Z] when given (dicts with keys p_ev, a, b, c, q;
    a, b, c default to the plain form), else the single outermost subshell
    (ionization_ev[Z], 4.5e-14, 0, 0, lotz_q[Z])."""
    out = []
    for z in range(spc["z_max"]):
        if spc.get("lotz_shells"):
            out.append([(float(sh["p_ev"]), float(sh.get("a", LOTZ_A)), float(sh.get("b", 0.0)),
                         float(sh.get("c", 0.0)), float(sh["q"])) for sh in spc["lotz_shells"][z]])
        else:
            out.append([(float(spc["ionization_ev"][z]), LOTZ_A, 0.0, 0.0, float(spc["lotz_q"][z]))])
    return out


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


def ion_uniforms(seed: int, ion_ids, ion_species: int, step: int, nevents: int = 1):
    """The ionisation draws of each ion: uniform j (j < 8) is word j % 4 of
    the Philox block of counter (id, species, 2, step) for j < 4 and of
    counter (id, species, 6, step) for j >= 4.  Returns (n,) for one event,
    else (n, nevents)."""
    out = np.empty((len(ion_ids), nevents))
    for t, pid in enumerate(ion_ids):
        for blk, purpose in ((0, 2), (1, 6)):
            if 4 * blk >= nevents:
                break
            wd = philox4x64_10([int(pid), ion_species, purpose, step], [seed, 0])
            for j in range(4 * blk, min(nevents, 4 * blk + 4)):
                out[t, j] = ((float(int(wd[j - 4 * blk]) >> 11)) + 0.5) * 2.0**-53
    return out[:, 0] if nevents == 1 else out


def ionize_step(st, cfg: dict, e_index: int, ion_index: int, id_base_new: int, ion_id_offset: int,
                uniforms=None, return_details=False):
    """One Monte Carlo ionisation step on an oracle State, in place.

    Per ion with Z < z_max: cell of the ion (NGP), n_e and kT_e of that cell,
    nu = n_e <sigma v>(kT_e; subshells of Z), p = 1 - exp(-nu dt/omega_p); if
    the uniform r < p then Z += 1 and an electron is born at the ion's
    position with the ion's momentum and weight.  Its id is
    id_base_new + (ion id - ion_id_offset) * z_max + (Z_new - 1), unique
    because each ion passes each charge state at most once.

    With max_events = m > 1 the step is the waiting-time chain of the module
    docstring (uniforms of shape (n, m)); with energy_loss the cell's
    electrons (those present before the step) then pay the events' energy.
    """
    g = st.grid
    gc = cfg["grid"]
    spc = cfg["species"][ion_index]
    ion = st.species[ion_index]
    el = st.species[e_index]
    zmax = spc["z_max"]
    m_ev = int(spc.get("max_events", 1))
    shells = lotz_shells(spc)
    dV = g.dx * g.dy * g.dz
    mom = cell_moments(st, e_index)
    ne_c, kT_c = density_temperature(mom, dV, gc["n_ref_cm3"])
    i = np.floor(ion.x).astype(np.int64) % g.nx
    j = np.floor(ion.y).astype(np.int64) % g.ny
    k = np.floor(ion.z).astype(np.int64) % g.nz
    cell = i + g.nx * (j + g.ny * k)
    Z0 = ion.zstate.astype(np.int64)
    ne = ne_c[cell]
    kT = kT_c[cell]
    lit = (ne > 0) & (kT > 0)
    dtp = g.dt / omega_p(gc["n_ref_cm3"])

    def nu_of(Z):
        out = np.zeros(Z.shape)
        for z in range(zmax):
            sel = (Z == z) & lit
            if sel.any():
                out[sel] = rate_shells(kT[sel], ne[sel], shells[z])
        return out

    nu = nu_of(Z0)
    prob = -np.expm1(-nu * dtp)
    if uniforms is None:
        uniforms = ion_uniforms(gc["seed"], ion.id, ion_index, st.step, m_ev)
    U = np.asarray(uniforms, dtype=np.float64).reshape(len(Z0), -1)
    if m_ev == 1:
        nev = ((Z0 < zmax) & (U[:, 0] < prob)).astype(np.int64)
    else:
        nev = chain_events(Z0, zmax, m_ev, U, dtp, lambda Z, e: nu if e == 0 else nu_of(Z))
    fire = nev > 0
    # births: ions in input order, each with its events in order of Z
    src = np.repeat(np.arange(len(Z0)), nev)
    znew = Z0[src] + (np.arange(src.size) - np.repeat(np.cumsum(nev) - nev, nev)) + 1
    new_ids = id_base_new + (ion.id[src] - ion_id_offset) * zmax + (znew - 1)
    dE = None
    if spc.get("energy_loss", 0) and src.size:
        P_of = np.asarray(spc["ionization_ev"][:zmax], dtype=np.float64)
        dE = np.bincount(cell[src], weights=ion.w[src] * P_of[znew - 1], minlength=len(ne_c))
        energy_loss(st, e_index, mom, kT_c, dE)
    ion.zstate[:] = Z0 + nev
    for name in ("x", "y", "z", "ux", "uy", "uz", "w"):
        setattr(el, name, np.ascontiguousarray(np.concatenate([getattr(el, name), getattr(ion, name)[src]])))
    el.id = np.ascontiguousarray(np.concatenate([el.id, new_ids.astype(np.int64)]))
    if return_details:
        return dict(nu=nu, prob=prob, uniforms=uniforms, fire=fire, nevents=nev, ne=ne, kT=kT,
                    new_ids=new_ids, dE=dE)
    return int(src.size)


def chain_events(Z0, zmax: int, m_ev: int, U, dtp: float, nu_fn):
    """Events per ion of the waiting-time chain: starting in state Z0 at t = 0,
    event e (e = 0, 1, ...) adds the waiting time -ln(1 - U[:, e]) / nu_fn(Z, e)
    with Z = Z0 + e, and happens while the running time stays below dtp, Z
    stays below zmax and the rate is positive; at most m_ev events."""
    nev = np.zeros(len(Z0), dtype=np.int64)
    t = np.zeros(len(Z0))
    going = np.asarray(Z0) < zmax
    for e in range(m_ev):
        Z = Z0 + nev
        going &= Z < zmax
        nz = nu_fn(Z, e)
        going &= nz > 0
        t = np.where(going, t + (-np.log1p(-U[:, e])) / np.where(nz > 0, nz, 1.0), t)
        going &= t < dtp
        nev[going] += 1
    return nev


def energy_loss(st, e_index: int, mom, kT_c, dE):
    """Scale the momenta of species e_index about their cell's mean momentum
    by f = sqrt(max(0, 1 - dE / (3/2 N kT))) per cell (N = sum w, kT in eV,
    dE in eV times weight), with the moments taken before the step."""
    g = st.grid
    s = st.species[e_index]
    N = mom[:, 0]
    heat = 1.5 * N * kT_c
    f2 = np.where((dE > 0) & (heat > 0), 1.0 - dE / np.where(heat > 0, heat, 1.0), 1.0)
    f = np.sqrt(np.maximum(f2, 0.0))
    safe = np.where(N > 0, N, 1.0)
    ub = mom[:, 1:4] / safe[:, None]
    cell = (np.floor(s.x).astype(np.int64) % g.nx
            + g.nx * ((np.floor(s.y).astype(np.int64) % g.ny) + g.ny * (np.floor(s.z).astype(np.int64) % g.nz)))
    fc = f[cell]
    s.ux = ub[cell, 0] + fc * (s.ux - ub[cell, 0])
    s.uy = ub[cell, 1] + fc * (s.uy - ub[cell, 1])
    s.uz = ub[cell, 2] + fc * (s.uz - ub[cell, 2])
    return f
