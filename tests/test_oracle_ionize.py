"""Pins of the FP64 ionisation oracle and the surrogate-network reference.

The Gauss-Laguerre rate is checked against the closed form through the
exponential integral E1 (scipy), against direct adaptive integration of
sigma(E) v(E) f(E) over the Maxwellian, and the quadrature rule against its
defining moments.  Cell moments are checked on hand-built cells, the draw
against its definition, charge conservation over a run with ionisation, and
the network's backpropagation against central differences.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads
from oracle import ionize, mlp


def test_gl64_rule_moments():
    x, w = ionize.gl64()
    assert abs(w.sum() - 1.0) < 1e-14
    for m in range(1, 21):
        assert abs(np.sum(w * x**m) / math.factorial(m) - 1.0) < 1e-12


@pytest.mark.parametrize("kT,P", [(5.0, 11.3), (11.3, 11.3), (50.0, 392.0), (204.0, 64.5), (1.0, 490.0)])
def test_lotz_rate_matches_e1_closed_form(kT, P):
    """<sigma v> = vbar a q E1(P/kT) / (P kT); GL-64 is exact to ~1e-13 for kT <= P."""
    q = 2.0
    got = ionize.sigma_v_exact(kT, P, q)
    z = P / kT
    want = ionize.vbar(kT) * ionize.LOTZ_A * q * special.exp1(z) / (P * kT)
    tol = 1e-12 if kT <= P else 1e-6
    assert abs(got / want - 1) < tol


def test_lotz_rate_quadrature_error_grows_with_temperature():
    """GL-64 versus E1 at kT/P ~ 9, 88, 885: the documented quadrature error."""
    for ratio, tol in ((9.0, 3e-6), (88.0, 1e-3), (885.0, 3e-3)):
        P = 11.3
        kT = ratio * P
        got = ionize.sigma_v_exact(kT, P, 1.0)
        want = ionize.vbar(kT) * ionize.LOTZ_A * special.exp1(P / kT) / (P * kT)
        assert abs(got / want - 1) < tol


@pytest.mark.parametrize("kT,P,q", [(20.0, 24.4, 1.0), (300.0, 47.9, 2.0), (3.0, 11.3, 2.0)])
def test_lotz_rate_direct_maxwellian_integral(kT, P, q):
    """Integrate sigma(E) v(E) f(E) dE with f the Maxwellian energy density."""
    me_g = 9.1093837015e-28          # g
    erg_per_ev = 1.602176634e-12

    def integrand(E):
        sigma = ionize.LOTZ_A * q * math.log(E / P) / (E * P)                # cm^2
        v = math.sqrt(2 * E * erg_per_ev / me_g)                              # cm/s
        f = 2.0 / math.sqrt(math.pi) * kT**-1.5 * math.sqrt(E) * math.exp(-E / kT)  # 1/eV
        return sigma * v * f

    val, err = integrate.quad(integrand, P, P + 200 * kT, epsabs=0, epsrel=1e-12, limit=400)
    got = ionize.sigma_v_exact(kT, P, q)
    # m_e in grams and m_e c^2 in eV agree to ~1e-9; above kT = P the GL-64 error (~1e-6) dominates
    assert abs(got / val - 1) < (1e-8 if kT <= P else 3e-6)


def test_cell_moments_and_temperature():
    cfg = workloads.config(0, nx=8, ny=8, nz=4)
    st = oracle.init_state(cfg)
    e = st.species[0]
    # rebuild cell 0 by hand: four electrons with u = drift + (+-a, 0, 0), (0, +-a, 0)
    sel = np.nonzero((np.floor(e.x) == 0) & (np.floor(e.y) == 0) & (np.floor(e.z) == 0))[0]
    assert sel.size == 8
    a, drift = 0.03, np.array([0.1, -0.05, 0.02])
    dirs = [(a, 0, 0), (-a, 0, 0), (0, a, 0), (0, -a, 0), (0, 0, a), (0, 0, -a), (0, 0, 0), (0, 0, 0)]
    for p, dvec in zip(sel, dirs):
        e.ux[p], e.uy[p], e.uz[p] = drift + np.array(dvec)
    mom = ionize.cell_moments(st, 0)
    ne, kT = ionize.density_temperature(mom, 1.0, 1e21)
    assert abs(ne[0] - 1e21) < 1e6
    # <|u - ubar|^2> = 6 a^2 / 8 ; kT = m c^2 * that / 3
    assert abs(kT[0] / (ionize.ME_C2_EV * (6 * a * a / 8) / 3) - 1) < 1e-12


def test_omega_p_reference_density():
    assert abs(ionize.omega_p(1e21) / 1.784e15 - 1) < 1e-3


def _small_carbon_state(box=(8, 8, 4)):
    cfg = workloads.reduced(3, *box)
    st = oracle.init_state(cfg)
    return cfg, st


def test_ionize_step_draw_and_bookkeeping():
    cfg, st = _small_carbon_state()
    ion = st.species[1]
    ntot = sum(s.n for s in st.species)
    n_e0 = st.species[0].n
    d = ionize.ionize_step(st, cfg, 0, 1, ntot, st.species[0].n, return_details=True)
    # uniforms are the Philox draws of (id, species, purpose 2, step)
    w = oracle.philox4x64_10([int(ion.id[5]), 1, 2, 0], [cfg["grid"]["seed"], 0])
    assert d["uniforms"][5] == oracle.u01(w[0])
    assert np.array_equal(d["fire"], d["uniforms"] < d["prob"])
    nf = int(d["fire"].sum())
    assert st.species[0].n == n_e0 + nf
    assert np.all(ion.zstate[d["fire"]] == 3) and np.all(ion.zstate[~d["fire"]] == 2)
    if nf:
        assert np.array_equal(st.species[0].x[n_e0:], ion.x[d["fire"]])
        assert len(set(st.species[0].id.tolist())) == st.species[0].n


def test_ionize_forced_uniforms_and_binomial_count():
    cfg, st = _small_carbon_state()
    n_ion = st.species[1].n
    ntot = sum(s.n for s in st.species)
    s0 = st.copy()
    got = ionize.ionize_step(s0, cfg, 0, 1, ntot, st.species[0].n, uniforms=np.zeros(n_ion))
    assert got == n_ion  # every active ion has p > 0 at kT ~ 200 eV
    s1 = st.copy()
    assert ionize.ionize_step(s1, cfg, 0, 1, ntot, st.species[0].n, uniforms=np.ones(n_ion)) == 0
    s2 = st.copy()
    d = ionize.ionize_step(s2, cfg, 0, 1, ntot, st.species[0].n, return_details=True)
    mean = d["prob"].sum()
    sd = math.sqrt(np.sum(d["prob"] * (1 - d["prob"])))
    assert abs(d["fire"].sum() - mean) < 5 * sd + 1


def test_gauss_invariant_with_ionisation():
    """A new electron is born on its ion and the ion gains +1: rho is unchanged,
    so G = div E - rho stays at its t = 0 value across PIC + ionisation steps."""
    cfg, st = _small_carbon_state((8, 8, 8))
    G0 = oracle.gauss_residual(st)
    ntot = sum(s.n for s in st.species)
    fired = 0
    for _ in range(4):
        oracle.step(st, 1)
        fired += ionize.ionize_step(st, cfg, 0, 1, ntot, 8 * 8 * 8 * 8)
    assert fired > 0
    rmax = np.abs(oracle.rho(st)).max()
    assert np.max(np.abs(oracle.gauss_residual(st) - G0)) < 1e-12 * rmax


# ---------------------------------------------------------------------------
# Surrogate reference network.

def test_mlp_backprop_matches_central_differences():
    p = mlp.init_params(3)
    T, ne, Z = workloads.loguniform_rate_inputs(5, 32)
    X = mlp.features(T, ne, Z)
    t = workloads.rng(6).normal(size=32)
    loss, g = mlp.loss_and_grad(p, X, t)
    h = 1e-6
    r = workloads.rng(7)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in r.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(p, X, t)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(p, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-7 * max(1e-3, abs(an)) + 1e-10


def test_prior_residual_is_bounded_by_e1_inequalities():
    """ln nu_exact - ln nu_prior = ln(e^z E1(z) / ln(1 + 1/z)) lies in
    [ln(ln(1 + 2/z) / (2 ln(1 + 1/z))), 0] (Abramowitz & Stegun 5.1.20)."""
    T, ne, Z = workloads.loguniform_rate_inputs(8, 2000, t_range=(1.0, 200.0))
    P = np.array(workloads.CARBON_IONIZATION_EV)[Z]
    q = np.array(workloads.CARBON_LOTZ_Q)[Z]
    z = P / T
    r = ionize.ln_rate_exact(T, ne, P, q) - mlp.ln_rate_prior(T, ne, P, q)
    lo = np.log(np.log1p(2 / z) / (2 * np.log1p(1 / z)))
    assert np.all(r <= 1e-12) and np.all(r >= lo - 1e-12)
