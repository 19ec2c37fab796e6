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

@pytest.mark.parametrize("act", ["silu", "relu"])
def test_mlp_backprop_matches_central_differences(act):
    """Analytic gradients against central differences of the loss (ReLU: no
    pre-activation of these seeded samples lies within h of its kink)."""
    p = mlp.init_params(3)
    T, ne, Z = workloads.loguniform_rate_inputs(5, 32)
    X = mlp.features(T, ne, Z)
    t = workloads.rng(6).normal(size=32)
    loss, g = mlp.loss_and_grad(p, X, t, act)
    h = 1e-6
    r = workloads.rng(7)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in r.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(p, X, t, act)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(p, X, t, act)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-7 * max(1e-3, abs(an)) + 1e-10


def test_mlp_relu_network_is_positively_homogeneous():
    """max(a z, 0) = a max(z, 0) for a > 0: scaling W1, b1, b2 by a and W3 by
    1/a leaves a ReLU network's output unchanged (the property that lets one
    set of base-2 scaled inference weights serve both activations); a SiLU
    network changes.  Its output is also piecewise linear in x0: second
    differences vanish where no unit switches."""
    p = mlp.init_params(11)
    T, ne, Z = workloads.loguniform_rate_inputs(12, 64)
    X = mlp.features(T, ne, Z)
    a = 1.4426950408889634
    q = dict(p, W1=p["W1"] * a, b1=p["b1"] * a, b2=p["b2"] * a, W3=p["W3"] / a)
    y0, _ = mlp.forward(p, X, "relu")
    y1, _ = mlp.forward(q, X, "relu")
    assert np.max(np.abs(y1 - y0)) < 1e-13 * max(1.0, np.max(np.abs(y0)))
    s0, _ = mlp.forward(p, X, "silu")
    s1, _ = mlp.forward(q, X, "silu")
    assert np.max(np.abs(s1 - s0)) > 1e-3
    d = 1e-4
    Xs = [X.copy() for _ in range(3)]
    for k, Xk in enumerate(Xs):
        Xk[:, 0] += (k - 1) * d
    (ym, c0), (yc, c1), (yp, c2) = (mlp.forward(p, Xk, "relu") for Xk in Xs)
    same = np.all((c0["z1"] > 0) == (c2["z1"] > 0), axis=1) & np.all((c0["z2"] > 0) == (c2["z2"] > 0), axis=1)
    assert same.sum() > 50
    assert np.max(np.abs((yp - 2 * yc + ym)[same])) < 1e-11


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


# ---------------------------------------------------------------------------
# Subshells with Lotz's b, c terms; successive events; ionisation-energy loss.

@pytest.mark.parametrize("kT,P,b,c", [(5.0, 11.3, 0.7, 0.4), (40.0, 64.5, 0.3, 2.5), (2.0, 24.4, 0.9, 0.05),
                                      (100.0, 392.0, 0.5, 1.0)])
def test_lotz_bc_subshell_matches_e1_closed_form(kT, P, b, c):
    """With E = P + kT x the b-term integral is e^{c} E1(z + c) / (1 + c/z) (z = P/kT):
    <sigma v> = vbar a q / (P kT) [E1(z) - b e^{c} E1(z + c) / (1 + c/z)]."""
    a, q = 3.9e-14, 2.0
    got = ionize.sigma_v_exact(kT, P, q, a, b, c)
    z = P / kT
    want = ionize.vbar(kT) * a * q / (P * kT) * (special.exp1(z) - b * math.exp(c) * special.exp1(z + c) / (1 + c / z))
    assert abs(got / want - 1) < 1e-12
    # b = 0 is the plain form whatever c is
    assert ionize.sigma_v_exact(kT, P, q, a, 0.0, c) == pytest.approx(ionize.sigma_v_exact(kT, P, q, a), rel=1e-15)


def test_lotz_two_subshells_direct_maxwellian_integral():
    """sigma(E) summed over two subshells with their own thresholds and b, c,
    integrated against the Maxwellian directly (no substitution)."""
    shells = [(24.4, 4.0e-14, 0.6, 0.6, 1.0), (300.0, 3.0e-14, 0.75, 0.3, 2.0)]
    me_g = 9.1093837015e-28
    erg_per_ev = 1.602176634e-12
    for kT, tol in ((20.0, 1e-8), (150.0, 3e-6)):     # GL-64 error grows once kT > P (see above)
        def integrand(E):
            sig = 0.0
            for (P, a, b, c, q) in shells:
                if E >= P:
                    sig += a * q * math.log(E / P) / (E * P) * (1 - b * math.exp(-c * (E / P - 1)))
            v = math.sqrt(2 * E * erg_per_ev / me_g)
            f = 2.0 / math.sqrt(math.pi) * kT**-1.5 * math.sqrt(E) * math.exp(-E / kT)
            return sig * v * f
        lo, hi = shells[0][0], shells[1][0]
        v1, _ = integrate.quad(integrand, lo, hi, epsabs=0, epsrel=1e-12, limit=400)
        v2, _ = integrate.quad(integrand, hi, hi + 200 * kT, epsabs=0, epsrel=1e-12, limit=400)
        got = ionize.sigma_v_shells(kT, shells)
        assert abs(got / (v1 + v2) - 1) < tol


def test_ln_rate_shells_without_underflow():
    shells = [(392.0, 4.5e-14, 0.2, 0.5, 2.0), (490.0, 4.5e-14, 0.0, 0.0, 1.0)]
    ne = np.array([1e21, 3e20])
    kT = np.array([60.0, 0.25])         # e^{-392/0.25} underflows in <sigma v>
    ln = ionize.ln_rate_shells(kT, ne, shells)
    assert np.all(np.isfinite(ln))
    assert abs(ln[0] - math.log(ionize.rate_shells(kT[0], ne[0], shells))) < 1e-13 * abs(ln[0])
    assert ionize.rate_shells(kT[1], ne[1], shells) == 0.0
    # one subshell: the single-shell formula
    one = [shells[0]]
    assert np.allclose(ionize.ln_rate_shells(kT, ne, one), ionize.ln_rate_exact(kT, ne, 392.0, 2.0, 4.5e-14, 0.2, 0.5),
                       rtol=1e-14, atol=0)


def test_chain_events_poisson_for_equal_rates():
    """With the same rate nu in every state the number of events in dt is a
    Poisson(nu dt) count truncated at min(m, z_max - Z0)."""
    n, m, zmax = 200_000, 4, 6
    nu, dtp = 1.0, 1.3
    U = workloads.rng(11).random((n, m))
    Z0 = np.full(n, 1)
    nev = ionize.chain_events(Z0, zmax, m, U, dtp, lambda Z, e: np.full(Z.shape, nu))
    lam = nu * dtp
    pk = [math.exp(-lam) * lam**k / math.factorial(k) for k in range(m)]
    pk.append(1 - sum(pk))
    for k in range(m + 1):
        got = np.mean(nev == k)
        assert abs(got - pk[k]) < 5 * math.sqrt(pk[k] * (1 - pk[k]) / n), (k, got, pk[k])
    # truncation by the charge states left
    nev = ionize.chain_events(np.full(n, zmax - 2), zmax, m, U, dtp, lambda Z, e: np.full(Z.shape, nu))
    assert nev.max() == 2 and np.mean(nev == 2) == pytest.approx(1 - pk[0] - pk[1], abs=5e-3)


def test_chain_events_two_rates_hypoexponential():
    """Two events with rates nu1 != nu2 happen within dt with probability
    1 - (nu2 e^{-nu1 dt} - nu1 e^{-nu2 dt}) / (nu2 - nu1)."""
    n = 200_000
    nu1, nu2, dtp = 0.8, 2.5, 1.0
    U = workloads.rng(12).random((n, 2))
    nev = ionize.chain_events(np.zeros(n, dtype=np.int64), 3, 2, U, dtp,
                              lambda Z, e: np.where(Z == 0, nu1, nu2))
    p2 = 1 - (nu2 * math.exp(-nu1 * dtp) - nu1 * math.exp(-nu2 * dtp)) / (nu2 - nu1)
    p1 = 1 - math.exp(-nu1 * dtp) - p2
    assert abs(np.mean(nev == 2) - p2) < 5 * math.sqrt(p2 * (1 - p2) / n)
    assert abs(np.mean(nev == 1) - p1) < 5 * math.sqrt(p1 * (1 - p1) / n)


def test_multi_event_step_forced_uniforms_and_ids():
    cfg, st = _small_carbon_state()
    cfg["species"][1]["max_events"] = 3
    n_ion = st.species[1].n
    ntot = sum(s.n for s in st.species)
    n_e0 = st.species[0].n
    s0 = st.copy()
    d = ionize.ionize_step(s0, cfg, 0, 1, ntot, n_e0, uniforms=np.full((n_ion, 3), 1e-300), return_details=True)
    # C2+ (z_max 6): every ion in a cell with electrons climbs three states
    assert np.all(s0.species[1].zstate == 5)
    assert s0.species[0].n == n_e0 + 3 * n_ion
    ids = s0.species[0].id[n_e0:]
    assert len(set(ids.tolist())) == ids.size
    want = ntot + np.repeat((st.species[1].id - n_e0) * 6, 3) + np.tile([2, 3, 4], n_ion)
    assert np.array_equal(ids, want)
    s1 = st.copy()
    assert ionize.ionize_step(s1, cfg, 0, 1, ntot, n_e0, uniforms=np.full((n_ion, 3), 1 - 2.0**-53)) == 0
    # the first decision equals the single-event rule (u < 1 - e^{-nu dt}) away from ties
    s2 = st.copy()
    d = ionize.ionize_step(s2, cfg, 0, 1, ntot, n_e0, return_details=True)
    u0 = d["uniforms"][:, 0]
    clear = np.abs(u0 - d["prob"]) > 1e-12
    assert np.array_equal((d["nevents"] > 0)[clear], (u0 < d["prob"])[clear])
    assert np.all(d["nevents"] <= 3)


def test_energy_loss_lowers_cell_temperature_by_the_event_energy():
    """After the step, 3/2 N (kT_before - kT_after) = dE in every cell whose
    electrons can pay (moments of the pre-existing electrons), the cell's mean
    momentum is unchanged, and a cell that cannot pay is left at kT = 0."""
    cfg, st = _small_carbon_state()
    cfg["species"][1]["energy_loss"] = 1
    ntot = sum(s.n for s in st.species)
    n_e0 = st.species[0].n
    g = st.grid
    dV = g.dx * g.dy * g.dz
    m0 = ionize.cell_moments(st, 0)
    _, kT0 = ionize.density_temperature(m0, dV, 1e21)
    s1 = st.copy()
    u = np.where(np.arange(st.species[1].n) % 3 == 0, 0.0, 1.0)     # every third ion fires
    d = ionize.ionize_step(s1, cfg, 0, 1, ntot, n_e0, uniforms=u, return_details=True)
    assert d["fire"].sum() > 0
    old = s1.copy()
    for name in ("x", "y", "z", "ux", "uy", "uz", "w", "id"):
        setattr(old.species[0], name, getattr(s1.species[0], name)[:n_e0].copy())
    m1 = ionize.cell_moments(old, 0)
    _, kT1 = ionize.density_temperature(m1, dV, 1e21)
    N = m0[:, 0]
    dE = d["dE"]
    pay = (dE > 0) & (dE < 1.5 * N * kT0)
    assert pay.sum() > 0
    assert np.allclose(1.5 * N[pay] * (kT0[pay] - kT1[pay]), dE[pay], rtol=1e-9, atol=0)
    assert np.allclose(kT1[dE == 0], kT0[dE == 0], rtol=1e-12, atol=0)
    assert np.allclose(m1[:, 1:4], m0[:, 1:4], rtol=0, atol=1e-12 * np.abs(m0[:, 1:4]).max())
    # a cell that cannot pay
    f = ionize.energy_loss(st.copy(), 0, m0, kT0, np.where(np.arange(len(N)) == 0, 10 * 1.5 * N * kT0, 0.0))
    assert f[0] == 0.0 and np.all(f[1:] == 1.0)
