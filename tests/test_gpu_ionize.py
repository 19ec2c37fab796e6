"""GPU parity of the Monte Carlo ionisation step and of the learned rate
surrogate against the FP64 oracle, through the C ABI.

Exact path: ln nu from the GPU's FP64 64-point Gauss-Laguerre quadrature
agrees with the oracle's to 1e-12; cell moments agree to 1e-12; ionisation
decisions on the same Philox uniforms agree except where |r - p| is below the
FP64 rounding of p, and every new electron matches its ion.
Surrogate: BF16-MFMA training gradients within 2e-2 (relative, per tensor) of
the oracle's FP64 backpropagation with cosine > 0.999; after training on GPU
the median relative rate error on a held-out set is <= 1 %, and the network
beats its analytic prior alone.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import ionize, mlp
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_02862_amd as pkg
    pkg.load()
    return pkg


def _print(*a):
    print(*a, flush=True)


def _carbon_cfg(box=(16, 16, 8)):
    return workloads.reduced(3, *box)


# ---------------------------------------------------------------------------
# exact rates and moments

def test_exact_rate_matches_oracle(P):
    cfg = _carbon_cfg()
    T, ne, Z = workloads.loguniform_rate_inputs(11, 20000, t_range=(0.5, 3e4), n_range=(1e18, 1e24))
    with P.Pic(cfg) as pic:
        got = pic.rate_eval("exact", 1, T, ne, Z)
    Pz = np.array(workloads.CARBON_IONIZATION_EV)[Z]
    qz = np.array(workloads.CARBON_LOTZ_Q)[Z]
    want = ionize.ln_rate_exact(T, ne, Pz, qz)
    fin = np.isfinite(want)
    err = np.abs(got[fin] - want[fin])
    _print("exact ln-rate max abs err", err.max())
    assert np.all(np.isfinite(got[fin]))
    assert err.max() < 1e-12 * np.maximum(1.0, np.abs(want[fin])).max()


def test_cell_moments_match_oracle(P):
    cfg = _carbon_cfg()
    with P.Pic(cfg) as pic:
        pic.step(3)
        st = parity.pull_state(pic, oracle.init_state(cfg))
        ne, kT = pic.cell_moments(1)
    g = st.grid
    ne_ref, kT_ref = ionize.density_temperature(ionize.cell_moments(st, 0), g.dx * g.dy * g.dz,
                                                cfg["grid"]["n_ref_cm3"])
    assert np.max(np.abs(ne / ne_ref - 1)) < 1e-12
    assert np.max(np.abs(kT - kT_ref) / kT_ref) < 1e-10


def test_cell_moments_device_arrays_are_the_librarys(P):
    """pic_cell_moments_device leaves n_e and kT_e in the library's own device
    arrays: their contents equal the host copy, and the addresses stay the
    same from call to call."""
    import ctypes
    cfg = _carbon_cfg()
    with P.Pic(cfg) as pic:
        pic.step(3)
        ne_h, kT_h = pic.cell_moments(1)
        pne, pkT = pic.cell_moments_device(1)
        torch.cuda.synchronize()
        # the HIP runtime already in the process (torch's), for a plain copy
        hip = ctypes.CDLL(next(l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l))
        ne_d, kT_d = np.empty(ne_h.size), np.empty(kT_h.size)
        for dst, src in ((ne_d, pne), (kT_d, pkT)):
            rc = hip.hipMemcpy(ctypes.c_void_p(dst.ctypes.data), ctypes.c_void_p(src), ctypes.c_size_t(dst.nbytes), 2)
            assert rc == 0
        assert pic.cell_moments_device(1) == (pne, pkT)
    # recomputed: FP64 LDS sums, equal up to their order
    assert np.allclose(ne_d, ne_h, rtol=1e-13, atol=0) and np.allclose(kT_d, kT_h, rtol=1e-12, atol=1e-12)
    assert ne_h.max() > 0 and kT_h.max() > 0


def _shared_carbon_state(pic, cfg, warm=4):
    st = oracle.init_state(cfg)
    oracle.step(st, warm)
    s0 = parity.shared_start(pic, st)
    s0.step = 0  # the handle has taken no cycles: its ionisation draws use step 0
    return s0


def test_ionize_exact_matches_oracle(P):
    # 32x16x16 cells, 32768 C2+ ions: this state fires about 80 events in the
    # step (the oracle counts 84), enough to compare decisions, appended
    # electrons and their ids on a real sample
    box = (32, 16, 16)
    cfg = _carbon_cfg(box)
    ncell = box[0] * box[1] * box[2]
    n_e0, n_c0 = ncell * 8, ncell * 4
    with P.Pic(cfg) as pic:
        s0 = _shared_carbon_state(pic, cfg)
        ref = s0.copy()
        d = ionize.ionize_step(ref, cfg, 0, 1, n_e0 + n_c0, n_e0, return_details=True)
        stats = pic.ionize("exact")
        got = parity.pull_state(pic, s0)
    fire_ref = d["fire"]
    _print("ionised gpu/ref", stats["ionized"], int(fire_ref.sum()), "active", stats["ions_active"])
    assert stats["ions_active"] == n_c0
    assert fire_ref.sum() > 20  # the test state must actually ionise
    # decisions may differ only where r is within FP64 rounding of p
    zg = got.species[1].zstate
    zr = ref.species[1].zstate
    differ = np.nonzero(zg != zr)[0]
    assert len(differ) <= 2
    for k in differ:
        assert abs(d["uniforms"][k] - d["prob"][k]) < 1e-12 * max(d["prob"][k], 1e-300)
    if len(differ) == 0:
        assert stats["ionized"] == int(fire_ref.sum())
        # new electrons: same ids, born on their ion with its momentum and weight
        eg, er = got.species[0], ref.species[0]
        er.sort_by_id()
        assert np.array_equal(eg.id, er.id)
        for a in ("x", "y", "z", "ux", "uy", "uz", "w"):
            assert np.array_equal(getattr(eg, a), getattr(er, a)), a


def test_ionisation_conserves_charge_over_a_run(P):
    """Gauss's law G = div E - rho keeps its reference value through PIC
    cycles interleaved with ionisation (each event adds +1 to an ion and a -1
    electron at the same position)."""
    cfg = _carbon_cfg()
    with P.Pic(cfg) as pic:
        total = 0
        for _ in range(5):
            pic.step(2)
            total += pic.ionize("exact")["ionized"]
        m = pic.moments()
    _print("ionised over run", total, "gauss", m["gauss_max"], "rho_max", m["rho_max"])
    assert total > 0
    assert m["gauss_max"] <= 1e-4 * m["rho_max"]


def test_ionize_requires_surrogate_before_mlp_mode(P):
    cfg = _carbon_cfg((8, 8, 4))
    with P.Pic(cfg) as pic:
        with pytest.raises(P.PicError) as e:
            pic.ionize("mlp")
        assert e.value.code == -7


# ---------------------------------------------------------------------------
# surrogate: gradients, training, accuracy, gain

def _bf16(a):
    a = np.asarray(a, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _flat(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def _unflat(v):
    o, d = 0, {}
    for k, shape in (("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)), ("b3", (1,))):
        n = int(np.prod(shape))
        d[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return d


@pytest.mark.parametrize("act", ["silu", "relu"])
def test_mlp_gradient_matches_oracle_backprop(P, act):
    cfg = _carbon_cfg((8, 8, 4))
    p = mlp.init_params(4)
    flat = _bf16(_flat(p))           # BF16-representable weights on both sides
    pref = _unflat(flat)
    T, ne, Z = workloads.loguniform_rate_inputs(12, 4096)
    X = mlp.features(T, ne, Z)
    X = _bf16(X).astype(np.float64)  # features the GPU sees exactly
    t = workloads.rng(13).normal(size=4096)
    loss_ref, g_ref = mlp.loss_and_grad(pref, X, t, act)
    with P.Pic(cfg) as pic:
        pic.mlp_set_params(1, flat, [0.0, 1.0], activation=act)
        loss, g = pic.mlp_loss_grad(1, X, t)
    gg = _unflat(g)
    _print("loss gpu/ref", loss, loss_ref)
    assert abs(loss / loss_ref - 1) < 2e-2
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        a, b = gg[k].ravel(), g_ref[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        _print(k, "rel", rel, "cos", cos)
        assert rel < 2e-2 and cos > 0.999, k


def test_mlp_training_is_bitwise_reproducible(P):
    """The training step sums its gradient without atomics (per-workgroup rows
    added in a fixed order), so two trainings from one seed give the same
    parameters bit for bit, and the gradient entry point the same gradient."""
    cfg = _carbon_cfg((8, 8, 4))
    out = []
    for _ in range(2):
        with P.Pic(cfg) as pic:
            rep = pic.mlp_train(1, seed=7, n_train=65536, batch=4096, steps=300)
            p = pic.mlp_get_params(1)
            T, ne, Z = workloads.loguniform_rate_inputs(14, 1024)
            X = mlp.features(T, ne, Z)
            g = pic.mlp_loss_grad(1, X, workloads.rng(15).normal(size=1024))
        out.append((rep, p, g))
    (r0, p0, g0), (r1, p1, g1) = out
    assert r0["loss_first"] == r1["loss_first"] and r0["loss_last"] == r1["loss_last"]
    assert r0["loss_last"] < r0["loss_first"]
    assert np.array_equal(p0[0].view(np.uint32), p1[0].view(np.uint32))
    assert np.array_equal(p0[1], p1[1])
    assert g0[0] == g1[0] and np.array_equal(g0[1].view(np.uint32), g1[1].view(np.uint32))


@pytest.mark.parametrize("act", ["silu", "relu"])
def test_mlp_inference_matches_oracle_forward(P, act):
    """The fused inference kernel (transposed MFMA layout, augmented layer-1 K,
    head on MFMA, hidden layers in base 2) evaluates the same network as the
    oracle's plain FP64 forward.  The GPU differs by the BF16 rounding of the
    128 activations (relative 2^-9 each), by the BF16 re-rounding of W1 and
    W3 after the base-2 scaling (log2 e into W1, 1/log2 e into W3; relative
    2^-9 each), FP32 sums and the FP32 prior; per sample, |d ln nu| must stay
    within s times the first-order bound of those roundings propagated
    through the activation's derivative (ReLU: its Lipschitz constant 1, since
    a rounding may move a pre-activation across 0), W2 and W3, plus 1e-4 for
    the FP32 parts."""
    cfg = _carbon_cfg((8, 8, 4))
    r = workloads.rng(31)
    p = mlp.init_params(5)
    p["b1"] = r.uniform(-0.5, 0.5, 64)
    p["b2"] = r.uniform(-0.5, 0.5, 64)
    p["b3"] = np.array([0.3])
    flat = _flat(p).astype(np.float32)
    for k, (o, n) in {"W1": (0, 512), "W2": (576, 4096), "W3": (4736, 64)}.items():
        flat[o:o + n] = _bf16(flat[o:o + n])
    pref = _unflat(flat)
    mu, s = -0.1, 0.5
    T, ne, Z = workloads.loguniform_rate_inputs(32, 50000)
    Pt, qt = workloads.CARBON_IONIZATION_EV, workloads.CARBON_LOTZ_Q
    with P.Pic(cfg) as pic:
        pic.mlp_set_params(1, flat, [mu, s], [1.0, 1e4, 1e19, 1e23], activation=act)
        got = pic.rate_eval("mlp", 1, T, ne, Z)
    want = mlp.ln_rate(pref, mu, s, T, ne, Z, Pt, qt, act=act)
    X = mlp.features(T, ne, Z)
    _, c = mlp.forward(pref, X, act)
    dact = mlp.dsilu if act == "silu" else np.ones_like
    dz1 = 2.0**-9 * (np.abs(X) @ np.abs(pref["W1"]).T)                       # W1 re-rounding
    dh1 = np.abs(c["h1"]) * 2.0**-9 + np.abs(dact(c["z1"])) * dz1            # + activation rounding
    dz2 = dh1 @ np.abs(pref["W2"]).T
    bound = (np.abs(dact(c["z2"])) * dz2 + 2 * np.abs(c["h2"]) * 2.0**-9) @ np.abs(pref["W3"][0])  # + W3
    err = np.abs(got - want)
    _print("inference vs oracle: max", err.max(), "median", np.median(err), "max err/bound",
           (err / (s * bound + 1e-4)).max())
    assert np.all(np.isfinite(got))
    assert np.all(err <= s * 1.1 * bound + 1e-4)


@pytest.fixture(scope="module", params=["silu", "relu"])
def trained(P, request):
    """Train the surrogate on the GPU with the full recipe (1M samples), once
    per hidden activation."""
    cfg = _carbon_cfg((8, 8, 4))
    tr = dict(workloads.MLP_TRAIN, activation=request.param)
    pic = P.Pic(cfg)
    rep = pic.mlp_train(1, seed=workloads.MLP_TRAIN_SEED, **tr)
    _print("training report", request.param, rep)
    yield pic, rep
    pic.close()


def test_mlp_training_converges(trained):
    pic, rep = trained
    assert rep["loss_last"] < 1e-2 * rep["loss_first"]
    assert rep["steps"] == workloads.MLP_TRAIN["steps"]


def test_mlp_rate_error_and_gain_on_heldout_set(trained):
    """Median relative rate error <= 1 % against the exact GL-64 rate (the
    reference), on held-out log-uniform inputs; the analytic prior alone is
    reported for the gain."""
    pic, _ = trained
    T, ne, Z = workloads.loguniform_rate_inputs(workloads.MLP_HELDOUT_SEED, 1_000_000)
    got = pic.rate_eval("mlp", 1, T, ne, Z)
    Pz = np.array(workloads.CARBON_IONIZATION_EV)[Z]
    qz = np.array(workloads.CARBON_LOTZ_Q)[Z]
    exact = ionize.ln_rate_exact(T, ne, Pz, qz)
    prior = mlp.ln_rate_prior(T, ne, Pz, qz)
    rel = np.abs(np.expm1(got - exact))
    relp = np.abs(np.expm1(prior - exact))
    _print("surrogate median/p99/max", np.median(rel), np.quantile(rel, 0.99), rel.max(),
           "prior median", np.median(relp))
    assert np.median(rel) <= 1e-2
    assert np.median(rel) < 0.1 * np.median(relp)


def test_mlp_out_of_range_uses_exact_fallback(trained):
    pic, _ = trained
    T = np.array([0.3, 5e4, 100.0, 100.0])
    ne = np.array([1e21, 1e21, 1e17, 1e25])
    Z = np.array([0, 1, 2, 3])
    got = pic.rate_eval("mlp", 1, T, ne, Z)
    want = pic.rate_eval("exact", 1, T, ne, Z)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_mlp_params_roundtrip(trained):
    pic, _ = trained
    p, ms, rng, act = pic.mlp_get_params(1)
    assert np.all(np.isfinite(p)) and ms[1] > 0
    assert tuple(rng) == (1.0, 1e4, 1e19, 1e23)
    assert act in ("silu", "relu")
    # a copy through set_params evaluates identically
    T, ne, Z = workloads.loguniform_rate_inputs(44, 4096)
    with type(pic)(_carbon_cfg((8, 8, 4))) as other:
        other.mlp_set_params(1, p, ms, rng, act)
        assert np.array_equal(other.rate_eval("mlp", 1, T, ne, Z), pic.rate_eval("mlp", 1, T, ne, Z))


def test_ionize_mlp_tracks_exact(trained, P):
    """On one state, the surrogate's per-ion rates match the exact ones to the
    surrogate's accuracy, and the ionisation count to binomial noise."""
    pic_tr, _ = trained
    params, ms, rng, act = pic_tr.mlp_get_params(1)
    cfg = _carbon_cfg()
    counts = {}
    for mode in ("exact", "mlp"):
        with P.Pic(cfg) as pic:
            pic.mlp_set_params(1, params, ms, rng, act)
            pic.step(2)
            counts[mode] = pic.ionize(mode)
    _print(counts)
    a, b = counts["exact"]["ionized"], counts["mlp"]["ionized"]
    assert abs(a - b) <= 5 * np.sqrt(max(a, 1)) + 2
    assert counts["mlp"]["ions_active"] == counts["exact"]["ions_active"]


def test_ionize_mlp_with_every_ion_out_of_range_equals_exact(trained, P):
    """A trained range that excludes every cell sends every ion through the
    surrogate path's exact fallback (the compacted list and its FP64
    quadrature kernel): from one shared state the step must then reproduce
    the exact step (same rates, same Philox uniforms, same decisions, same
    new electrons)."""
    pic_tr, _ = trained
    params, ms, _, act = pic_tr.mlp_get_params(1)
    cfg = _carbon_cfg()
    with P.Pic(cfg) as pic:
        s0 = _shared_carbon_state(pic, cfg, warm=2)
    out = {}
    for mode in ("exact", "mlp"):
        with P.Pic(cfg) as pic:
            parity.push_state(pic, s0)
            pic.mlp_set_params(1, params, ms, [1e5, 1e6, 1e19, 1e23], act)  # kT < 1e5 eV everywhere
            stats = pic.ionize(mode)
            el = pic.get_particles(0)
            o = np.argsort(el["id"], kind="stable")  # appended electrons: their order is not defined
            out[mode] = (stats, pic.get_particles(1), {k: v[o] for k, v in el.items()})
    se, ions_e, el_e = out["exact"]
    sm, ions_m, el_m = out["mlp"]
    _print("exact", se, "mlp", sm)
    assert sm["fallback"] == sm["ions_active"] == se["ions_active"] > 0
    assert sm["ionized"] == se["ionized"] > 0
    assert np.array_equal(ions_e["zstate"], ions_m["zstate"])
    for k in ("id", "x", "y", "z", "ux", "uy", "uz", "w"):
        assert np.array_equal(el_e[k], el_m[k]), k


# ---------------------------------------------------------------------------
# full size: the benchmark's ionisation workload

def test_full_size_carbon_ionize_sampled_parity(P):
    """128^3, 8 electrons + 4 C2+ per cell (25M particles), exact rates, the
    launch configuration the benchmark times: cell moments of every cell from
    the oracle over all electrons pulled from the GPU; for a sample of ions,
    the oracle's GL-64 rate, Philox draw and decision against the GPU's new
    charge state; every sampled event's electron sits on its ion."""
    from types import SimpleNamespace
    cfg = workloads.config(3)
    gc = cfg["grid"]
    ncell = gc["nx"] * gc["ny"] * gc["nz"]
    n_e0, n_c0 = ncell * 8, ncell * 4
    _print("full-size 128^3 carbon ionisation sampled parity")
    with P.Pic(cfg) as pic:
        pic.step(2)
        el = pic.get_particles(0)
        ion = pic.get_particles(1)
        ne_g, kT_g = pic.cell_moments(1)
        stats = pic.ionize("exact")
        ion2 = pic.get_particles(1)
        el2 = pic.get_particles(0)
    g = oracle.grid_from_config(cfg)
    st = SimpleNamespace(grid=g, species=[SimpleNamespace(**{k: el[k].astype(np.float64)
                                                             for k in ("x", "y", "z", "ux", "uy", "uz", "w")})])
    ne_r, kT_r = ionize.density_temperature(ionize.cell_moments(st, 0), g.dx * g.dy * g.dz, gc["n_ref_cm3"])
    assert np.max(np.abs(ne_g / ne_r - 1)) < 1e-12
    assert np.max(np.abs(kT_g - kT_r) / kT_r) < 1e-10
    # sampled ions: GPU decision against the oracle's
    o1, o2 = np.argsort(ion["id"]), np.argsort(ion2["id"])
    assert np.array_equal(ion["id"][o1], ion2["id"][o2])
    k = workloads.rng(91).choice(n_c0, 20000, replace=False)
    ids = ion["id"][o1][k]
    Z0 = ion["zstate"][o1][k]
    Z1 = ion2["zstate"][o2][k]
    x, y, z = (ion[c][o1][k] for c in ("x", "y", "z"))
    cell = ((np.floor(x).astype(np.int64) % g.nx) + g.nx * ((np.floor(y).astype(np.int64) % g.ny)
                                                           + g.ny * (np.floor(z).astype(np.int64) % g.nz)))
    sh = ionize.lotz_shells(cfg["species"][1])
    nu = np.zeros(k.size)
    for zz in np.unique(Z0):
        m = Z0 == zz
        nu[m] = ionize.rate_shells(kT_r[cell[m]], ne_r[cell[m]], sh[int(zz)])
    p = -np.expm1(-nu * gc["dt"] / ionize.omega_p(gc["n_ref_cm3"]))
    u = ionize.ion_uniforms(gc["seed"], ids, 1, 2)
    want = (u < p).astype(np.int64)
    got = (Z1 - Z0).astype(np.int64)
    _print("sampled ions", k.size, "events ref/gpu", int(want.sum()), int(got.sum()), "all events", stats["ionized"])
    assert stats["ions_active"] == n_c0 and stats["ionized"] > 1000
    differ = np.nonzero(got != want)[0]
    assert len(differ) <= 1
    for i in differ:
        assert abs(u[i] - p[i]) < 1e-12 * p[i]
    # electrons of the sampled events, on their ions
    fired = np.nonzero(got == 1)[0]
    assert fired.size > 0
    new_ids = n_e0 + n_c0 + (ids[fired] - n_e0) * cfg["species"][1]["z_max"] + Z0[fired]
    order = np.argsort(el2["id"])
    sid = el2["id"][order]
    at = np.searchsorted(sid, new_ids)
    assert np.array_equal(sid[at], new_ids)
    q = order[at]
    assert np.array_equal(el2["x"][q], x[fired]) and np.array_equal(el2["y"][q], y[fired])
    assert np.array_equal(el2["z"][q], z[fired])
    assert el2["id"].size == n_e0 + stats["ionized"]
