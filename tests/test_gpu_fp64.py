"""GPU parity of the FP64 variant of the PIC cycle (the paper benchmarks the
cycle in single and in double precision, section "Evaluation") against the
FP64 oracle, through the C ABI.

With both sides in FP64 the differences are round-off: the order of sums in
the gather and the Esirkepov weights, the FP64 LDS and global atomics, and
the arrangement of the Boris arithmetic.  Bars: momenta, positions, J, E and
B within 1e-12 (relative as in the FP32 tests) after one step from a shared
state; the 100-step energy trace within 1e-9; Gauss's law to 1e-12 of
max|rho|.
"""
import numpy as np
import pytest

import oracle
import workloads
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


def _fp64(cfg):
    cfg["grid"]["precision"] = "fp64"
    return cfg


@pytest.mark.parametrize("idx,box", [(0, (16, 16, 16)), (2, (16, 16, 8)), (1, (16, 16, 8))])
def test_fp64_init_matches_oracle(P, idx, box):
    cfg = _fp64(workloads.reduced(idx, *box))
    _print("fp64 init parity", idx, box)
    with P.Pic(cfg) as pic:
        st = oracle.init_state(cfg)
        for i, sref in enumerate(st.species):
            g = pic.get_particles(i)
            assert g["ux"].dtype == np.float64
            assert np.array_equal(g["id"], sref.id)
            for a in ("x", "y", "z"):
                assert np.max(np.abs(g[a] - getattr(sref, a))) < 1e-13
            for a in ("ux", "uy", "uz"):
                ref = getattr(sref, a)
                assert np.max(np.abs(g[a] - ref)) <= 1e-15 * max(np.abs(ref).max(), 1e-300)
            assert np.all(g["w"] == sref.w[0])
        m = pic.moments()
        assert m["count"] == [s.n for s in st.species]
        assert m["gauss_max"] <= 1e-13 * max(m["rho_max"], 1.0)
        # the oracle forms gamma - 1 as sqrt(1 + u^2) - 1 (the definition), which
        # loses up to 2 eps gamma per particle to cancellation; the GPU uses the
        # well-conditioned u^2 / (1 + gamma)
        k_ref = oracle.kinetic(st)
        bound = sum(float(np.sum(s.w * s.m * 2.0**-51 * np.sqrt(1 + s.ux**2 + s.uy**2 + s.uz**2)))
                    for s in st.species) + 1e-14 * k_ref
        assert abs(m["kinetic_total"] - k_ref) <= bound


@pytest.mark.parametrize("idx,box,warm", [
    (0, (16, 16, 16), 10),       # CIC electrons, immobile background
    (1, (16, 16, 8), 10),        # CIC shear layer with drift 0.2c (many movers)
    (2, (16, 16, 8), 10),        # TSC electrons + protons in B0
    (2, (24, 8, 12), 6),         # TSC, ragged supercell counts per axis
])
def test_fp64_one_step_parity(P, idx, box, warm):
    cfg = _fp64(workloads.reduced(idx, *box))
    _print("fp64 one-step parity", idx, box)
    st = oracle.init_state(cfg)
    oracle.step(st, warm)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-12
    assert max(err["x"]) <= 1e-12
    assert err["J"] <= 1e-12
    assert err["E"] <= 1e-12 and err["B"] <= 1e-12


def test_fp64_one_step_parity_pcs(P):
    cfg = _fp64(workloads.config(2, nx=16, ny=16, nz=8, shape="pcs"))
    st = oracle.init_state(cfg)
    oracle.step(st, 6)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print("fp64 PCS", err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-12 and max(err["x"]) <= 1e-12 and err["J"] <= 1e-12


@pytest.mark.parametrize("shape", ["cic", "pcs"])
def test_fp64_one_step_parity_galerkin(P, shape):
    cfg = _fp64(workloads.config(2, nx=16, ny=16, nz=8, shape=shape, gather="galerkin"))
    st = oracle.init_state(cfg)
    oracle.step(st, 6)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print("fp64 Galerkin", shape, err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-12 and max(err["x"]) <= 1e-12 and err["J"] <= 1e-12


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_fp64_one_step_parity_particles_on_faces(P, shape):
    """Particles on cell and supercell faces, at cell centres and one FP64
    step either side of a face (degenerate shape weights and exits)."""
    cfg = _fp64(workloads.config(2, nx=16, ny=16, nz=8, shape=shape))
    st = oracle.init_state(cfg)
    oracle.step(st, 6)
    r = workloads.rng(62)
    for sp in st.species:
        for c, n in (("x", 16), ("y", 16), ("z", 8)):
            k = np.arange(n, dtype=np.float64)
            cand = np.concatenate([k, k + 0.5, np.nextafter(k + 1, 0.0), np.nextafter(k, float(n))])
            v = getattr(sp, c).copy()
            pick = r.random(v.size) < 0.5
            v[pick] = cand[r.integers(0, cand.size, int(pick.sum()))]
            setattr(sp, c, v)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print("fp64 faces", shape, err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-12 and max(err["x"]) <= 1e-12 and err["J"] <= 1e-12


def test_fp64_energy_trace_100_steps(P):
    cfg = _fp64(workloads.config(0))
    nsteps = cfg["steps"]
    st = oracle.init_state(cfg)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        ref = s0.copy()
        tr = oracle.step(ref, nsteps, trace=True)
        t_ref = oracle.energy_trace_total(tr)
        ms = []
        for _ in range(nsteps + 1):
            ms.append(pic.moments())
            if len(ms) <= nsteps:
                pic.step(1)
    we = np.array([m["w_e"] for m in ms])
    wb = np.array([m["w_b"] for m in ms])
    k = np.array([m["kinetic_total"] for m in ms])
    t_gpu = we[:-1] + wb[:-1] + 0.5 * (k[:-1] + k[1:])
    rel = np.abs(t_gpu - t_ref) / t_ref
    rel_we = np.abs(we[1:-1] - tr[1:, 0]) / tr[1:, 0]
    _print("fp64 trace max rel", rel.max(), "W_E max rel", rel_we.max(), "gauss", ms[-1]["gauss_max"],
           "rho_max", ms[-1]["rho_max"])
    assert rel.max() <= 1e-9
    assert rel_we.max() <= 1e-6
    assert ms[-1]["gauss_max"] <= 1e-12 * ms[-1]["rho_max"]


def test_fp64_full_size_shear128_sampled_parity(P):
    """128^3, 16 ppc (33.6M electrons) in FP64: sampled momenta against the
    oracle's push from the GPU's own pre-step state; Gauss over the run."""
    cfg = _fp64(workloads.config(1))
    _print("fp64 full-size 128^3 sampled parity")
    with P.Pic(cfg) as pic:
        pic.step(4)
        pre = pic.get_particles(0)
        E, B, _ = pic.get_fields()
        rng = workloads.rng(79)
        idx = rng.choice(pre["id"].size, 2000, replace=False)
        pre = {k: pre[k][idx] for k in ("x", "y", "z", "ux", "uy", "uz", "id")}
        pic.step(1)
        post = pic.get_particles(0)
        post = {k: post[k][idx] for k in ("ux", "uy", "uz", "id")}
        m = pic.moments()
    g = oracle.grid_from_config(cfg)
    Ep, Bp = oracle.gather(g, E, B, pre["x"], pre["y"], pre["z"])
    ux, uy, uz = oracle.boris(-1.0, g.dt, Ep, Bp, pre["ux"], pre["uy"], pre["uz"])
    assert np.array_equal(post["id"], pre["id"])
    du = np.sqrt((post["ux"] - ux) ** 2 + (post["uy"] - uy) ** 2 + (post["uz"] - uz) ** 2)
    nu = np.maximum(np.sqrt(ux**2 + uy**2 + uz**2), 0.01)
    _print("fp64 sampled momentum error", float((du / nu).max()), "gauss", m["gauss_max"], m["rho_max"])
    assert float((du / nu).max()) <= 1e-12
    assert m["count"][0] == 128**3 * 16
    assert m["gauss_max"] <= 1e-12 * m["rho_max"]
