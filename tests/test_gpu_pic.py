"""GPU parity of the PIC hot path against the FP64 oracle, through the C ABI.

Bars: momenta max|u_gpu - u_ref| / max(|u_ref|, u_th) <= 1e-5 after one step
from a shared FP32 state with non-zero fields; J within 1e-4 of max|J|;
total-energy trace within 1e-3 over 100 steps from one shared start.
"""
import math

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


# ---------------------------------------------------------------------------
# initial state

@pytest.mark.parametrize("idx,box", [(0, (16, 16, 16)), (2, (16, 16, 8)), (1, (16, 16, 8))])
def test_init_matches_oracle(P, idx, box):
    cfg = workloads.reduced(idx, *box)
    _print("init parity", idx, box)
    with P.Pic(cfg) as pic:
        st = oracle.init_state(cfg)
        for i, sref in enumerate(st.species):
            g = pic.get_particles(i)
            assert np.array_equal(g["id"], sref.id)
            for a in ("x", "y", "z"):
                assert np.max(np.abs(g[a] - getattr(sref, a))) < 1e-6
            for a in ("ux", "uy", "uz"):
                ref = getattr(sref, a)
                assert np.max(np.abs(g[a] - ref) / (np.abs(ref) + 1e-30)) < 1e-6
            assert np.all(g["w"] == np.float32(sref.w[0]))
        m = pic.moments()
        assert m["count"] == [s.n for s in st.species]
        assert m["w_e"] == 0.0 and m["w_b"] == 0.0
        assert m["gauss_max"] <= 1e-13 * max(m["rho_max"], 1.0)  # FP64 atomic order only
        assert abs(m["kinetic_total"] / oracle.kinetic(st) - 1) < 1e-5


# ---------------------------------------------------------------------------
# one-step parity from a shared state with non-zero fields

def _s0(cfg, warm):
    st = oracle.init_state(cfg)
    oracle.step(st, warm)
    return st


@pytest.mark.parametrize("idx,box,warm", [
    (0, (16, 16, 16), 10),       # CIC electrons, immobile background
    (1, (16, 16, 8), 10),        # CIC shear layer with drift 0.2c (many movers)
    (2, (16, 16, 8), 10),        # TSC electrons + protons in B0
    (2, (24, 8, 12), 6),         # TSC, ragged supercell counts per axis
])
def test_one_step_parity(P, idx, box, warm):
    cfg = workloads.reduced(idx, *box)
    _print("one-step parity", idx, box)
    st = _s0(cfg, warm)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-5
    assert err["J"] <= 1e-4
    assert max(err["x"]) <= 2e-6
    assert err["E"] <= 1e-4 and err["B"] <= 1e-4


@pytest.mark.parametrize("idx,box,warm", [
    (0, (16, 16, 16), 10),       # PCS electrons, immobile background
    (2, (16, 16, 8), 10),        # PCS electrons + protons in B0
])
def test_one_step_parity_pcs(P, idx, box, warm):
    """The cubic B-spline (PCS) shape: 4-node gather, 5-node Esirkepov window,
    a 2-node low guard in the staged field tile."""
    cfg = workloads.config(idx, nx=box[0], ny=box[1], nz=box[2], shape="pcs")
    _print("one-step parity PCS", idx, box)
    st = _s0(cfg, warm)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-5
    assert err["J"] <= 1e-4
    assert max(err["x"]) <= 2e-6
    assert err["E"] <= 1e-4 and err["B"] <= 1e-4


def _face_positions(x, n, r):
    """Move about half of the coordinates onto cell faces, cell centres and the
    FP32 neighbours of faces (supercell faces included), all in [0, n)."""
    k = np.arange(n, dtype=np.float32)
    cand = np.concatenate([k, k + np.float32(0.5),
                           np.nextafter(k + np.float32(1), np.float32(0)),   # largest float below each face
                           np.nextafter(k, np.float32(n))]).astype(np.float64)
    pick = r.random(x.size) < 0.5
    out = x.copy()
    out[pick] = cand[r.integers(0, cand.size, int(pick.sum()))]
    return out


@pytest.mark.parametrize("shape", ["cic", "tsc", "pcs"])
def test_one_step_parity_particles_on_faces(P, shape):
    """Degenerate positions: particles exactly on cell and supercell faces, at
    cell centres (the staggered weights' ties) and one FP32 step either side
    of a face, with non-zero fields; the same bars as the other one-step
    tests."""
    cfg = workloads.config(2, nx=16, ny=16, nz=8, shape=shape)
    st = _s0(cfg, 6)
    r = workloads.rng(61)
    for sp in st.species:
        sp.x = _face_positions(sp.x, 16, r)
        sp.y = _face_positions(sp.y, 16, r)
        sp.z = _face_positions(sp.z, 8, r)
    _print("one-step parity, particles on faces", shape)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-5
    assert err["J"] <= 1e-4
    assert max(err["x"]) <= 2e-6
    assert err["E"] <= 1e-4 and err["B"] <= 1e-4


@pytest.mark.parametrize("shape", ["cic", "tsc", "pcs"])
def test_one_step_parity_galerkin(P, shape):
    """The Galerkin gather: each component's shape one order lower along the
    axes on which it is staggered (nearest node for CIC), same deposit."""
    cfg = workloads.config(2, nx=16, ny=16, nz=8, shape=shape, gather="galerkin")
    _print("one-step parity Galerkin", shape)
    st = _s0(cfg, 10)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert err["jmax"] > 0
    assert max(err["u"]) <= 1e-5
    assert err["J"] <= 1e-4
    assert max(err["x"]) <= 2e-6
    assert err["E"] <= 1e-4 and err["B"] <= 1e-4


def test_galerkin_gather_differs_from_standard(P):
    """The switch reaches the kernel: one step from the same state with the two
    gathers gives different momenta (by far more than round-off)."""
    cfg = workloads.config(2, nx=16, ny=16, nz=8)
    st = _s0(cfg, 10)
    out = {}
    for gather in ("standard", "galerkin"):
        cfg["grid"]["gather"] = gather
        with P.Pic(cfg) as pic:
            parity.shared_start(pic, st)
            pic.step(1)
            p = pic.get_particles(0)
            out[gather] = p["ux"][np.argsort(p["id"])]
    du = np.max(np.abs(out["standard"] - out["galerkin"]))
    _print("standard vs Galerkin max |dux|", du)
    assert du > 1e-4 * np.max(np.abs(out["standard"]))


def test_energy_trace_100_steps_galerkin_tsc(P):
    cfg = workloads.config(0, shape="tsc", gather="galerkin")
    nsteps = 100
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
    _print("Galerkin TSC trace max rel", rel.max())
    assert rel.max() <= 1e-3
    assert ms[-1]["gauss_max"] <= 1e-4 * ms[-1]["rho_max"]


def test_energy_trace_100_steps_pcs(P):
    cfg = workloads.config(0, shape="pcs")
    nsteps = 100
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
    _print("PCS trace max rel", rel.max(), "gauss", ms[-1]["gauss_max"], "rho_max", ms[-1]["rho_max"])
    assert rel.max() <= 1e-3
    assert ms[-1]["gauss_max"] <= 1e-4 * ms[-1]["rho_max"]


def test_one_step_parity_single_supercell_wraps_onto_itself(P):
    """An 8x8x4 box is one supercell: every guard and every mover wraps to itself."""
    cfg = workloads.reduced(2, 8, 8, 4)
    st = _s0(cfg, 6)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
    _print(err)
    assert max(err["u"]) <= 1e-5 and err["J"] <= 1e-4


# ---------------------------------------------------------------------------
# energy trace and invariants over 100 steps

def test_energy_trace_100_steps(P):
    cfg = workloads.config(0)
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
    _print("trace max rel", rel.max(), "W_E ref/gpu", tr[-1, 0], we[-2], "gauss", ms[-1]["gauss_max"],
           "rho_max", ms[-1]["rho_max"])
    assert rel.max() <= 1e-3
    # Gauss's law holds to FP32 round-off over the run; div B stays zero
    assert ms[-1]["gauss_max"] <= 1e-4 * ms[-1]["rho_max"]
    assert ms[-1]["divb_max"] <= 1e-5
    assert abs(ms[-1]["charge_total"]) < 1e-6 * ms[-1]["rho_max"] * 16**3


def test_khi_magnetic_growth_tracks_oracle(P):
    """The paper's Kelvin-Helmholtz workload (electrons + protons at 16 ppc
    each, TSC, +-0.2c shear) on a 16x16x8 box: the magnetic energy grows by
    orders of magnitude from particle noise, and the GPU's W_B trace follows
    the oracle's step by step; total energy and Gauss's law hold."""
    cfg = workloads.reduced(5, 16, 16, 8)
    nsteps = 100
    st = oracle.init_state(cfg)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        ref = s0.copy()
        tr = oracle.step(ref, nsteps, trace=True)
        ms = []
        for _ in range(nsteps + 1):
            ms.append(pic.moments())
            if len(ms) <= nsteps:
                pic.step(1)
    wb = np.array([m["w_b"] for m in ms])[:nsteps]
    wb_ref = tr[:, 1]
    we = np.array([m["w_e"] for m in ms])
    k = np.array([m["kinetic_total"] for m in ms])
    t_gpu = we[:-1] + wb + 0.5 * (k[:-1] + k[1:])
    t_ref = oracle.energy_trace_total(tr)
    rel_b = np.abs(wb[1:] - wb_ref[1:]) / wb_ref[1:]
    _print("W_B ref", wb_ref[[1, 10, 50, 99]], "gpu", wb[[1, 10, 50, 99]], "max rel", rel_b.max(),
           "total max rel", (np.abs(t_gpu - t_ref) / t_ref).max())
    assert wb_ref[99] > 100 * wb_ref[10] and wb[99] > 100 * wb[10]
    assert rel_b.max() <= 1e-2
    assert (np.abs(t_gpu - t_ref) / t_ref).max() <= 1e-3
    assert ms[-1]["gauss_max"] <= 1e-4 * ms[-1]["rho_max"]


def test_migration_keeps_every_particle(P):
    cfg = workloads.reduced(1, 16, 16, 8)
    with P.Pic(cfg) as pic:
        ids0 = pic.get_particles(0)["id"]
        pic.step(20)
        p = pic.get_particles(0)
        m = pic.moments()
    assert np.array_equal(p["id"], ids0)
    assert m["count"][0] == ids0.size
    for a, n in zip(("x", "y", "z"), (16, 16, 8)):
        assert np.all(p[a] >= 0) and np.all(p[a] < n)
    assert m["gauss_max"] <= 1e-4 * m["rho_max"]


def test_one_step_parity_ragged_and_empty_supercells(P):
    """Electrons at random positions in part of the box only: one column of
    supercells stays empty, the others hold random (ragged) counts with
    partly filled last frames; the proton species has no particles at all.
    Random non-zero E and B."""
    cfg = workloads.reduced(2, 24, 16, 8)
    g = oracle.grid_from_config(cfg)
    r = workloads.rng(41)
    n = 5000
    x = r.uniform(0.0, 13.0, n)  # supercell columns 0 and 1 (partly); column 2 empty
    e = oracle.Species(x, r.uniform(0, 16, n), r.uniform(0, 8, n), r.normal(0, 0.05, n), r.normal(0, 0.05, n),
                       r.normal(0, 0.05, n), np.full(n, 0.125), np.arange(n, dtype=np.int64), q=-1.0, m=1.0)
    z0 = np.zeros(0)
    prot = oracle.Species(z0, z0, z0, z0, z0, z0, z0, np.zeros(0, dtype=np.int64), q=1.0,
                          m=workloads.PROTON_MASS)
    E, B = workloads.random_fields(42, 24, 16, 8, amp=0.05)
    st = oracle.State(g, [e, prot], E, B, np.zeros_like(E), 0)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        counts = pic.moments()["count"]
        err = parity.one_step_errors(pic, cfg, s0)
        after = pic.moments()["count"]
    _print("ragged/empty", counts, after, err)
    assert counts[0] == n and counts[1] == 0 and after[0] == n and after[1] == 0
    assert err["jmax"] > 0
    assert err["u"][0] <= 1e-5 and err["J"] <= 1e-4 and err["x"][0] <= 2e-6


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_one_step_parity_leavers_in_every_direction(P, shape):
    """Every particle of the centre supercell of a 3x3x3 grid of supercells
    leaves it in one step: the directions cycle through all 26 neighbours
    from one slot to the next (so each wave hands over to many destinations),
    then a block of 300 leaves through the same face (one destination for
    whole waves).  Positions after the step are global, so they check that
    every leaver reached the right neighbour in the right place."""
    cfg = workloads.config(1, nx=24, ny=24, nz=12, shape=shape)
    g = oracle.grid_from_config(cfg)
    r = workloads.rng(43)
    dirs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    d = np.array([dirs[i % 26] for i in range(26 * 20)] + [(1, 0, 0)] * 300)
    n = len(d)
    lo, ext = np.array([8.0, 8.0, 4.0]), np.array([8.0, 8.0, 4.0])
    pos = np.empty((n, 3))
    for a in range(3):
        inside = lo[a] + r.uniform(0.5, ext[a] - 0.5, n)
        pos[:, a] = np.where(d[:, a] < 0, lo[a] + 0.1, np.where(d[:, a] > 0, lo[a] + ext[a] - 0.1, inside))
    u = 0.8 * d + r.normal(0, 0.01, (n, 3))
    e = oracle.Species(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), u[:, 0].copy(), u[:, 1].copy(),
                       u[:, 2].copy(), np.full(n, 1.0 / 16), np.arange(n, dtype=np.int64), q=-1.0, m=1.0)
    E, B = workloads.random_fields(44, 24, 24, 12, amp=0.05)
    st = oracle.State(g, [e], E, B, np.zeros_like(E), 0)
    _print("leavers in every direction", shape, n)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
        err = parity.one_step_errors(pic, cfg, s0)
        got = pic.get_particles(0)
    _print(err)
    assert np.array_equal(np.sort(got["id"]), np.arange(n))
    # every particle left the centre supercell
    c = np.stack([got["x"], got["y"], got["z"]], axis=1)
    inside = np.all((c >= lo) & (c < lo + ext), axis=1)
    assert not inside.any()
    assert err["u"][0] <= 1e-5 and err["x"][0] <= 2e-6 and err["J"] <= 1e-4


# ---------------------------------------------------------------------------
# full-size workload in the benchmark's configuration: sampled parity

def test_full_size_shear128_sampled_parity(P):
    """128^3, 16 ppc (33.6M electrons): the oracle recomputes the push of a
    sample of particles one by one from the GPU's own pre-step state; charge
    conservation (Gauss) and particle count hold over the run."""
    cfg = workloads.config(1)
    _print("full-size 128^3 sampled parity")
    with P.Pic(cfg) as pic:
        pic.step(4)
        pre = pic.get_particles(0)
        E, B, _ = pic.get_fields()
        rng = workloads.rng(77)
        idx = rng.choice(pre["id"].size, 2000, replace=False)
        pic.step(1)
        post = pic.get_particles(0)
        m = pic.moments()
    g = oracle.grid_from_config(cfg)
    Ep, Bp = oracle.gather(g, E.astype(np.float64), B.astype(np.float64), pre["x"][idx], pre["y"][idx], pre["z"][idx])
    ux, uy, uz = oracle.boris(-1.0, g.dt, Ep, Bp, pre["ux"][idx].astype(np.float64),
                              pre["uy"][idx].astype(np.float64), pre["uz"][idx].astype(np.float64))
    assert np.array_equal(post["id"], pre["id"])
    du = np.sqrt((post["ux"][idx] - ux) ** 2 + (post["uy"][idx] - uy) ** 2 + (post["uz"][idx] - uz) ** 2)
    nu = np.maximum(np.sqrt(ux**2 + uy**2 + uz**2), 0.01)
    _print("sampled momentum error", float((du / nu).max()), "gauss", m["gauss_max"], m["rho_max"])
    assert float((du / nu).max()) <= 1e-5
    assert m["count"][0] == 128**3 * 16
    assert m["gauss_max"] <= 1e-4 * m["rho_max"]


@pytest.mark.parametrize("idx,gather", [
    (2, "standard"),   # 256x256x128 TSC, electrons + protons at 8 ppc each in B0 (134M particles)
    (5, "standard"),   # 128^3 TSC Kelvin-Helmholtz shear flow, electrons + protons at 16 ppc each (67M)
    (1, "galerkin"),   # 128^3 CIC shear layer (33.6M electrons) with the Galerkin gather
])
def test_full_size_sampled_parity(P, idx, gather):
    """Full-size workloads in the benchmark's launch configuration: sampled
    momenta and positions of every species against the oracle's gather, Boris
    and move from the GPU's own pre-step state; Gauss and particle counts over
    the run."""
    cfg = workloads.config(idx, gather=gather)
    gc = cfg["grid"]
    nx, ny, nz = gc["nx"], gc["ny"], gc["nz"]
    nsp = len(cfg["species"])
    _print("full-size sampled parity", cfg["workload"], gather)
    g = oracle.grid_from_config(cfg)
    with P.Pic(cfg) as pic:
        pic.step(3)
        E, B, _ = pic.get_fields()
        pre = [pic.get_particles(i) for i in range(nsp)]
        rng = workloads.rng(78)
        sel = [rng.choice(p["id"].size, 1500, replace=False) for p in pre]
        pre = [{k: p[k][i] for k in ("x", "y", "z", "ux", "uy", "uz", "id")} for p, i in zip(pre, sel)]
        pic.step(1)
        post = [pic.get_particles(i) for i in range(nsp)]
        post = [{k: p[k][i] for k in ("x", "y", "z", "ux", "uy", "uz", "id")} for p, i in zip(post, sel)]
        m = pic.moments()
    E, B = E.astype(np.float64), B.astype(np.float64)
    for sp, a, b in zip(cfg["species"], pre, post):
        assert np.array_equal(a["id"], b["id"])
        Ep, Bp = oracle.gather(g, E, B, a["x"], a["y"], a["z"])
        ux, uy, uz = oracle.boris(sp["charge"] / sp["mass"], g.dt, Ep, Bp, a["ux"], a["uy"], a["uz"])
        du = np.sqrt((b["ux"] - ux) ** 2 + (b["uy"] - uy) ** 2 + (b["uz"] - uz) ** 2)
        eu = float((du / np.maximum(np.sqrt(ux**2 + uy**2 + uz**2), sp["u_th"])).max())
        ig = 1.0 / np.sqrt(1.0 + ux**2 + uy**2 + uz**2)
        ex = 0.0
        for c, uc, n in (("x", ux, nx), ("y", uy, ny), ("z", uz, nz)):
            want = np.mod(a[c] + g.dt * uc * ig, n)
            d = np.abs(b[c] - want)
            ex = max(ex, float(np.minimum(d, n - d).max()))
        _print(sp["name"], "sampled momentum error", eu, "position error", ex)
        assert eu <= 1e-5 and ex <= 4e-6
    _print("gauss", m["gauss_max"], m["rho_max"], "counts", m["count"])
    assert list(m["count"])[:nsp] == [nx * ny * nz * sp["ppc"] for sp in cfg["species"]]
    assert m["gauss_max"] <= 1e-4 * m["rho_max"]


# ---------------------------------------------------------------------------
# error paths forced from the host (every kernel still exits normally)

def test_capacity_error_on_set(P):
    cfg = workloads.reduced(0, 16, 16, 16)
    with P.Pic(cfg) as pic:
        n = 8 * 256 * 2  # twice the frames one supercell holds (cap 12 ppc)
        r = workloads.rng(1)
        p = dict(x=r.uniform(0, 8, n), y=r.uniform(0, 8, n), z=r.uniform(0, 4, n), ux=np.zeros(n), uy=np.zeros(n),
                 uz=np.zeros(n), w=np.full(n, 0.125), id=np.arange(n))
        with pytest.raises(P.PicError) as e:
            pic.set_particles(0, p)
        assert e.value.code == -4


def test_migration_overflow_reports_capacity(P):
    """Every particle of one supercell leaves through the same face in one
    step: more arrivals than the destination's migration buffer holds."""
    cfg = workloads.reduced(0, 16, 16, 16)
    with P.Pic(cfg) as pic:
        n = 2048
        r = workloads.rng(2)
        p = dict(x=r.uniform(7.9, 7.99, n), y=r.uniform(0, 8, n), z=r.uniform(0, 4, n), ux=np.full(n, 3.0),
                 uy=np.zeros(n), uz=np.zeros(n), w=np.full(n, 0.125), id=np.arange(n))
        pic.set_particles(0, p)
        with pytest.raises(P.PicError) as e:
            pic.step(1)
        assert e.value.code == -4


def test_nonfinite_field_is_reported(P):
    """Opposite extreme E_y in neighbouring cells overflow the curl: B becomes
    infinite in the first half step, the push sees it (PIC_ERR_CFL guards every
    non-finite displacement) and the diagnostics report PIC_ERR_NONFINITE."""
    cfg = workloads.reduced(0, 16, 16, 16)
    with P.Pic(cfg) as pic:
        E = np.zeros((3, 16, 16, 16), dtype=np.float32)
        E[1, 3, 3, 3] = 3e38
        E[1, 3, 3, 4] = -3e38
        pic.set_fields(E=E)
        with pytest.raises(P.PicError) as e:
            pic.step(2)  # B overflows in the first Yee update; the second push sees it
        assert e.value.code == -5
        with pytest.raises(P.PicError) as e2:
            pic.moments()
        assert e2.value.code == -6
