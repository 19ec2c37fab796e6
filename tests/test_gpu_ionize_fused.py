"""The fused ionisation step with the exact rate (pic_ionize: moments, rate
and draw per supercell in one launch) against the staged one
(pic_ionize_staged: three launches over the grid), through the C ABI on the
GPU.

From one shared state both must give the same step: the same counts, the
same charge state of every ion and the same new electrons (compared sorted
by id: the order of appended electrons within a supercell is defined by
neither), and the same cell moments.  With energy loss the heated-down
electron momenta agree to FP64 rounding (the per-cell energy sums are
atomic adds in either order).  The staged step itself is checked against
the oracle in the other ionisation tests; the fused one is also what their
exact-rate cases run by default.
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


def _cfg(box=(16, 16, 8), max_events=1, energy_loss=0, n_ref=1e21):
    cfg = workloads.reduced(3, *box)
    cfg["grid"]["n_ref_cm3"] = n_ref
    c = cfg["species"][1]
    c["max_events"] = max_events
    c["energy_loss"] = energy_loss
    return cfg


def _shared(P, cfg, warm=4):
    st = oracle.init_state(cfg)
    oracle.step(st, warm)
    with P.Pic(cfg) as pic:
        s0 = parity.shared_start(pic, st)
    s0.step = 0
    return s0


def _run(P, cfg, s0, mode, staged):
    with P.Pic(cfg) as pic:
        parity.push_state(pic, s0)
        stats = pic.ionize(mode, staged=staged)
        ne, kT = pic.cell_moments(1)
        ions, el = pic.get_particles(1), pic.get_particles(0)
    o = np.argsort(el["id"], kind="stable")
    oi = np.argsort(ions["id"], kind="stable")
    return stats, {k: v[oi] for k, v in ions.items()}, {k: v[o] for k, v in el.items()}, (ne, kT)


def _compare(a, b, eloss=False):
    sa, ia, ea, ma = a
    sb, ib, eb, mb = b
    _print("staged", sa, "fused", sb)
    for k in ("ions_active", "ionized", "fallback", "electrons"):
        assert sa[k] == sb[k], k
    assert np.array_equal(ia["zstate"], ib["zstate"])
    assert np.array_equal(ea["id"], eb["id"])
    for k in ("x", "y", "z", "w"):
        assert np.array_equal(ea[k], eb[k]), k
    for k in ("ux", "uy", "uz"):
        if eloss:
            assert np.allclose(ea[k], eb[k], rtol=1e-6, atol=1e-9), k
        else:
            assert np.array_equal(ea[k], eb[k]), k
    # recomputed after the step; FP64 LDS sums, so equal up to their order
    assert np.allclose(ma[0], mb[0], rtol=1e-13, atol=0) and np.allclose(ma[1], mb[1], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("variant", ["one_event", "chain", "energy_loss"])
def test_fused_exact_step_equals_staged(P, variant):
    # reference densities that put the rates high enough for hundreds of
    # events on 16x16x8 cells (1e24 with max_events 4: a share of the ions
    # take several)
    n_ref = 1e24 if variant == "chain" else 1e23
    cfg = _cfg(max_events=4 if variant == "chain" else 1, energy_loss=1 if variant == "energy_loss" else 0,
               n_ref=n_ref)
    _print("fused vs staged", variant, n_ref)
    s0 = _shared(P, cfg)
    a = _run(P, cfg, s0, "exact", True)
    b = _run(P, cfg, s0, "exact", False)
    assert b[0]["rate_ms"] == -1.0 and a[0]["rate_ms"] > 0.0
    assert a[0]["ionized"] > 100
    if variant == "chain":
        z0 = s0.species[1].zstate[np.argsort(s0.species[1].id, kind="stable")]
        assert int((a[1]["zstate"].astype(np.int64) - z0).max()) >= 2
    _compare(a, b, eloss=variant == "energy_loss")


def test_surrogate_and_table_steps_run_staged(P):
    """pic_ionize runs the surrogate and the table staged: their rate stage
    is timed."""
    cfg = _cfg()
    with P.Pic(cfg) as pic:
        pic.mlp_train(1, seed=workloads.MLP_TRAIN_SEED, n_train=65536, batch=4096, steps=50)
        pic.step(1)
        for mode in ("mlp", "table"):
            assert pic.ionize(mode)["rate_ms"] > 0.0
