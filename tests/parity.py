"""Parity harness: move one state between the FP64 oracle and the GPU library
and measure the differences after the same steps.

Protocol (both sides start from one FP32-representable state): the oracle
produces a state, it is written to the GPU (rounded to FP32 there), read back,
and that exact FP32 state, widened to FP64, becomes the oracle's start.
"""
from __future__ import annotations

import numpy as np

import oracle


def _species_dict(s: oracle.Species) -> dict:
    d = dict(x=s.x, y=s.y, z=s.z, ux=s.ux, uy=s.uy, uz=s.uz, w=s.w, id=s.id)
    d["zstate"] = s.zstate
    return d


def push_state(pic, st: oracle.State):
    """Write an oracle state into the GPU handle (particles, E, B; J zero)."""
    for i, s in enumerate(st.species):
        pic.set_particles(i, _species_dict(s))
    pic.set_fields(E=st.E, B=st.B, J=np.zeros_like(st.E))
    pic.mark_reference()


def pull_state(pic, like: oracle.State) -> oracle.State:
    """The GPU state as an FP64 oracle State (particles sorted by id)."""
    E, B, J = pic.get_fields()
    species = []
    for i, ref in enumerate(like.species):
        p = pic.get_particles(i)
        zs = p["zstate"].astype(np.int32) if ref.zstate is not None else None
        species.append(oracle.Species(
            *(np.ascontiguousarray(p[k], dtype=np.float64) for k in ("x", "y", "z", "ux", "uy", "uz", "w")),
            id=np.ascontiguousarray(p["id"], dtype=np.int64), q=ref.q, m=ref.m, mobile=ref.mobile,
            zstate=None if zs is None else np.ascontiguousarray(zs)))
    return oracle.State(like.grid, species, E.astype(np.float64), B.astype(np.float64), J.astype(np.float64),
                        like.step)


def shared_start(pic, st: oracle.State) -> oracle.State:
    """Give both sides the same FP32-representable state; returns the oracle's copy."""
    for s in st.species:
        s.sort_by_id()
    push_state(pic, st)
    return pull_state(pic, st)


def momentum_error(gpu: oracle.Species, ref: oracle.Species, u_th: float) -> float:
    """max_p |u_gpu - u_ref| / max(|u_ref|, u_th)."""
    assert np.array_equal(gpu.id, ref.id)
    du = np.sqrt((gpu.ux - ref.ux) ** 2 + (gpu.uy - ref.uy) ** 2 + (gpu.uz - ref.uz) ** 2)
    nu = np.sqrt(ref.ux**2 + ref.uy**2 + ref.uz**2)
    return float(np.max(du / np.maximum(nu, u_th))) if du.size else 0.0


def position_error(gpu: oracle.Species, ref: oracle.Species, dims) -> float:
    """max periodic distance between positions, in cells."""
    err = 0.0
    for a, n in zip(("x", "y", "z"), dims):
        d = np.abs(getattr(gpu, a) - getattr(ref, a))
        d = np.minimum(d, n - d)
        err = max(err, float(d.max()) if d.size else 0.0)
    return err


def one_step_errors(pic, cfg: dict, st0: oracle.State) -> dict:
    """Both sides take one step from st0 (already shared); errors per quantity."""
    ref = st0.copy()
    oracle.step(ref, 1)
    pic.step(1)
    got = pull_state(pic, st0)
    dims = (cfg["grid"]["nx"], cfg["grid"]["ny"], cfg["grid"]["nz"])
    out = dict(u=[], x=[])
    for i, sp in enumerate(cfg["species"]):
        if not sp["mobile"]:
            continue
        out["u"].append(momentum_error(got.species[i], ref.species[i], sp["u_th"]))
        out["x"].append(position_error(got.species[i], ref.species[i], dims))
    jmax = float(np.abs(ref.J).max())
    out["J"] = float(np.abs(got.J - ref.J).max()) / jmax if jmax > 0 else 0.0
    out["E"] = float(np.abs(got.E - ref.E).max()) / max(float(np.abs(ref.E).max()), 1e-30)
    out["B"] = float(np.abs(got.B - ref.B).max()) / max(float(np.abs(ref.B).max()), 1e-30)
    out["jmax"] = jmax
    return out
