"""FP64 CPU oracle for the particle-in-cell hot path (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never loads it and shares no code with
it.  The PIC cycle is plain C (`pic_oracle.c`, FP64, global arrays, periodic
wrap); the Monte Carlo ionisation rates and the MLP reference live in
`ionize.py` and `mlp.py` (numpy, FP64).

The paper names its methods only (section "Evaluation": Boris pusher,
Esirkepov current solver, Yee field solver, separable field interpolation,
TSC shape); each routine is the textbook definition of that method.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pic_oracle.c")
_lib = None


def build(src: str = _SRC, out: str = _SO) -> str:
    """Compile the C oracle (IEEE FP64: no fast-math, no FMA contraction).
    src / out name another copy of the source and its library (the tests
    compile copies with planted mistakes to show that the pins catch them)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp",
                           "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


def load_library(path: str):
    """A compiled copy of the oracle at `path`, declared like the default one."""
    L = C.CDLL(path)
    _declare(L)
    return L


def use_library(L):
    """Make L the library every wrapper below calls; returns the previous one."""
    global _lib
    prev, _lib = lib(), L
    return prev


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("order", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("b0", C.c_double * 3), ("rho_bg", C.c_double), ("gather", C.c_int32), ("pad", C.c_int32)]


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.POINTER(C.c_double)) for k in ("x", "y", "z", "ux", "uy", "uz", "w")] + [
        ("id", C.POINTER(C.c_int64)), ("zstate", C.POINTER(C.c_int32)),
        ("q", C.c_double), ("m", C.c_double), ("mobile", C.c_int32)]


class _InitSpec(C.Structure):
    _fields_ = [("index", C.c_int32), ("ppc", C.c_int32), ("id_offset", C.c_int64), ("u_th", C.c_double),
                ("drift_u", C.c_double * 3), ("layout", C.c_int32), ("pos_index", C.c_int32),
                ("pos_ppc", C.c_int32), ("pos_id_offset", C.c_int64), ("w", C.c_double)]


_D = C.POINTER(C.c_double)
_U64 = C.POINTER(C.c_uint64)


def _declare(L):
    L.orc_philox4x64_10.argtypes = [_U64, _U64, _U64]
    L.orc_u01.argtypes = [C.c_uint64]
    L.orc_u01.restype = C.c_double
    L.orc_shape.argtypes = [C.c_int, C.c_double]
    L.orc_shape.restype = C.c_double
    gp = C.POINTER(Grid)
    L.orc_gather.argtypes = [gp, _D, _D, C.c_int64, _D, _D, _D, _D, _D]
    L.orc_boris.argtypes = [C.c_int64, _D, C.c_double, _D, _D, _D, _D, _D]
    L.orc_esirkepov.argtypes = [gp, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]
    L.orc_deposit_rho.argtypes = [gp, C.c_int64, _D, _D, _D, _D, _D]
    L.orc_update_b.argtypes = [gp, C.c_double, _D, _D]
    L.orc_update_e.argtypes = [gp, C.c_double, _D, _D, _D]
    L.orc_div_nodes.argtypes = [gp, _D, _D]
    L.orc_div_cells.argtypes = [gp, _D, _D]
    L.orc_field_energy.argtypes = [gp, _D, _D, _D]
    L.orc_kinetic.argtypes = [C.POINTER(_Particles)]
    L.orc_kinetic.restype = C.c_double
    L.orc_rho.argtypes = [gp, C.c_int, C.POINTER(_Particles), _D]
    L.orc_step.argtypes = [gp, C.c_int, C.POINTER(_Particles), _D, _D, _D, C.c_int, _D]
    L.orc_step.restype = C.c_int
    L.orc_step_threads.argtypes = [gp, C.c_int, C.POINTER(_Particles), _D, _D, _D, C.c_int, C.c_int]
    L.orc_step_threads.restype = C.c_int
    L.orc_init_species.argtypes = [gp, C.c_uint64, C.POINTER(_InitSpec), _D, _D, _D, _D, _D, _D, _D,
                                   C.POINTER(C.c_int64)]


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


# ---------------------------------------------------------------------------
# Thin wrappers.

def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(c.ctypes.data_as(_U64), k.ctypes.data_as(_U64), o.ctypes.data_as(_U64))
    return o


def u01(word: int) -> float:
    return lib().orc_u01(C.c_uint64(int(word)))


def shape(order: int, d: float) -> float:
    return lib().orc_shape(order, float(d))


def make_grid(nx, ny, nz, order, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.0), rho_bg=0.0,
              galerkin=False) -> Grid:
    g = Grid()
    g.nx, g.ny, g.nz, g.order = nx, ny, nz, order
    g.dx, g.dy, g.dz, g.dt = dx, dy, dz, dt
    g.b0[:] = list(b0)
    g.rho_bg = rho_bg
    g.gather = 1 if galerkin else 0
    return g


def grid_from_config(cfg: dict) -> Grid:
    gc = cfg["grid"]
    order = {"cic": 1, "tsc": 2, "pcs": 3}[gc["shape"]]
    return make_grid(gc["nx"], gc["ny"], gc["nz"], order, gc["dx"], gc["dy"], gc["dz"], gc["dt"],
                     gc["b0"], gc["rho_bg"], galerkin=gc.get("gather", "standard") == "galerkin")


def zero_fields(g: Grid) -> np.ndarray:
    return np.zeros((3, g.nz, g.ny, g.nx))


def gather(g: Grid, E, B, x, y, z):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    x, y, z = (np.ascontiguousarray(np.atleast_1d(a), dtype=np.float64) for a in (x, y, z))
    n = x.size
    Ep = np.zeros((n, 3))
    Bp = np.zeros((n, 3))
    lib().orc_gather(C.byref(g), _dp(E), _dp(B), n, _dp(x), _dp(y), _dp(z), _dp(Ep), _dp(Bp))
    return Ep, Bp


def boris(qm, dt, Ep, Bp, ux, uy, uz):
    """In-place on copies; returns (ux, uy, uz)."""
    ux, uy, uz = (np.array(np.atleast_1d(a), dtype=np.float64) for a in (ux, uy, uz))
    n = ux.size
    qm = np.ascontiguousarray(np.broadcast_to(np.asarray(qm, dtype=np.float64), (n,)))
    Ep = np.ascontiguousarray(Ep, dtype=np.float64).reshape(n, 3)
    Bp = np.ascontiguousarray(Bp, dtype=np.float64).reshape(n, 3)
    lib().orc_boris(n, _dp(qm), dt, _dp(Ep), _dp(Bp), _dp(ux), _dp(uy), _dp(uz))
    return ux, uy, uz


def esirkepov(g: Grid, qw, x0, y0, z0, x1, y1, z1, J=None):
    arrs = [np.ascontiguousarray(np.atleast_1d(a), dtype=np.float64) for a in (x0, y0, z0, x1, y1, z1)]
    n = arrs[0].size
    qw = np.ascontiguousarray(np.broadcast_to(np.asarray(qw, dtype=np.float64), (n,)))
    if J is None:
        J = zero_fields(g)
    lib().orc_esirkepov(C.byref(g), n, _dp(qw), *[_dp(a) for a in arrs], _dp(J))
    return J


def deposit_rho(g: Grid, qw, x, y, z, rho=None):
    x, y, z = (np.ascontiguousarray(np.atleast_1d(a), dtype=np.float64) for a in (x, y, z))
    n = x.size
    qw = np.ascontiguousarray(np.broadcast_to(np.asarray(qw, dtype=np.float64), (n,)))
    if rho is None:
        rho = np.zeros((g.nz, g.ny, g.nx))
    lib().orc_deposit_rho(C.byref(g), n, _dp(qw), _dp(x), _dp(y), _dp(z), _dp(rho))
    return rho


def update_b(g: Grid, coef, E, B):
    lib().orc_update_b(C.byref(g), coef, _dp(E), _dp(B))


def update_e(g: Grid, coef, B, J, E):
    lib().orc_update_e(C.byref(g), coef, _dp(B), _dp(J) if J is not None else None, _dp(E))


def div_nodes(g: Grid, F):
    out = np.zeros((g.nz, g.ny, g.nx))
    lib().orc_div_nodes(C.byref(g), _dp(np.ascontiguousarray(F)), _dp(out))
    return out


def div_cells(g: Grid, F):
    out = np.zeros((g.nz, g.ny, g.nx))
    lib().orc_div_cells(C.byref(g), _dp(np.ascontiguousarray(F)), _dp(out))
    return out


def field_energy(g: Grid, E, B):
    out = np.zeros(2)
    lib().orc_field_energy(C.byref(g), _dp(E), _dp(B), _dp(out))
    return float(out[0]), float(out[1])


# ---------------------------------------------------------------------------
# Whole-simulation state.

@dataclass
class Species:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    w: np.ndarray
    id: np.ndarray
    q: float
    m: float
    mobile: bool = True
    zstate: np.ndarray | None = None

    @property
    def n(self):
        return self.x.size

    def copy(self):
        return Species(*(getattr(self, k).copy() for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id")),
                       q=self.q, m=self.m, mobile=self.mobile,
                       zstate=None if self.zstate is None else self.zstate.copy())

    def _struct(self):
        s = _Particles()
        s.n = self.n
        for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
            a = getattr(self, k)
            assert a.dtype == np.float64 and a.flags.c_contiguous
            setattr(s, k, a.ctypes.data_as(_D))
        assert self.id.dtype == np.int64
        s.id = self.id.ctypes.data_as(C.POINTER(C.c_int64))
        if self.zstate is not None:
            assert self.zstate.dtype == np.int32
            s.zstate = self.zstate.ctypes.data_as(C.POINTER(C.c_int32))
        s.q, s.m, s.mobile = self.q, self.m, int(self.mobile)
        return s

    def sort_by_id(self):
        o = np.argsort(self.id, kind="stable")
        for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id"):
            setattr(self, k, np.ascontiguousarray(getattr(self, k)[o]))
        if self.zstate is not None:
            self.zstate = np.ascontiguousarray(self.zstate[o])


@dataclass
class State:
    grid: Grid
    species: list
    E: np.ndarray
    B: np.ndarray
    J: np.ndarray
    step: int = 0
    extra: dict = field(default_factory=dict)

    def copy(self):
        return State(self.grid, [s.copy() for s in self.species], self.E.copy(), self.B.copy(),
                     self.J.copy(), self.step, dict(self.extra))


def _structs(species):
    arr = (_Particles * max(1, len(species)))()
    for i, s in enumerate(species):
        arr[i] = s._struct()
    return arr


def step(st: State, nsteps: int = 1, trace: bool = False):
    """Advance `st` in place by nsteps PIC cycles.  With trace, returns an
    (nsteps, 4) array of W_E^n, W_B^n, K^{n-1/2}, K^{n+1/2}."""
    tr = np.zeros((nsteps, 4)) if trace else None
    structs = _structs(st.species)
    rc = lib().orc_step(C.byref(st.grid), len(st.species), structs, _dp(st.E), _dp(st.B), _dp(st.J),
                        nsteps, _dp(tr) if trace else None)
    assert rc == 0
    st.step += nsteps
    return tr


def step_threads(st: State, nsteps: int, nthreads: int) -> int:
    """orc_step's cycle with the particle loop split over nthreads threads
    (private current arrays summed in thread order); for timing the host's
    cores.  Returns the number of threads that ran."""
    structs = _structs(st.species)
    used = lib().orc_step_threads(C.byref(st.grid), len(st.species), structs, _dp(st.E), _dp(st.B), _dp(st.J),
                                  nsteps, nthreads)
    assert used >= 1
    st.step += nsteps
    return used


def rho(st: State):
    out = np.zeros((st.grid.nz, st.grid.ny, st.grid.nx))
    structs = _structs(st.species)
    lib().orc_rho(C.byref(st.grid), len(st.species), structs, _dp(out))
    return out


def kinetic(st: State) -> float:
    return float(sum(lib().orc_kinetic(C.byref(s._struct())) for s in st.species))


def gauss_residual(st: State):
    """G = div E - rho at every node (backward differences)."""
    return div_nodes(st.grid, st.E) - rho(st)


def energy_trace_total(tr: np.ndarray) -> np.ndarray:
    """T_n = W_E^n + W_B^n + (K^{n-1/2} + K^{n+1/2}) / 2."""
    return tr[:, 0] + tr[:, 1] + 0.5 * (tr[:, 2] + tr[:, 3])


_LAYOUT = {"uniform": 0, "shear": 1, "beams": 2}


def init_state(cfg: dict) -> State:
    """The configuration's initial state (t = 0 fields zero; u stored at t = -1/2)."""
    g = grid_from_config(cfg)
    gc = cfg["grid"]
    ncell = g.nx * g.ny * g.nz
    dV = g.dx * g.dy * g.dz
    offsets = []
    off = 0
    for sp in cfg["species"]:
        offsets.append(off)
        off += ncell * sp["ppc"]
    species = []
    for si, sp in enumerate(cfg["species"]):
        n = ncell * sp["ppc"]
        arrs = [np.zeros(n) for _ in range(7)]
        ids = np.zeros(n, dtype=np.int64)
        spec = _InitSpec()
        spec.index = si
        spec.ppc = sp["ppc"]
        spec.id_offset = offsets[si]
        spec.u_th = sp["u_th"]
        beta = np.asarray(sp["drift_beta"], dtype=np.float64)
        gam = 1.0 / np.sqrt(1.0 - float(beta @ beta))
        spec.drift_u[:] = list(gam * beta)
        spec.layout = _LAYOUT[sp["layout"]]
        cw = sp["coincident_with"]
        if cw >= 0:
            spec.pos_index = cw
            spec.pos_ppc = cfg["species"][cw]["ppc"]
            spec.pos_id_offset = offsets[cw]
            assert sp["ppc"] <= spec.pos_ppc
        else:
            spec.pos_index, spec.pos_ppc, spec.pos_id_offset = si, sp["ppc"], offsets[si]
        spec.w = sp["density"] * dV / sp["ppc"]
        lib().orc_init_species(C.byref(g), C.c_uint64(gc["seed"]), C.byref(spec), *[_dp(a) for a in arrs],
                               ids.ctypes.data_as(C.POINTER(C.c_int64)))
        zst = None
        if sp["z_max"] > 0:
            zst = np.full(n, sp["z_init"], dtype=np.int32)
        species.append(Species(*arrs, id=ids, q=sp["charge"], m=sp["mass"], mobile=sp["mobile"], zstate=zst))
    z = zero_fields(g)
    return State(g, species, z.copy(), z.copy(), z.copy())
