"""Python handle over the C ABI: marshals workload dictionaries into the C
structs, supplies device memory from PyTorch's caching allocator and the
current HIP stream, and copies state in and out as numpy arrays.  Every
step of the simulation runs in the HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as A

_LAYOUT = {"uniform": 0, "shear": 1, "beams": 2}
_MODE = {"exact": 0, "mlp": 1, "table": 2}
_ACT = {"silu": 0, "relu": 1}  # hidden-layer activation of the rate surrogate
_ACT_NAME = {v: k for k, v in _ACT.items()}


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def gauss_laguerre64():
    """The library's own 64-point Gauss-Laguerre rule (host code, no GPU needed)."""
    lib = A.load()
    x = np.zeros(64)
    w = np.zeros(64)
    A.check(lib.pic_gauss_laguerre64(_dptr(x), _dptr(w)))
    return x, w


_SHAPE = {"cic": 1, "tsc": 2, "pcs": 3}
_PRECISION = {"fp32": 0, "fp64": 1}
LOTZ_A = 4.5e-14  # cm^2 eV^2, the plain Lotz constant


def grid_struct(cfg: dict) -> A.GridT:
    gc = cfg["grid"]
    g = A.GridT()
    g.nx, g.ny, g.nz = gc["nx"], gc["ny"], gc["nz"]
    g.dx, g.dy, g.dz, g.dt = gc["dx"], gc["dy"], gc["dz"], gc["dt"]
    g.b0[:] = list(gc["b0"])
    g.rho_bg = gc["rho_bg"]
    g.seed = gc["seed"]
    g.n_ref_cm3 = gc.get("n_ref_cm3", 1e21)
    g.precision = _PRECISION[gc.get("precision", "fp32")]
    g.gather = {"standard": 0, "galerkin": 1}[gc.get("gather", "standard")]
    g.options = ((A.PIC_OPT_DETERMINISTIC_J if gc.get("deterministic_j") else 0) |
                 (A.PIC_OPT_CONTINUITY if gc.get("continuity") else 0))
    return g


def species_structs(cfg: dict):
    sps = cfg["species"]
    arr = (A.SpeciesT * len(sps))()
    for i, sp in enumerate(sps):
        s = arr[i]
        s.charge, s.mass, s.density, s.u_th = sp["charge"], sp["mass"], sp["density"], sp["u_th"]
        s.drift_beta[:] = list(sp["drift_beta"])
        s.ppc = sp["ppc"]
        s.layout = _LAYOUT[sp["layout"]]
        s.mobile = int(sp["mobile"])
        s.coincident_with = sp["coincident_with"]
        s.z_init, s.z_max = sp["z_init"], sp["z_max"]
        s.cap_ppc = sp.get("cap_ppc") or 0
        s.ionize_into = sp.get("ionize_into", -1)
        s.max_events = sp.get("max_events", 1)
        s.energy_loss = int(sp.get("energy_loss", 0))
        for z, ev in enumerate(sp["ionization_ev"]):
            s.ionization_ev[z] = ev
            # "lotz_shells"[z]: dicts (p_ev, q, and a, b, c defaulting to the plain
            # form); otherwise one subshell (ionization_ev, 4.5e-14, 0, 0, lotz_q)
            shells = (sp["lotz_shells"][z] if sp.get("lotz_shells")
                      else [dict(p_ev=ev, q=sp["lotz_q"][z])])
            for j, sh in enumerate(shells):
                L = s.lotz[z][j]
                L.p_ev, L.q = sh["p_ev"], sh["q"]
                L.a, L.b, L.c = sh.get("a", LOTZ_A), sh.get("b", 0.0), sh.get("c", 0.0)
    return arr


class TorchAllocator:
    """Device memory for the library from torch.empty(uint8) blocks, kept
    alive until the library frees them."""

    def __init__(self, device):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self._alloc = A.ALLOC_FN(self._do_alloc)
        self._free = A.FREE_FN(self._do_free)
        self.struct = A.AllocT(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _do_free(self, ptr, user):
        self.live.pop(ptr, None)


class Pic:
    """One simulation on one GPU.  cfg is a workload dictionary (see
    workloads.py).  stream: a torch.cuda.Stream (default: the current one)."""

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None, torch_alloc: bool = True, allocator=None):
        import torch
        self.lib = A.load()
        self.cfg = cfg
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nsp = len(cfg["species"])
        self.shape = cfg["grid"]["nx"], cfg["grid"]["ny"], cfg["grid"]["nz"]
        self.fp64 = cfg["grid"].get("precision", "fp32") == "fp64"
        self._rt = np.float64 if self.fp64 else np.float32  # host type of momenta, weights and fields
        # allocator: an object with .struct (an AllocT), e.g. a TorchAllocator
        self._alloc = allocator if allocator is not None else (TorchAllocator(self.device) if torch_alloc else None)
        self._g = grid_struct(cfg)
        self._s = species_structs(cfg)
        h = C.c_void_p()
        rc = self.lib.pic_init(C.byref(h), C.byref(self._g), self._s, self.nsp, _SHAPE[cfg["grid"]["shape"]],
                               C.byref(self._alloc.struct) if self._alloc else None,
                               C.c_void_p(self.stream.cuda_stream))
        A.check(rc, None)
        self.h = h

    # ------------------------------------------------------------------ life
    def close(self):
        if getattr(self, "h", None):
            self.lib.pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ steps
    def step(self, n: int = 1):
        A.check(self.lib.pic_step(self.h, int(n)), self.h)

    def moments(self) -> dict:
        m = A.MomentsT()
        rc = self.lib.pic_moments(self.h, C.byref(m))
        d = dict(w_e=m.w_e, w_b=m.w_b, kinetic=list(m.kinetic)[: self.nsp], kinetic_total=m.kinetic_total,
                 charge_total=m.charge_total, rho_max=m.rho_max, gauss_max=m.gauss_max, divb_max=m.divb_max,
                 count=list(m.count)[: self.nsp], step=m.step, nonfinite=m.nonfinite,
                 continuity_max=m.continuity_max, j_max=m.j_max)
        A.check(rc, self.h)
        return d

    def get_run_state(self) -> dict:
        r = A.RunStateT()
        A.check(self.lib.pic_get_run_state(self.h, C.byref(r)), self.h)
        return dict(step=r.step, seed=r.seed, weight_bound=list(r.weight_bound)[: self.nsp])

    def set_run_state(self, st: dict):
        r = A.RunStateT()
        r.step, r.seed = st["step"], st["seed"]
        for i, b in enumerate(st["weight_bound"]):
            r.weight_bound[i] = b
        A.check(self.lib.pic_set_run_state(self.h, C.byref(r)), self.h)

    def mark_reference(self):
        A.check(self.lib.pic_mark_reference(self.h), self.h)

    def timing(self, enable: int = -1) -> dict:
        t = A.TimingT()
        A.check(self.lib.pic_timing(self.h, int(enable), C.byref(t)), self.h)
        return dict(push_ms=t.push_ms, migrate_ms=t.migrate_ms, field_ms=t.field_ms,
                    push_launches=t.push_launches, push_particles=t.push_particles)

    # ------------------------------------------------------------------ ionisation
    def ionize(self, mode: str = "exact", staged: bool = False) -> dict:
        """One ionisation step (pic_ionize, fused; staged: pic_ionize_staged,
        with the rate stage timed on its own)."""
        st = A.IonizeStatsT()
        fn = self.lib.pic_ionize_staged if staged else self.lib.pic_ionize
        A.check(fn(self.h, _MODE[mode], C.byref(st)), self.h)
        return dict(ions_active=st.ions_active, ionized=st.ionized, fallback=st.fallback, electrons=st.electrons,
                    rate_ms=st.rate_ms, total_ms=st.total_ms)

    def cell_moments(self, species: int):
        nx, ny, nz = self.shape
        ne = np.zeros(nx * ny * nz)
        kT = np.zeros(nx * ny * nz)
        A.check(self.lib.pic_cell_moments(self.h, species, _dptr(ne), _dptr(kT)), self.h)
        return ne, kT

    def cell_moments_device(self, species: int) -> tuple[int, int]:
        """Device addresses of the library-owned per-cell n_e and kT_e arrays
        (pic_cell_moments_device; nx*ny*nz doubles each, computed on the
        handle's stream)."""
        ne, kT = C.c_void_p(), C.c_void_p()
        A.check(self.lib.pic_cell_moments_device(self.h, species, C.byref(ne), C.byref(kT)), self.h)
        return ne.value, kT.value

    def rate_eval(self, mode: str, species: int, kT, ne, Z, noalloc: bool = False) -> np.ndarray:
        """ln nu per sample; noalloc stages through the library's static buffer
        (pic_rate_eval_noalloc, at most PIC_RATE_EVAL_NOALLOC_MAX samples)."""
        kT = np.ascontiguousarray(kT, dtype=np.float64)
        ne = np.ascontiguousarray(ne, dtype=np.float64)
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        out = np.zeros(kT.size)
        fn = self.lib.pic_rate_eval_noalloc if noalloc else self.lib.pic_rate_eval
        A.check(fn(self.h, _MODE[mode], species, kT.size, _dptr(kT), _dptr(ne),
                   Z.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(out)), self.h)
        return out

    def mlp_train(self, species: int, n_train=1_000_000, batch=4096, steps=20000, lr=3e-3, lr_final=1e-5,
                  seed=0, t_range=(1.0, 1e4), n_range=(1e19, 1e23), activation="silu") -> dict:
        cfg = A.MlpTrainCfgT(n_train, batch, steps, lr, lr_final, seed, t_range[0], t_range[1], n_range[0],
                             n_range[1], _ACT[activation], 0)
        rep = A.MlpReportT()
        A.check(self.lib.pic_mlp_train(self.h, species, C.byref(cfg), C.byref(rep)), self.h)
        return dict(loss_first=rep.loss_first, loss_last=rep.loss_last, mu=rep.mu, s=rep.s, train_ms=rep.train_ms,
                    steps=rep.steps)

    def mlp_get_params(self, species: int):
        """(params, (mu, s), trained range, activation name)."""
        p = np.zeros(A.PIC_MLP_NPARAM, dtype=np.float32)
        mu_s = np.zeros(2)
        rng = np.zeros(4)
        act = C.c_int32()
        A.check(self.lib.pic_mlp_get_params(self.h, species, p.ctypes.data_as(C.POINTER(C.c_float)), _dptr(mu_s),
                                            _dptr(rng), C.byref(act)), self.h)
        return p, mu_s, rng, _ACT_NAME[act.value]

    def mlp_set_params(self, species: int, params, mu_s, rng=None, activation="silu"):
        p = np.ascontiguousarray(params, dtype=np.float32)
        ms = np.ascontiguousarray(mu_s, dtype=np.float64)
        r = None if rng is None else np.ascontiguousarray(rng, dtype=np.float64)
        A.check(self.lib.pic_mlp_set_params(self.h, species, p.ctypes.data_as(C.POINTER(C.c_float)), _dptr(ms),
                                            None if r is None else _dptr(r), _ACT[activation]), self.h)

    def mlp_loss_grad(self, species: int, X, t):
        X = np.ascontiguousarray(X, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        loss = C.c_double()
        g = np.zeros(A.PIC_MLP_NPARAM, dtype=np.float32)
        A.check(self.lib.pic_mlp_loss_grad(self.h, species, X.shape[0], X.ctypes.data_as(C.POINTER(C.c_float)),
                                           t.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                           g.ctypes.data_as(C.POINTER(C.c_float))), self.h)
        return loss.value, g

    # ------------------------------------------------------------------ state
    def count(self, s: int) -> int:
        n = C.c_int64()
        A.check(self.lib.pic_particle_count(self.h, s, C.byref(n)), self.h)
        return n.value

    def get_particles(self, s: int) -> dict:
        n = self.count(s)
        out = {k: np.zeros(n, dtype=np.float64) for k in ("x", "y", "z")}
        out.update({k: np.zeros(n, dtype=self._rt) for k in ("ux", "uy", "uz", "w")})
        out["id"] = np.zeros(n, dtype=np.int64)
        out["zstate"] = np.zeros(n, dtype=np.int32)
        v = self._view(out, n)
        v.capacity = n
        get = self.lib.pic_get_particles64 if self.fp64 else self.lib.pic_get_particles
        A.check(get(self.h, s, C.byref(v)), self.h)
        return out

    def set_particles(self, s: int, p: dict):
        n = len(p["x"])
        arr = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ("x", "y", "z")}
        arr.update({k: np.ascontiguousarray(p[k], dtype=self._rt) for k in ("ux", "uy", "uz", "w")})
        arr["id"] = np.ascontiguousarray(p["id"], dtype=np.int64)
        arr["zstate"] = np.ascontiguousarray(p["zstate"], dtype=np.int32) if p.get("zstate") is not None else None
        v = self._view(arr, n)
        put = self.lib.pic_set_particles64 if self.fp64 else self.lib.pic_set_particles
        A.check(put(self.h, s, C.byref(v)), self.h)

    def _view(self, a: dict, n: int):
        v = A.ParticlesView64T() if self.fp64 else A.ParticlesViewT()
        ct = C.c_double if self.fp64 else C.c_float
        v.count = n
        v.capacity = n
        for k in ("x", "y", "z"):
            setattr(v, k, a[k].ctypes.data_as(C.POINTER(C.c_double)))
        for k in ("ux", "uy", "uz", "w"):
            setattr(v, k, a[k].ctypes.data_as(C.POINTER(ct)))
        v.id = a["id"].ctypes.data_as(C.POINTER(C.c_int64))
        if a.get("zstate") is not None:
            v.zstate = a["zstate"].ctypes.data_as(C.POINTER(C.c_int32))
        return v

    def get_fields(self):
        nx, ny, nz = self.shape
        E, B, J = (np.zeros((3, nz, ny, nx), dtype=self._rt) for _ in range(3))
        get = self.lib.pic_get_fields64 if self.fp64 else self.lib.pic_get_fields
        A.check(get(self.h, E.ctypes.data, B.ctypes.data, J.ctypes.data), self.h)
        return E, B, J

    def set_fields(self, E=None, B=None, J=None):
        nx, ny, nz = self.shape
        conv = [None if f is None else np.ascontiguousarray(np.asarray(f, dtype=self._rt).reshape(3, nz, ny, nx))
                for f in (E, B, J)]
        ptrs = [None if f is None else f.ctypes.data for f in conv]
        put = self.lib.pic_set_fields64 if self.fp64 else self.lib.pic_set_fields
        A.check(put(self.h, *ptrs), self.h)
