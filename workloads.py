"""Workload presets and seeded input generators.

This module is the only thing the HIP path and the FP64 oracle both use.  It
holds plain parameters (grid sizes, time step, particles per cell, thermal and
drift speeds, masses, charges) and seeded random numbers, and none of the
method's arithmetic: each side converts drift speeds to momenta, macro-particle
weights and so on by itself.

The presets mirror the benchmark the paper runs (section "Evaluation": a
Kelvin-Helmholtz shear flow on a 128^3 grid with electrons and ions, Boris,
Esirkepov, Yee, TSC) at the sizes used here: a small FP64-checkable case, a
128^3 CIC electron shear layer, a 256x256x128 TSC electron-proton plasma in a
background field, and a 128^3 electron-carbon plasma with Monte Carlo
electron-impact ionisation (exact quadrature rates or the learned surrogate).
Units are normalised: c = eps0 = 1, e = m_e = 1, n0 = 1, lengths in c/omega_p.
"""
from __future__ import annotations

import copy

import numpy as np

SEED_BASE = 160602862

# Carbon: ionisation energies (eV) of C^{Z+} for Z = 0..5 and the number of
# electrons in the outermost subshell of each state (2p2, 2p1, 2s2, 2s1, 1s2, 1s1).
CARBON_IONIZATION_EV = (11.3, 24.4, 47.9, 64.5, 392.0, 490.0)
CARBON_LOTZ_Q = (2, 1, 2, 1, 2, 1)
PROTON_MASS = 1836.0
CARBON_MASS = 12.0 * 1822.888


def _electron(ppc, u_th, drift_beta=(0.0, 0.0, 0.0), layout="uniform", cap_ppc=None):
    return dict(name="electron", charge=-1.0, mass=1.0, ppc=ppc, density=1.0, u_th=u_th,
                drift_beta=tuple(drift_beta), layout=layout, mobile=True, coincident_with=-1,
                z_init=0, z_max=0, ionization_ev=(), lotz_q=(), cap_ppc=cap_ppc)


def _config(idx):
    if idx == 0:
        return dict(
            name="e16_cic", workload="16^3 CIC electrons, 8 ppc, u_th 0.05, immobile background",
            grid=dict(nx=16, ny=16, nz=16, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.0),
                      rho_bg=1.0, shape="cic", seed=SEED_BASE + 0, n_ref_cm3=1e21),
            species=[_electron(8, 0.05)], steps=100)
    if idx == 1:
        return dict(
            name="shear128_cic", workload="128^3 CIC electron shear layer +-0.2c, 16 ppc, sorted every step",
            grid=dict(nx=128, ny=128, nz=128, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.0),
                      rho_bg=1.0, shape="cic", seed=SEED_BASE + 1, n_ref_cm3=1e21),
            species=[_electron(16, 0.01, (0.2, 0.0, 0.0), "shear")], steps=200)
    if idx == 2:
        prot = dict(name="proton", charge=1.0, mass=PROTON_MASS, ppc=8, density=1.0, u_th=0.0005,
                    drift_beta=(0.0, 0.0, 0.0), layout="uniform", mobile=True, coincident_with=0,
                    z_init=0, z_max=0, ionization_ev=(), lotz_q=(), cap_ppc=None)
        return dict(
            name="ep256_tsc", workload="256x256x128 TSC electrons+protons 8+8 ppc, B0=0.1 z",
            grid=dict(nx=256, ny=256, nz=128, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.1),
                      rho_bg=0.0, shape="tsc", seed=SEED_BASE + 2, n_ref_cm3=1e21),
            species=[_electron(8, 0.02), prot], steps=100)
    if idx in (3, 4):
        carbon = dict(name="carbon", charge=1.0, mass=CARBON_MASS, ppc=4, density=0.5,
                      u_th=1.35e-4, drift_beta=(0.0, 0.0, 0.0), layout="uniform", mobile=True,
                      coincident_with=0, z_init=2, z_max=6,
                      ionization_ev=CARBON_IONIZATION_EV, lotz_q=CARBON_LOTZ_Q, cap_ppc=None, ionize_into=0)
        return dict(
            name="ec128_tsc_ionize" + ("_mlp" if idx == 4 else "_exact"),
            workload="128^3 TSC electrons 8 ppc + C2+ 4 ppc, B0=0.1 z, Monte Carlo ionisation ("
                     + ("MLP surrogate" if idx == 4 else "exact GL-64") + ")",
            grid=dict(nx=128, ny=128, nz=128, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.1),
                      rho_bg=0.0, shape="tsc", seed=SEED_BASE + idx, n_ref_cm3=1e21),
            species=[_electron(8, 0.02, cap_ppc=28), carbon], steps=100,
            rate_mode="mlp" if idx == 4 else "exact")
    if idx == 5:
        # the paper's benchmark: Kelvin-Helmholtz shear flow, electrons and ions
        # at 16 ppc each, TSC; both species drift together in each layer (no
        # net current), ions at the electrons' temperature
        ion = dict(name="proton", charge=1.0, mass=PROTON_MASS, ppc=16, density=1.0,
                   u_th=0.01 / PROTON_MASS ** 0.5, drift_beta=(0.2, 0.0, 0.0), layout="shear", mobile=True,
                   coincident_with=0, z_init=0, z_max=0, ionization_ev=(), lotz_q=(), cap_ppc=None)
        return dict(
            name="khi128_tsc", workload="128^3 TSC Kelvin-Helmholtz shear flow +-0.2c, electrons + protons 16 ppc each",
            grid=dict(nx=128, ny=128, nz=128, dx=1.0, dy=1.0, dz=1.0, dt=0.5, b0=(0.0, 0.0, 0.0),
                      rho_bg=0.0, shape="tsc", seed=SEED_BASE + 5, n_ref_cm3=1e21),
            species=[_electron(16, 0.01, (0.2, 0.0, 0.0), "shear"), ion], steps=1000)
    raise ValueError(f"no preset {idx}")


def config(idx: int, **grid_overrides) -> dict:
    """Preset `idx` (0..5); keyword arguments replace grid entries (e.g. a
    smaller nx/ny/nz for a parity run at the same physics)."""
    c = copy.deepcopy(_config(idx))
    c["grid"].update(grid_overrides)
    return c


def reduced(idx: int, nx: int, ny: int, nz: int) -> dict:
    """Preset `idx` on a smaller periodic box (same physics and seed rule)."""
    return config(idx, nx=nx, ny=ny, nz=nz)


# --------------------------------------------------------------------------
# Seeded generators (random numbers only).

def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_fields(seed: int, nx: int, ny: int, nz: int, amp: float = 0.05) -> tuple[np.ndarray, np.ndarray]:
    """E and B with independent uniform(-amp, amp) entries, shape (3, nz, ny, nx), fp32-representable."""
    g = rng(seed)
    E = g.uniform(-amp, amp, size=(3, nz, ny, nx)).astype(np.float32).astype(np.float64)
    B = g.uniform(-amp, amp, size=(3, nz, ny, nx)).astype(np.float32).astype(np.float64)
    return E, B


def random_particles(seed: int, n: int, nx: int, ny: int, nz: int, u_scale: float = 0.1) -> dict:
    """n particles at uniform random positions in the box and Gaussian momenta."""
    g = rng(seed)
    return dict(
        x=g.uniform(0, nx, n), y=g.uniform(0, ny, n), z=g.uniform(0, nz, n),
        ux=g.normal(0, u_scale, n), uy=g.normal(0, u_scale, n), uz=g.normal(0, u_scale, n),
        w=np.full(n, 0.125), id=np.arange(n, dtype=np.int64))


# Surrogate training recipe: 1M log-uniform samples, batch 4096, ~20k Adam
# steps with cosine decay from 3e-3; held-out evaluation on a different seed.
MLP_TRAIN = dict(n_train=1_000_000, batch=4096, steps=20000, lr=3e-3, lr_final=1e-5, t_range=(1.0, 1e4),
                 n_range=(1e19, 1e23))
MLP_TRAIN_SEED = SEED_BASE + 100
MLP_HELDOUT_SEED = SEED_BASE + 200


def loguniform_rate_inputs(seed: int, n: int, t_range=(1.0, 1e4), n_range=(1e19, 1e23), zmax: int = 6):
    """Electron temperature (eV), density (cm^-3) and charge state samples:
    log-uniform T and n, Z uniform over 0..zmax-1."""
    g = rng(seed)
    T = 10.0 ** g.uniform(np.log10(t_range[0]), np.log10(t_range[1]), n)
    ne = 10.0 ** g.uniform(np.log10(n_range[0]), np.log10(n_range[1]), n)
    Z = g.integers(0, zmax, n).astype(np.uint8)
    return T, ne, Z
