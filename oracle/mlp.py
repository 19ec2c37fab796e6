"""FP64 reference of the ionisation-rate surrogate network
(TEST INFRASTRUCTURE; only tests and the benchmark's CPU leg use it).

The network replaces the per-ion Maxwellian-averaged Lotz quadrature:
  inputs  x0 = (log10 T_e[eV] - 2)/2, x1 = (log10 n_e[cm^-3] - 21)/2,
          x2..x7 = one-hot of the charge state Z in 0..5;
  layers  h1 = f(W1 x + b1), h2 = f(W2 h1 + b2), y = W3 h2 + b3, widths
          8 -> 64 -> 64 -> 1, with f = SiLU(z) = z sigmoid(z) (the default) or
          f = ReLU(z) = max(z, 0) (derivative taken as 1 for z > 0, else 0);
  output  ln nu = ln nu_prior + mu + s * y, where the prior is the rate with
          e^z E1(z) replaced by its upper bound ln(1 + 1/z), z = P/kT:
          ln nu_prior = ln(n_e vbar a q / (P kT)) - z + ln ln(1 + 1/z).
The learned residual ln nu - ln nu_prior = ln(e^z E1(z) / ln(1+1/z)) is
bounded because (1/2) ln(1 + 2/z) < e^z E1(z) < ln(1 + 1/z).
Training loss: mean of (y - target)^2 over a batch.
"""
from __future__ import annotations

import math

import numpy as np

from .ionize import LOTZ_A, ME_C2_EV, vbar

N_IN, N_H = 8, 64


def features(T_eV, ne_cm3, Z):
    T_eV, ne_cm3 = np.asarray(T_eV, dtype=np.float64), np.asarray(ne_cm3, dtype=np.float64)
    Z = np.asarray(Z).astype(np.int64)
    X = np.zeros((T_eV.size, N_IN))
    X[:, 0] = (np.log10(T_eV) - 2.0) / 2.0
    X[:, 1] = (np.log10(ne_cm3) - 21.0) / 2.0
    X[np.arange(T_eV.size), 2 + Z] = 1.0
    return X


def ln_rate_prior(kT, ne, P, q, a=LOTZ_A):
    """The analytic prior: the outermost subshell's plain Lotz rate with
    e^z E1(z) replaced by ln(1 + 1/z) (z = P/kT)."""
    kT, ne, P, q, a = (np.asarray(v, dtype=np.float64) for v in (kT, ne, P, q, a))
    z = P / kT
    return np.log(ne * vbar(kT) * a * q / (P * kT)) - z + np.log(np.log1p(1.0 / z))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def relu(z):
    return np.maximum(z, 0.0)


def drelu(z):
    return (np.asarray(z) > 0.0).astype(np.float64)


ACTIVATIONS = {"silu": (silu, dsilu), "relu": (relu, drelu)}


def init_params(seed: int):
    """He-style uniform initial weights (any fixed initialisation will do)."""
    r = np.random.default_rng(seed)
    W1 = r.uniform(-1, 1, (N_H, N_IN)) * math.sqrt(3.0 / N_IN)
    W2 = r.uniform(-1, 1, (N_H, N_H)) * math.sqrt(3.0 / N_H)
    W3 = r.uniform(-1, 1, (1, N_H)) * math.sqrt(3.0 / N_H)
    return dict(W1=W1, b1=np.zeros(N_H), W2=W2, b2=np.zeros(N_H), W3=W3, b3=np.zeros(1))


def forward(p, X, act: str = "silu"):
    f = ACTIVATIONS[act][0]
    z1 = X @ p["W1"].T + p["b1"]
    h1 = f(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = f(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(p, X, t, act: str = "silu"):
    """MSE loss mean((y - t)^2) and its analytic gradient (backpropagation)."""
    df = ACTIVATIONS[act][1]
    y, c = forward(p, X, act)
    B = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / B) * r[:, None]                 # (B,1)
    g = {}
    g["W3"] = dy.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * df(c["z2"])
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * df(c["z1"])
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def ln_rate(p, mu, s, T_eV, ne_cm3, Z, P_table, q_table, a_table=None, act: str = "silu"):
    """Surrogate ln nu for given inputs (FP64 evaluation of the network);
    P, q, a of each state's outermost subshell (a defaults to 4.5e-14)."""
    Z = np.asarray(Z).astype(np.int64)
    P = np.asarray(P_table, dtype=np.float64)[Z]
    q = np.asarray(q_table, dtype=np.float64)[Z]
    a = LOTZ_A if a_table is None else np.asarray(a_table, dtype=np.float64)[Z]
    y, _ = forward(p, features(T_eV, ne_cm3, Z), act)
    return ln_rate_prior(T_eV, ne_cm3, P, q, a) + mu + s * y


__all__ = ["features", "ln_rate_prior", "silu", "relu", "ACTIVATIONS", "forward", "loss_and_grad", "init_params",
           "ln_rate", "ME_C2_EV"]
