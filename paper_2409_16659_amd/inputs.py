"""Seeded synthetic films: parameter sets and initial height fields.

This module only *draws inputs*; it holds none of the solver's arithmetic.
It is the one module that both the HIP path and the FP64 oracle consume, so
that both always see byte-identical inputs.

The paper initialises flat films plus a small random perturbation,
h_i = h_{0,i} + eps * noise (Sec. IV.A, IV.E, IV.F); it does not state the
noise distribution, so each workload fixes its own (multi-mode random phase,
uniform, or lognormal), always drawn in FP64 from numpy's PCG64(seed).

A film is a plain dict:
    n_layers, nx, ny, tau, hstar, exp_a, exp_b,
    gamma  [N]  gamma_{i,i+1}, i = 1..N (gamma_N is layer N / gas)
    mu     [N]  viscosities
    slip   [N]  slip lengths (0 = no slip)
    spread {(l, k): S_lk}  spreading coefficients, l = 0..N-1, k = 1..N-l
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "film_params", "young_spreading", "multimode_noise", "uniform_noise",
    "lognormal_heights", "initial_heights", "WORKLOADS", "workload", "batch_scan",
]


def young_spreading(gamma_above: float, theta_deg: float) -> float:
    """Spreading coefficient of a layer that meets the phase below at angle
    theta: S = gamma (cos theta - 1).  Input recipe only (Young's law,
    Eq. youngs_law, with S = gamma_sv - gamma_sl - gamma)."""
    return gamma_above * (math.cos(math.radians(theta_deg)) - 1.0)


def film_params(n_layers, nx, ny, *, gamma, mu, hstar, spread=None, tau=1.0,
                exp_a=9, exp_b=3, slip=None) -> dict:
    n = int(n_layers)
    if not 1 <= n <= 4:
        raise ValueError("1 <= n_layers <= 4")
    return {
        "n_layers": n, "nx": int(nx), "ny": int(ny), "tau": float(tau),
        "hstar": float(hstar), "exp_a": int(exp_a), "exp_b": int(exp_b),
        "gamma": [float(g) for g in gamma][:n],
        "mu": [float(m) for m in mu][:n],
        "slip": [0.0] * n if slip is None else [float(s) for s in slip][:n],
        "spread": {} if spread is None else {tuple(k): float(v) for k, v in dict(spread).items()},
    }


def multimode_noise(rng, nx, ny, modes, rms):
    """sum_{m=1}^{modes} cos(2 pi m x / nx + phase_m), phases ~ U[0, 2pi),
    scaled to the requested RMS; constant along y."""
    x = np.arange(nx, dtype=np.float64)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    amp = rms * math.sqrt(2.0 / modes)
    row = np.zeros(nx)
    for m in range(1, modes + 1):
        row += np.cos(2.0 * math.pi * m * x / nx + ph[m - 1])
    return np.broadcast_to(amp * row, (ny, nx)).copy()


def uniform_noise(rng, shape, amp):
    return rng.uniform(-amp, amp, size=shape)


def lognormal_heights(rng, hbar, shape, sigma):
    z = rng.standard_normal(size=shape)
    return hbar * np.exp(sigma * z - 0.5 * sigma * sigma)


def initial_heights(film: dict, hbar, noise: str, seed: int, amp: float, modes: int = 64):
    """h[N][ny][nx] in FP64 for the given noise recipe."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, nx, ny = film["n_layers"], film["nx"], film["ny"]
    h = np.empty((n, ny, nx))
    for i in range(n):
        if noise == "multimode":
            h[i] = hbar[i] + multimode_noise(rng, nx, ny, modes, amp)
        elif noise == "uniform":
            h[i] = hbar[i] + uniform_noise(rng, (ny, nx), amp)
        elif noise == "lognormal":
            h[i] = lognormal_heights(rng, hbar[i], (ny, nx), amp)
        elif noise == "none":
            h[i] = hbar[i]
        else:
            raise ValueError(noise)
    return h


# ---------------------------------------------------------------------------
# Workloads shaped like the paper's experiments (Sec. IV).  Spreading
# coefficients follow the 3-layer rupture pattern of Sec. IV.E: single-layer
# coefficients negative (contact angle 20 degrees), multi-layer ones zero.


def _film2_pseudo1d(nx=512):
    # Lubrication regime of the tau = 1 scheme: the collective friction
    # 3 mu / (h1 + h2)^2 dominates the lattice's own flux damping at the
    # unstable wavenumbers, the explicit friction stays stable down to h*
    # (largest eigenvalue of -K with layers at h* is 1.2 < 2), and the
    # capillary term is stable at every wavenumber.
    g = 0.1
    return film_params(2, nx, 1, gamma=[g, g], mu=[0.038, 0.038], hstar=0.5,
                       spread={(0, 1): 0.0, (1, 1): young_spreading(g, 8.0), (0, 2): 0.0})


def _film3(nx, ny):
    gam = [1.0e-2, 0.7e-2, 0.5e-2]
    mu = [2e-3 * 1.0, 2e-3 * 1.5, 2e-3 * 2.0]
    spread = {(l, 1): young_spreading(gam[l], 20.0) for l in range(3)}
    spread.update({(0, 2): 0.0, (1, 2): 0.0, (0, 3): 0.0})
    return film_params(3, nx, ny, gamma=gam, mu=mu, hstar=0.15, spread=spread)


def _film4(nx, ny):
    gam = [1.0e-2, 0.8e-2, 0.6e-2, 0.5e-2]
    mu = [1e-3 * 1.0, 1e-3 * 1.5, 1e-3 * 2.0, 1e-3 * 2.5]
    spread = {(l, 1): young_spreading(gam[l], 20.0) for l in range(4)}
    return film_params(4, nx, ny, gamma=gam, mu=mu, hstar=0.1, spread=spread)


WORKLOADS = {
    # 2 layers, pseudo-1D, FP64: noise-perturbed flat films as in the
    # linear-stability comparison (Sec. IV.A).
    "film2_pseudo1d_512": dict(make=lambda: _film2_pseudo1d(512), hbar=(1.0, 1.0),
                               noise="multimode", amp=0.01, seed=1, steps=10_000,
                               precision="f64"),
    # 3 layers on a 2D periodic field, FP32: spinodal rupture (Sec. IV.E).
    "film3_2d_1024": dict(make=lambda: _film3(1024, 1024), hbar=(1.0, 0.8, 0.6),
                          noise="uniform", amp=1e-3, seed=2, steps=100_000,
                          precision="f32"),
    # same parameters on a field too large for the on-die caches
    "film3_2d_4096": dict(make=lambda: _film3(4096, 4096), hbar=(1.0, 0.8, 0.6),
                          noise="uniform", amp=1e-3, seed=2, steps=1_000,
                          precision="f32"),
    # 4 layers, 4096^2, 16-bit population storage (IEEE-half moving
    # populations; the rest population, which carries the height, in FP32)
    "film4_2d_4096": dict(make=lambda: _film4(4096, 4096), hbar=(1.0, 0.8, 0.6, 0.4),
                          noise="lognormal", amp=1e-3, seed=4, steps=50_000,
                          precision="f16mix"),
    # the [0:512, 0:512] window of the 4096^2 fields above, run as its own
    # periodic domain (accuracy of the 16-bit storage against FP64)
    "film4_2d_512": dict(make=lambda: _film4(512, 512), crop_of="film4_2d_4096",
                         hbar=(1.0, 0.8, 0.6, 0.4), noise="lognormal", amp=1e-3,
                         seed=4, steps=50_000, precision="f16mix"),
}


def batch_scan(count=256, seed=3, side_min=64, side_max=512, hstar=0.15):
    """Films of a stability scan (the paper's parameter sweeps, Sec. IV):
    square side uniform on the multiples of 16 in [side_min, side_max],
    N uniform in {2, 3, 4}, gamma_i ~ U[0.5, 1.5]e-2, contact angle theta ~
    U[10, 30] degrees giving S_l1 = gamma_{l+1}(cos theta - 1) (multi-layer
    S = 0), mean heights (1, 0.8, 0.6, 0.4)[:N], a single mode
    1e-3 cos(2 pi m x / s) with m ~ U{1..s/16} plus U(-1e-5, 1e-5) noise,
    h* = 0.15 and mu_i = 0.09 h*^2 U[0.5, 1] (with every layer at h* the
    largest friction rate stays below 1 for N <= 4).
    Returns a list of (film, h0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = np.arange(side_min, side_max + 1, 16)
    out = []
    for _ in range(count):
        s = int(rng.choice(sides))
        n = int(rng.integers(2, 5))
        gam = list(rng.uniform(0.5e-2, 1.5e-2, size=n))
        theta = float(rng.uniform(10.0, 30.0))
        mu = list(0.09 * hstar * hstar * rng.uniform(0.5, 1.0, size=n))
        spread = {(l, 1): young_spreading(gam[l], theta) for l in range(n)}
        film = film_params(n, s, s, gamma=gam, mu=mu, hstar=hstar, spread=spread)
        m = int(rng.integers(1, s // 16 + 1))
        x = np.arange(s, dtype=np.float64)
        mode = 1e-3 * np.cos(2.0 * math.pi * m * x / s)
        hbar = (1.0, 0.8, 0.6, 0.4)[:n]
        h0 = np.stack([hbar[i] + mode[None, :] + uniform_noise(rng, (s, s), 1e-5) for i in range(n)])
        out.append((film, h0))
    return out


def workload(name: str, nx=None, ny=None):
    """(film, h0, spec) for a named workload; nx/ny override the grid."""
    spec = WORKLOADS[name]
    film = spec["make"]()
    if nx is not None:
        film["nx"] = int(nx)
    if ny is not None:
        film["ny"] = int(ny)
    if "crop_of" in spec and nx is None and ny is None:
        parent = WORKLOADS[spec["crop_of"]]
        big = initial_heights(parent["make"](), parent["hbar"], parent["noise"],
                              parent["seed"], parent["amp"])
        h0 = np.ascontiguousarray(big[:, :film["ny"], :film["nx"]])
    else:
        h0 = initial_heights(film, spec["hbar"], spec["noise"], spec["seed"], spec["amp"])
    return film, h0, spec
