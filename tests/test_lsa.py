"""The N-layer linear stability tool (paper_2409_16659_amd/lsa.py) against
what fixes it independently of its own formulas:

* N = 2: the printed two-layer analysis (Sec. IV.A; mobility from
  tests/golden/mobility_2layer.txt), entry by entry;
* N = 1: the textbook single-film rate -q^2 h^3/(3 mu) (gamma q^2 + S phi'');
* the pressure Jacobian E against central differences of the oracle's
  discrete pressures (with the lattice Laplacian's symbol 2 - 2 cos k in
  place of q^2), and the mobility against the oracle's friction solve;
* Onsager symmetry without slip: P M symmetric positive definite and the
  interface-coordinate Hessian E P^-1 symmetric, hence real rates;
* the dynamics: an eigenmode of the lattice model, seeded into the FP64
  oracle, grows at the predicted rate (the paper's own validation compares
  the simulated spectrum with the continuum analysis; the lattice model
  makes that comparison sharp outside the friction-dominated regime).
"""
import math

import numpy as np
import pytest

from paper_2409_16659_amd import inputs, lsa
from tests.test_oracle_lsa import lsa_matrix


def random_film(rng, n, slip=False):
    gam = list(rng.uniform(0.5e-2, 1.5e-2, n))
    mu = list(rng.uniform(1e-3, 5e-3, n))
    spread = {(l, k): float(rng.uniform(-2e-3, 1e-3)) for l in range(n) for k in range(1, n - l + 1)}
    f = inputs.film_params(n, 64, 1, gamma=gam, mu=mu, hstar=0.15, spread=spread,
                           slip=list(rng.uniform(0.0, 1.0, n)) if slip else None)
    return f, rng.uniform(0.3, 1.2, n)


def test_two_layer_equals_printed_analysis():
    film, _, spec = inputs.workload("film2_pseudo1d_512")
    hbar = np.array(spec["hbar"])
    for q in (0.005, 0.03, 0.1, 0.4):
        A, B = lsa.growth_matrix(film, hbar, q), lsa_matrix(film, hbar, q)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max(), q
    rng = np.random.default_rng(1)
    for _ in range(5):   # every spreading coefficient non-zero, unequal layers
        film, hbar = random_film(rng, 2)
        for q in (0.02, 0.2):
            A, B = lsa.growth_matrix(film, hbar, q), lsa_matrix(film, hbar, q)
            assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


def test_single_layer_closed_form():
    rng = np.random.default_rng(2)
    for _ in range(5):
        film, hbar = random_film(rng, 1)
        h, mu, g, S = hbar[0], film["mu"][0], film["gamma"][0], film["spread"][(0, 1)]
        _, _, d2 = lsa.phi_derivatives(1, h, film["hstar"])
        for q in (0.01, 0.1, 0.5):
            want = -q * q * h ** 3 / (3 * mu) * (g * q * q + S * d2)
            got = lsa.growth_rates(film, hbar, q)[0].real
            assert abs(got - want) <= 1e-13 * abs(want)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_pressure_jacobian_matches_oracle_pressures(oracle_mod, n):
    rng = np.random.default_rng(10 + n)
    film, hbar = random_film(rng, n)
    nx, m, eps = 64, 3, 1e-6
    k = 2 * math.pi * m / nx
    x = np.arange(nx)
    E = lsa.pressure_jacobian(film, hbar, math.sqrt(2 - 2 * math.cos(k)))
    base = np.broadcast_to(hbar[:, None, None], (n, 1, nx)).copy()
    Efd = np.zeros((n, n))
    for j in range(n):
        hp, hm = base.copy(), base.copy()
        hp[j, 0] += eps * np.cos(k * x)
        hm[j, 0] -= eps * np.cos(k * x)
        dD = oracle_mod.pressure(film, hp)[1] - oracle_mod.pressure(film, hm)[1]
        Efd[:, j] = dD[:, 0] @ np.cos(k * x) / (eps * nx)
    assert np.abs(E - Efd).max() <= 1e-7 * np.abs(E).max()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("slip", [False, True])
def test_mobility_matches_oracle_friction(oracle_mod, n, slip):
    rng = np.random.default_rng(20 + n)
    film, hbar = random_film(rng, n, slip)
    K = np.stack([oracle_mod.friction(hbar, film["mu"], np.eye(n)[j], film["slip"]) for j in range(n)], axis=1)
    T = np.triu(np.ones((n, n))) * hbar[:, None]
    M = lsa.mobility(film, hbar)
    assert np.abs(M + np.linalg.solve(K, T)).max() <= 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_onsager_symmetry_without_slip(n):
    rng = np.random.default_rng(30 + n)
    P = np.tril(np.ones((n, n)))
    for _ in range(4):
        film, hbar = random_film(rng, n)
        PM = P @ lsa.mobility(film, hbar)
        assert np.abs(PM - PM.T).max() <= 1e-12 * np.abs(PM).max()
        assert np.linalg.eigvalsh(PM).min() > 0
        Ez = lsa.pressure_jacobian(film, hbar, 0.1) @ np.linalg.inv(P)
        assert np.abs(Ez - Ez.T).max() <= 1e-12 * np.abs(Ez).max()
        assert np.abs(lsa.growth_rates(film, hbar, 0.1).imag).max() == 0.0


def test_lattice_model_tends_to_lubrication():
    """With friction far above the growth and the lattice damping the two
    models agree: the relative gap falls like 1 / viscosity (the lattice
    damping and the inertia against the friction)."""
    film0, hbar = inputs._film3(256, 1), (1.0, 0.8, 0.6)
    for m in (2, 6, 10):
        q = 2 * math.pi * m / 256
        gaps = []
        for scale in (100, 1000):
            film = dict(film0, mu=[scale * v for v in film0["mu"]])
            a = lsa.growth_rates(film, hbar, q)[0].real
            b = lsa.growth_rates(film, hbar, q, "lattice")[0].real
            gaps.append(abs(b - a) / abs(a))
        assert gaps[1] <= 2e-3 and 8 <= gaps[0] / gaps[1] <= 12, (m, gaps)


def measured_rate(oracle_mod, film, hbar, m, t0=500, t1=5000, eps=1e-7):
    """Seed the leading lattice eigenmode of wavenumber 2 pi m / nx into a
    pseudo-1D film and measure the growth of that Fourier mode."""
    n, nx = film["n_layers"], film["nx"]
    q = 2 * math.pi * m / nx
    rate, dh, w = lsa.leading_mode(film, hbar, q, "lattice")
    x = np.arange(nx)
    hb = np.asarray(hbar)
    h0 = hb[:, None, None] + eps * dh[:, None, None] * np.cos(q * x)
    u0 = eps * w[:, None, None] * np.sin(q * x) / h0
    o = oracle_mod.Oracle(film)
    o.init(h0, u0)
    amp = []
    for t in (t0, t1):
        o.step(t - o.steps_done)
        amp.append(np.fft.fft(o.read()[0][:, 0, :] - hb[:, None], axis=1)[:, m])
    return rate, math.log(np.linalg.norm(amp[1]) / np.linalg.norm(amp[0])) / (t1 - t0)


@pytest.mark.parametrize("case", ["film2", "film3", "film4", "film3_tau0.8", "film3_tau1.3"])
def test_lattice_model_predicts_the_scheme(oracle_mod, case):
    """Measured growth of seeded eigenmodes across the unstable band within
    1 % of the lattice model (and, outside the friction-dominated regime,
    far from the lubrication rate)."""
    if case == "film2":
        film, _, spec = inputs.workload("film2_pseudo1d_512")
        hbar, modes = spec["hbar"], (2, 8, 12)
    elif case == "film4":
        film, hbar, modes = inputs._film4(256, 1), (1.0, 0.8, 0.6, 0.4), (2, 7, 12)
    else:
        film, hbar, modes = inputs._film3(256, 1), (1.0, 0.8, 0.6), (2, 6, 9)
        if "tau" in case:
            film = dict(film, tau=float(case.split("tau")[1]))
    for m in modes:
        want, got = measured_rate(oracle_mod, film, hbar, m)
        print(f"{case} m={m}: lattice {want:.4e} measured {got:.4e} "
              f"lubrication {lsa.growth_rates(film, hbar, 2 * math.pi * m / film['nx'])[0].real:.4e}")
        assert abs(got - want) <= 0.01 * abs(want), (m, want, got)
