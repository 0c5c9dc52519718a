"""Whole-step pins of the oracle: invariants of the scheme (mass, rest state,
lattice translations, thread count, D2Q9 on one row = D1Q3) and the exact
discrete linearisation about a flat multilayer film."""
import math

import numpy as np
import pytest

from paper_2409_16659_amd import inputs
from tests.test_oracle_pressure_friction import exact_friction_global


def small_film(n, nx, ny, seed=0, hstar=0.15):
    rng = np.random.default_rng(seed)
    gam = list(rng.uniform(0.5e-2, 1.5e-2, size=n))
    spread = {(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(n)}
    for l in range(n):
        for k in range(2, n - l + 1):
            spread[(l, k)] = rng.uniform(-2e-3, 2e-3)
    mu = list(rng.uniform(2e-3, 5e-3, size=n))
    return inputs.film_params(n, nx, ny, gamma=gam, mu=mu, hstar=hstar, spread=spread)


def noisy(n, nx, ny, seed, amp=1e-2, hbar=None):
    rng = np.random.default_rng(seed)
    hbar = hbar or [1.0 - 0.15 * i for i in range(n)]
    return np.stack([hbar[i] + amp * rng.uniform(-1, 1, size=(ny, nx)) for i in range(n)])


def test_flat_film_is_a_fixed_point(oracle_mod):
    """Uniform heights at rest: f = f^eq(h, 0) has zero pressure gradient and
    zero friction, so the state is reproduced bit for bit."""
    film = small_film(3, 9, 7)
    h = np.stack([np.full((7, 9), v) for v in (0.9, 0.6, 0.45)])
    o = oracle_mod.Oracle(film)
    o.init(h)
    f0 = o.get_f()
    o.step(200)
    assert np.array_equal(o.get_f(), f0)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_mass_conserved(oracle_mod, n):
    film = small_film(n, 24, 20, seed=n)
    o = oracle_mod.Oracle(film)
    o.init(noisy(n, 24, 20, seed=10 + n))
    m0 = o.mass()
    o.step(300)
    assert np.abs(o.mass() - m0).max() <= 1e-12 * m0.max() * 1e-1


def test_lattice_translation_equivariance(oracle_mod):
    """Shifting the input populations by a lattice vector shifts the output
    by the same vector, bit for bit (streaming and stencils are periodic and
    translation invariant)."""
    film = small_film(2, 11, 8, seed=3)
    o = oracle_mod.Oracle(film)
    o.init(noisy(2, 11, 8, seed=4))
    o.step(3)
    f = o.get_f()
    o.step(5)
    want = np.roll(np.roll(o.get_f(), 3, axis=3), -2, axis=2)
    o2 = oracle_mod.Oracle(film)
    o2.set_f(np.roll(np.roll(f, 3, axis=3), -2, axis=2))
    o2.step(5)
    assert np.array_equal(o2.get_f(), want)


def test_thread_count_does_not_change_results(oracle_mod):
    film = small_film(3, 30, 17, seed=5)
    h = noisy(3, 30, 17, seed=6)
    outs = []
    keep = oracle_mod.get_threads()
    try:
        for t in (1, 3, 8):
            oracle_mod.set_threads(t)
            o = oracle_mod.Oracle(film)
            o.init(h)
            o.step(20)
            outs.append(o.get_f())
    finally:
        oracle_mod.set_threads(keep)
    assert all(np.array_equal(outs[0], x) for x in outs[1:])


def test_d2q9_single_row_equals_d1q3(oracle_mod):
    """On an Nx x 1 grid the D2Q9 populations lumped per x-direction are the
    D1Q3 ones (weights 2/3, 1/6, 1/6), so both lattices give the same
    heights and fluxes up to rounding."""
    film = small_film(2, 64, 1, seed=7)
    h = noisy(2, 64, 1, seed=8)
    a = oracle_mod.Oracle(film, oracle_mod.D2Q9)
    b = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    a.init(h)
    b.init(h)
    a.step(2000)
    b.step(2000)
    ha, ua, va = a.read()
    hb, ub, _ = b.read()
    assert np.abs(ha - hb).max() <= 1e-13
    assert np.abs(ua - ub).max() <= 1e-10 * np.abs(ub).max()
    assert np.abs(va).max() < 1e-14 * np.abs(ua).max()


def test_nonpositive_height_is_reported(oracle_mod):
    film = small_film(2, 5, 4)
    o = oracle_mod.Oracle(film)
    h = np.ones((2, 4, 5))
    h[1, 2, 3] = -0.1
    with pytest.raises(oracle_mod.OracleError) as e:
        o.init(h)
    assert e.value.code == oracle_mod.ENONPOSITIVE
    h[1, 2, 3] = np.nan
    with pytest.raises(oracle_mod.OracleError) as e:
        o.init(h)
    assert e.value.code == oracle_mod.ENONFINITE


# --------------------------------------------- exact discrete linearisation
def phi2(k, d, hs, a=9, b=3):
    """Second derivative of phi_k(d) = (a r^b - b r^a)/(a - b), r = k h*/d."""
    r = k * hs / d
    return a * b * ((b + 1) * r ** b - (a + 1) * r ** a) / ((a - b) * d * d)


def phi0(k, d, hs, a=9, b=3):
    r = k * hs / d
    return (a * r ** b - b * r ** a) / (a - b)


def jump_operator(film, hbar, lam):
    """Linear map delta h -> delta Delta (pressure jumps) about a flat stack,
    for a mode whose Laplacian symbol is -lam.  delta z = P delta h, z_0 = 0;
    the (grad z)^2 terms are second order."""
    n, hs = film["n_layers"], film["hstar"]
    Z = np.concatenate([[0.0], np.cumsum(hbar)])
    S = film["spread"]
    E = np.zeros((n, n + 1))  # acts on (dz_0, ..., dz_N)
    for i in range(1, n + 1):
        ten = film["gamma"][i - 1] + sum(S.get((i, k), 0.0) * phi0(k, Z[i + k] - Z[i], hs)
                                         for k in range(1, n - i + 1))
        E[i - 1, i] += ten * lam
        for k in range(1, n - i + 1):
            c = S.get((i, k), 0.0) * phi2(k, Z[i + k] - Z[i], hs)
            E[i - 1, i + k] -= c
            E[i - 1, i] += c
        for l in range(0, i):
            c = S.get((l, i - l), 0.0) * phi2(i - l, Z[i] - Z[l], hs)
            E[i - 1, i] += c
            E[i - 1, l] -= c
    P = np.vstack([np.zeros(n), np.tril(np.ones((n, n)))])
    return E @ P


def step_matrix_1d(film, hbar, theta):
    """One LBM step (tau = 1) about a flat film at rest, for the Fourier mode
    exp(i theta x) on one row.  Post-collision f*_k = delta_k0 h + 3 w_k c_k Q
    with Q = q + F, F = -h grad p + K q; streaming gives
    h' = h - i sin(theta) Q and q' = cos(theta) Q."""
    n = film["n_layers"]
    lam = 4 * math.sin(theta / 2) ** 2
    J = jump_operator(film, hbar, lam)
    U = np.triu(np.ones((n, n)))  # p_i = sum_{j >= i} Delta_j
    K = np.stack([exact_friction_global(hbar, film["mu"], np.eye(n)[j]) for j in range(n)], 1)
    g = 1j * math.sin(theta)
    Qh = -np.diag(hbar) @ (g * (U @ J))          # dQ / dh
    Qq = np.eye(n) + K                           # dQ / dq
    top = np.hstack([np.eye(n) - g * Qh, -g * Qq])
    bot = np.hstack([math.cos(theta) * Qh, math.cos(theta) * Qq])
    return np.vstack([top, bot])


@pytest.mark.parametrize("lat", [0, 1])
def test_exact_discrete_linearisation(oracle_mod, lat):
    """At tiny amplitude every Fourier mode of the oracle follows the product
    of the per-mode linear step matrices (2N x 2N) derived from the scheme."""
    nx, steps = 128, 3000
    film = inputs.film_params(2, nx, 1, gamma=[0.01, 0.01], mu=[0.01, 0.01], hstar=0.3,
                              spread={(0, 1): 0.0, (1, 1): inputs.young_spreading(0.01, 20.0),
                                      (0, 2): -1e-4})
    hbar = np.array([1.0, 1.0])
    amp = 1e-7
    h0 = inputs.initial_heights(film, hbar, "multimode", seed=11, amp=amp, modes=40)
    o = oracle_mod.Oracle(film, lat)
    o.init(h0)
    o.step(steps)
    h, ux, _ = o.read()
    got_h = np.fft.fft(h[:, 0, :] - hbar[:, None], axis=1)
    got_q = np.fft.fft(h[:, 0, :] * ux[:, 0, :], axis=1)
    init_h = np.fft.fft(h0[:, 0, :] - hbar[:, None], axis=1)
    ref = np.abs(init_h).max()
    for m in range(1, nx // 2):
        A = step_matrix_1d(film, hbar, 2 * math.pi * m / nx)
        v = np.concatenate([init_h[:, m], np.zeros(2)])
        v = np.linalg.matrix_power(A, steps) @ v
        assert np.abs(got_h[:, m] - v[:2]).max() <= 2e-6 * ref + 2e-6 * np.abs(v[:2]).max(), m
        assert np.abs(got_q[:, m] - v[2:]).max() <= 2e-6 * ref * 1e-2 + 2e-6 * np.abs(v[2:]).max(), m
