"""Equilibrium contact angles of the oracle against Young's and Neumann's laws
(Sec. IV.B), measured as the paper does: fit a circular arc that shares the
drop's peak position and height by minimising the volume error
E(theta) = int |h - H_theta| / int h, and report E at the expected angle.

The paper states best-fit errors below 2 %, errors at the expected angle
below 15 % (often below 6 %), and some contact-line pinning ("numerical
hysteresis") when starting away from the expected angle.  Pseudo-1D films
(D1Q3) with a precursor of half a lattice unit so that the contact-line
region spans several nodes.
"""
import math

import numpy as np
import pytest

from paper_2409_16659_amd import inputs

pytestmark = pytest.mark.slow


def cap(x, x0, base_half_width, theta):
    """Circular cap of the given base half-width and contact angle."""
    rho = base_half_width / math.sin(theta)
    top = rho * (1 - math.cos(theta))
    return np.maximum(np.sqrt(np.maximum(rho ** 2 - (x - x0) ** 2, 0.0)) - (rho - top), 0.0)


def arc_fit(d):
    """Contact angle (degrees) of the best arc through the peak of the
    non-negative profile d, the best-fit error, and E(theta) itself."""
    x = np.arange(len(d), dtype=float)
    xp = int(np.argmax(d))
    hp = d[xp]

    def err(theta):
        rho = hp / (1 - math.cos(theta))
        a = np.sqrt(np.maximum(rho ** 2 - (x - xp) ** 2, 0.0)) - (rho - hp)
        return float(np.abs(d - np.maximum(a, 0.0)).sum() / d.sum())

    th = np.radians(np.linspace(3, 45, 841))
    es = np.array([err(t) for t in th])
    i = int(np.argmin(es))
    return math.degrees(th[i]), float(es[i]), err


@pytest.fixture(scope="module", autouse=True)
def threads(oracle_mod):
    keep = oracle_mod.get_threads()
    oracle_mod.set_threads(min(4, keep))
    yield
    oracle_mod.set_threads(keep)


@pytest.mark.parametrize("theta0", [40.0, 10.0])
def test_sessile_drop_relaxes_to_young_angle(oracle_mod, theta0):
    """One layer on the substrate with S = gamma (cos theta_Y - 1) (Eq.
    youngs_law, S = gamma_sv - gamma_sl - gamma): a drop started at twice or
    half the Young angle relaxes to it."""
    theta_y, nx, hs, g = 20.0, 200, 0.5, 0.005
    film = inputs.film_params(1, nx, 1, gamma=[g], mu=[0.02], hstar=hs,
                              spread={(0, 1): inputs.young_spreading(g, theta_y)})
    x = np.arange(nx) + 0.5
    h0 = (cap(x, nx / 2, 60, math.radians(theta0)) + hs)[None, None, :]
    o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    o.init(h0)
    o.step(150_000)
    h, ux, _ = o.read()
    assert np.abs(ux).max() < 1e-4  # essentially at rest
    d = h[0, 0] - np.median(np.concatenate([h[0, 0, :10], h[0, 0, -10:]]))
    theta, e_best, err = arc_fit(d)
    assert abs(theta - theta_y) <= 0.05 * theta_y, theta
    assert e_best < 0.02
    assert err(math.radians(theta_y)) < 0.06


@pytest.mark.parametrize("theta0", [20.0, 12.0])
def test_liquid_lens_neumann_angles(oracle_mod, theta0):
    """A symmetric lens of liquid 2 (gamma_12 = gamma_23 = gamma) on a bath of
    liquid 1 under gas: Neumann's law (Eq. neumanns_law) gives equal top and
    bottom angles with 2 gamma cos(theta) = gamma_13, i.e. the spreading
    coefficient S_11 = gamma_13 - 2 gamma = 2 gamma (cos theta - 1)."""
    theta_n, nx, hs, g, bath = 20.0, 256, 0.5, 0.004, 20.0
    s11 = 2 * g * (math.cos(math.radians(theta_n)) - 1)
    film = inputs.film_params(2, nx, 1, gamma=[g, g], mu=[0.05, 0.05], hstar=hs,
                              spread={(0, 1): 0.0, (1, 1): s11, (0, 2): 0.0})
    x = np.arange(nx) + 0.5
    a = cap(x, nx / 2, 60, math.radians(theta0))
    z1 = bath - a
    z2 = bath + a + hs
    o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    o.init(np.stack([z1, z2 - z1])[:, None, :])
    o.step(100_000 if theta0 == theta_n else 250_000)  # receding from below is slower
    h, _, _ = o.read()
    z1 = h[0, 0]
    z2 = z1 + h[1, 0]
    far = lambda z: np.median(np.concatenate([z[:8], z[-8:]]))  # noqa: E731
    top, e_top, err_top = arc_fit(z2 - far(z2))
    bot, e_bot, err_bot = arc_fit(far(z1) - z1)
    tol = 0.05 if theta0 == theta_n else 0.12  # started below: some pinning
    assert abs(top - theta_n) <= tol * theta_n, top
    assert abs(bot - theta_n) <= tol * theta_n, bot
    assert err_top(math.radians(theta_n)) < 0.15 and err_bot(math.radians(theta_n)) < 0.15
