"""Pins of the oracle's building blocks against what the paper and the
mathematics fix: lattice moments, equilibrium/forcing moments, stencil
exactness and Fourier symbols, wetting-potential identities, and the
spreading coefficients' free-energy bookkeeping."""
import itertools
import math

import numpy as np
import pytest

from tests._golden import evaluate, read_forms

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("lat", [0, 1])
def test_lattice_isotropy(oracle_mod, lat):
    """Weights and velocities reproduce the lattice tensors through 4th order
    (what the shallow-water Chapman-Enskog result of Sec. III relies on)."""
    cx, cy, w = oracle_mod.lattice(lat)
    c = np.stack([cx, cy], 1).astype(float)
    dim = 1 if lat == 1 else 2
    c = c[:, :dim]
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("k,ka->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("k,ka,kb->ab", w, c, c), CS2 * np.eye(dim), atol=1e-16)
    assert np.allclose(np.einsum("k,ka,kb,kc->abc", w, c, c, c), 0, atol=1e-16)
    d = np.eye(dim)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    if lat == 0:  # D1Q3 is not 4th-order isotropic (c^4 = c^2); D2Q9 is
        assert np.allclose(np.einsum("k,ka,kb,kc,kd->abcd", w, c, c, c, c), iso, atol=1e-16)
    # every velocity has its opposite (streaming is a permutation)
    pairs = {(int(a), int(b)) for a, b in zip(cx, cy)}
    assert all((-a, -b) in pairs for a, b in pairs)
    if lat == 0:
        # counter-clockwise from east, rest first (Sec. III, D2Q9 list)
        ang = [math.atan2(b, a) % (2 * math.pi) for a, b in zip(cx[1:], cy[1:])]
        assert ang == sorted(ang) and ang[0] == 0.0
        assert np.allclose(w, [4 / 9] + [1 / 9, 1 / 36] * 4)


@pytest.mark.parametrize("lat", [0, 1])
def test_equilibrium_moments(oracle_mod, lat):
    """sum f^eq = h, sum c f^eq = hU, sum c c f^eq = h U U: mass, momentum and
    the momentum flux of the shallow-water equations without a hydrostatic
    term (Sec. III, Eqs. shallow_water_1/2)."""
    cx, cy, w = oracle_mod.lattice(lat)
    rng = np.random.default_rng(0)
    for _ in range(50):
        h = rng.uniform(0.1, 3.0)
        ux = rng.uniform(-0.1, 0.1)
        uy = 0.0 if lat == 1 else rng.uniform(-0.1, 0.1)
        f = oracle_mod.equilibrium(h, ux, uy, lat)
        assert abs(f.sum() - h) <= 4e-16 * h * 4
        assert abs((cx * f).sum() - h * ux) <= 1e-15 * h
        assert abs((cy * f).sum() - h * uy) <= 1e-15 * h
        assert abs((cx * cx * f).sum() - h * ux * ux) <= 1e-15 * h
        assert abs((cx * cy * f).sum() - h * ux * uy) <= 1e-15 * h
        assert abs((cy * cy * f).sum() - h * uy * uy) <= 1e-15 * h
    # at rest everything sits in the rest population
    f = oracle_mod.equilibrium(1.7, 0.0, 0.0, lat)
    assert f[0] == 1.7 and np.all(f[1:] == 0)


@pytest.mark.parametrize("lat", [0, 1])
def test_forcing_moments(oracle_mod, lat):
    """The forcing adds no mass and exactly F to the momentum (Eq. BGK with
    c_s^2 = 1/3; first moment F as the shallow-water equations require)."""
    cx, cy, _ = oracle_mod.lattice(lat)
    rng = np.random.default_rng(1)
    for _ in range(50):
        fx, fy = rng.normal(size=2) * 1e-3
        if lat == 1:
            fy = 0.0
        g = oracle_mod.forcing(fx, fy, lat)
        tol = 4e-16 * (abs(fx) + abs(fy))
        assert abs(g.sum()) <= tol
        assert abs((cx * g).sum() - fx) <= tol
        assert abs((cy * g).sum() - fy) <= tol


def _poly(nx, ny, coef):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c, d, e, g = coef
    f = a + b * x + c * y + d * x * x + e * x * y + g * y * y
    return f, (b + 2 * d * x + e * y, c + e * x + 2 * g * y, 2 * d + 2 * g)


def test_stencils_exact_on_quadratics(oracle_mod):
    rng = np.random.default_rng(2)
    for _ in range(5):
        coef = rng.normal(size=6)
        f, (fx, fy, lap) = _poly(12, 10, coef)
        gx, gy = oracle_mod.grad(f)
        lp = oracle_mod.lap(f)
        inner = (slice(1, -1), slice(1, -1))  # away from the periodic seam
        scale = np.abs(f).max()
        assert np.abs(gx - fx)[inner].max() < 1e-13 * scale
        assert np.abs(gy - fy)[inner].max() < 1e-13 * scale
        assert np.abs(lp - lap)[inner].max() < 1e-13 * scale


@pytest.mark.parametrize("axis", [0, 1])
def test_stencil_fourier_symbols(oracle_mod, axis):
    """Along a lattice axis the gradient has symbol i sin(theta) and the
    Laplacian -4 sin^2(theta/2) (the 3-point central differences)."""
    n = 24
    for m in range(0, n // 2 + 1):
        th = 2 * math.pi * m / n
        s = np.arange(n)
        prof = np.cos(th * s + 0.3)
        f = np.tile(prof, (n, 1)) if axis == 1 else np.tile(prof[:, None], (1, n))
        gx, gy = oracle_mod.grad(f)
        g = gx if axis == 1 else gy
        want_g = -math.sin(th) * np.sin(th * s + 0.3)
        want_g = np.tile(want_g, (n, 1)) if axis == 1 else np.tile(want_g[:, None], (1, n))
        assert np.abs(g - want_g).max() < 1e-14
        want_l = -4 * math.sin(th / 2) ** 2 * f
        assert np.abs(oracle_mod.lap(f) - want_l).max() < 1e-14


def test_d2q9_single_row_equals_d1q3_stencils(oracle_mod):
    rng = np.random.default_rng(3)
    f = rng.normal(size=(1, 37))
    g9, gy = oracle_mod.grad(f, 0)
    g3, _ = oracle_mod.grad(f, 1)
    assert np.abs(g9 - g3).max() < 1e-15
    assert np.abs(gy).max() < 1e-15 * np.abs(f).max()  # rounding of the cancelling sum
    assert np.abs(oracle_mod.lap(f, 0) - oracle_mod.lap(f, 1)).max() < 1e-14


# -------------------------------------------------------------- wetting ----
EXPS = [(9, 3), (3, 2), (8, 2), (4, 3)]


@pytest.mark.parametrize("a,b", EXPS)
def test_wetting_potential_identities(oracle_mod, a, b):
    """phi_k(k h*) = 1 and phi'_k(k h*) = 0 (appendix limit z2 -> z1 + h*;
    Sec. II.A.3: phi' vanishes at k h* and decreases there), phi -> 0 for
    thick films, and phi' is the derivative of phi."""
    hs = 0.15
    for k in range(1, 5):
        d0 = k * hs
        assert abs(oracle_mod.phi(k, d0, hs, a, b) - 1.0) < 1e-15
        assert abs(oracle_mod.dphi(k, d0, hs, a, b)) < 1e-14
        assert abs(oracle_mod.phi(k, 1e5 * d0, hs, a, b)) < 1e-9
        assert abs(oracle_mod.dphi(k, 1e5 * d0, hs, a, b)) < 1e-12
        # monotone decreasing derivative around k h*
        e = 1e-3 * d0
        assert oracle_mod.dphi(k, d0 - e, hs, a, b) > 0 > oracle_mod.dphi(k, d0 + e, hs, a, b)
        for d in np.linspace(0.6 * d0, 8 * d0, 23):
            e = 1e-5 * d
            fd = (oracle_mod.phi(k, d + e, hs, a, b) - oracle_mod.phi(k, d - e, hs, a, b)) / (2 * e)
            an = oracle_mod.dphi(k, d, hs, a, b)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_wetting_potential_is_lennard_jones_like(oracle_mod):
    """phi_k(h) = 1 at the precursor thickness, decays as h^-b for thick films
    (the leading van-der-Waals-like power of Eq. wetting_potential)."""
    a, b, hs = 9, 3, 0.1
    d = np.array([10.0, 20.0, 40.0])
    v = np.array([oracle_mod.phi(1, x, hs, a, b) for x in d])
    slope = np.diff(np.log(v)) / np.diff(np.log(d))
    assert np.allclose(slope, -b, atol=1e-5)


def _tension_table(n, rng):
    g = np.zeros((n + 2, n + 2))
    for i in range(n + 2):
        for j in range(i + 1, n + 2):
            g[i, j] = g[j, i] = rng.uniform(0.5, 2.0)
    return g


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_spreading_coefficients_dewetting_bookkeeping(oracle_mod, n):
    """When a block of consecutive layers m..m+j-1 dewets (each at h*), every
    pair (l, k) spanning only dewetted layers has phi_k = 1 and all others
    vanish for thick films, so the flat free energy (appendix, Eq.
    free_energy_n_layer) sum_i gamma_{i,i+1} + sum S_lk must become that of the
    stack without those layers: the interfaces m-1..m+j-1 are replaced by the
    single interface (m-1, m+j)."""
    rng = np.random.default_rng(10 + n)
    for _ in range(10):
        g = _tension_table(n, rng)
        S = oracle_mod.spreading_from_tensions(n, g)
        base = sum(g[i, i + 1] for i in range(n + 1))
        for m in range(1, n + 1):
            for j in range(1, n - m + 2):
                block = set(range(m, m + j))
                e = base
                for (l, k), s in S.items():
                    if set(range(l + 1, l + k + 1)) <= block:
                        e += s
                want = base - sum(g[i, i + 1] for i in range(m - 1, m + j)) + g[m - 1, m + j]
                assert abs(e - want) < 1e-13


def test_spreading_coefficients_printed_limits(oracle_mod):
    """The tension combinations printed in the two-layer limit cases."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        g = _tension_table(2, rng)
        S = oracle_mod.spreading_from_tensions(2, g)
        ns = {f"g{i}{j}": g[i, j] for i, j in itertools.combinations(range(4), 2)}
        ns.update({f"S{l}{k}": v for (l, k), v in S.items()})
        for lhs, rhs in read_forms("spreading_limits_2layer.txt"):
            assert abs(evaluate(lhs, ns) - evaluate(rhs, ns)) < 1e-14, (lhs, rhs)
        # single layer: S = gamma_sv - gamma_sl - gamma
        g1 = _tension_table(1, rng)
        S1 = oracle_mod.spreading_from_tensions(1, g1)
        assert abs(S1[(0, 1)] - (g1[0, 2] - g1[0, 1] - g1[1, 2])) < 1e-15
