"""Pins of the oracle's pressure assembly and friction solve.

Pressure: against the explicit one-, two- and three-layer pressures the
paper prints (tests/golden/pressure_*.txt) evaluated with independently
written stencils, and against the free-energy variation for flat films.
Friction: against the closed forms for one layer, the paper's two-layer
mobility and its symmetric Pototsky form (tests/golden/mobility_2layer.txt),
and an exact rational solve of the boundary-condition system in the paper's
global coordinates for N = 1..4, with and without slip lengths.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests._golden import evaluate, read_forms


# Stencils written out in coefficient form (the isotropic 9-point lattice
# stencils, equal to the definition used by the oracle).
def _sh(f, dx, dy):
    return np.roll(np.roll(f, -dx, axis=1), -dy, axis=0)  # f(x + dx, y + dy)


def grad9(f):
    e, w, n, s = _sh(f, 1, 0), _sh(f, -1, 0), _sh(f, 0, 1), _sh(f, 0, -1)
    ne, nw, sw, se = _sh(f, 1, 1), _sh(f, -1, 1), _sh(f, -1, -1), _sh(f, 1, -1)
    gx = (e - w) / 3.0 + (ne + se - nw - sw) / 12.0
    gy = (n - s) / 3.0 + (ne + nw - se - sw) / 12.0
    return gx, gy


def lap9(f):
    e, w, n, s = _sh(f, 1, 0), _sh(f, -1, 0), _sh(f, 0, 1), _sh(f, 0, -1)
    ne, nw, sw, se = _sh(f, 1, 1), _sh(f, -1, 1), _sh(f, -1, -1), _sh(f, 1, -1)
    return (4.0 * (e + w + n + s) + (ne + nw + sw + se) - 20.0 * f) / 6.0


def smooth_heights(n, nx, ny, hbar, amp, seed):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    h = np.empty((n, ny, nx))
    for i in range(n):
        v = np.zeros((ny, nx))
        for _ in range(4):
            mx, my = rng.integers(0, 3, size=2)
            v += rng.normal() * np.cos(2 * np.pi * (mx * x / nx + my * y / ny) + rng.uniform(0, 6.3))
        h[i] = hbar[i] + amp * v
    return h


def film_for(n, seed, hstar=0.2):
    rng = np.random.default_rng(seed)
    spread = {(l, k): rng.uniform(-0.02, 0.02) for l in range(n) for k in range(1, n - l + 1)}
    return {
        "n_layers": n, "nx": 16, "ny": 12, "tau": 1.0, "hstar": hstar, "exp_a": 9, "exp_b": 3,
        "gamma": list(rng.uniform(0.5e-2, 2e-2, size=n)), "mu": [0.01] * n, "slip": [0.0] * n,
        "spread": spread,
    }


@pytest.mark.parametrize("n,golden", [(1, "pressure_1layer.txt"), (2, "pressure_2layer.txt"),
                                      (3, "pressure_3layer.txt")])
def test_pressure_matches_printed_forms(oracle_mod, n, golden):
    film = film_for(n, 100 + n)
    hbar = [0.9, 0.5, 0.35][:n]
    h = smooth_heights(n, film["nx"], film["ny"], hbar, 0.05, 200 + n)
    _, jump = oracle_mod.pressure(film, h)
    z = np.cumsum(h, axis=0)
    ns = {"h%d" % (i + 1): h[i] for i in range(n)}
    for i in range(n):
        gx, gy = grad9(z[i])
        ns["z%d" % (i + 1)] = z[i]
        ns["lapz%d" % (i + 1)] = lap9(z[i])
        ns["gz%dsq" % (i + 1)] = gx * gx + gy * gy
    ns["gz0sq"] = 0.0
    names = {1: ["g12"], 2: ["g12", "g2v"], 3: ["g12", "g23", "g3v"]}[n]
    for i, nm in enumerate(names):
        ns[nm] = film["gamma"][i]
    S = film["spread"]
    vphi = np.vectorize(lambda k, d: oracle_mod.phi(k, d, film["hstar"]))
    vdphi = np.vectorize(lambda k, d: oracle_mod.dphi(k, d, film["hstar"]))
    ns["phi"] = lambda l, k, d: S[(l, k)] * vphi(k, d)
    ns["dphi"] = lambda l, k, d: S[(l, k)] * vdphi(k, d)
    forms = read_forms(golden)
    assert len(forms) == n
    for i, (_, rhs) in enumerate(forms):
        want = evaluate(rhs, ns)
        scale = np.abs(want).max()
        assert np.abs(jump[i] - want).max() <= 1e-13 * scale, (i, rhs)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_flat_film_jumps_are_energy_derivatives(oracle_mod, n):
    """For a flat stack only the wetting energy sum_{l,k} S_lk phi_k(z_{l+k}-z_l)
    varies, and p_i - p_{i+1} = dF/dz_i (appendix, variation of the free
    energy): checked against a central difference of that energy."""
    film = film_for(n, 300 + n, hstar=0.1)
    film["nx"], film["ny"] = 3, 2
    rng = np.random.default_rng(400 + n)
    for _ in range(5):
        hv = rng.uniform(0.12, 0.6, size=n)
        h = np.broadcast_to(hv[:, None, None], (n, 2, 3)).copy()
        pres, jump = oracle_mod.pressure(film, h)
        assert np.ptp(pres, axis=(1, 2)).max() == 0.0  # uniform: no pressure gradient

        def energy(zv):
            zz = np.concatenate([[0.0], zv])
            return sum(s * oracle_mod.phi(k, zz[l + k] - zz[l], film["hstar"])
                       for (l, k), s in film["spread"].items())

        zv = np.cumsum(hv)
        for i in range(n):
            e = 1e-6
            zp, zm = zv.copy(), zv.copy()
            zp[i] += e
            zm[i] -= e
            fd = (energy(zp) - energy(zm)) / (2 * e)
            assert abs(jump[i, 0, 0] - fd) <= 1e-7 * max(1e-3, abs(fd))
        # p_i = sum_{j >= i} Delta_j
        assert np.allclose(pres[:, 0, 0], np.cumsum(jump[::-1, 0, 0])[::-1], rtol=0, atol=1e-17)


def test_single_layer_capillary_symbol(oracle_mod):
    """S = 0, one layer: p = -gamma lap h, so a cosine of wavenumber theta has
    pressure gamma 4 sin^2(theta/2) times its amplitude."""
    film = film_for(1, 7)
    film["spread"] = {(0, 1): 0.0}
    nx = film["nx"]
    x = np.arange(nx)
    for m in range(0, nx // 2 + 1):
        th = 2 * np.pi * m / nx
        h = (1.0 + 1e-3 * np.cos(th * x))[None, None, :].repeat(film["ny"], 1)
        pres, _ = oracle_mod.pressure(film, h)
        want = film["gamma"][0] * 4 * np.sin(th / 2) ** 2 * 1e-3 * np.cos(th * x)
        assert np.abs(pres[0] - want[None, :]).max() < 1e-17 + 1e-12 * np.abs(want).max()


# ------------------------------------------------------------- friction ----
def exact_friction_global(h, mu, q, slip=None):
    """Solve the boundary-condition system of Sec. II.A.2 exactly (rational
    arithmetic) in the paper's global vertical coordinate z, with
    u_i = a_i z^2 + b_i z + c_i: Eq. (no_slip) as printed,
    u_i(z_{i-1} - beta_i) = u_{i-1}(z_{i-1}) with u_0 = 0 (beta = 0: no slip
    at the substrate and continuity of velocity at every interface),
    continuity of stress at every interface, the flux constraint in every
    layer and no stress at the gas; returns 2 mu_i h_i a_i."""
    n = len(h)
    H = [Fraction(float(v)) for v in h]
    M = [Fraction(float(v)) for v in mu]
    Q = [Fraction(float(v)) for v in q]
    B = [Fraction(float(v)) for v in (slip if slip is not None else [0.0] * n)]
    z = [Fraction(0)]
    for v in H:
        z.append(z[-1] + v)
    m = 3 * n
    A = [[Fraction(0)] * (m + 1) for _ in range(m)]
    r = 0
    # u_1(z_0 - beta_1) = u_1(-beta_1) = 0
    A[r][0] = B[0] ** 2; A[r][1] = -B[0]; A[r][2] = Fraction(1); r += 1
    for i in range(n):
        lo, hi = z[i], z[i + 1]
        a, b, c = 3 * i, 3 * i + 1, 3 * i + 2
        # integral of u_i over [z_{i-1}, z_i] equals q_i
        A[r][a] = (hi ** 3 - lo ** 3) / 3
        A[r][b] = (hi ** 2 - lo ** 2) / 2
        A[r][c] = hi - lo
        A[r][m] = Q[i]; r += 1
        if i + 1 < n:
            # mu_i u_i'(z_i) = mu_{i+1} u_{i+1}'(z_i)
            A[r][a] = 2 * M[i] * hi; A[r][b] = M[i]
            A[r][a + 3] = -2 * M[i + 1] * hi; A[r][b + 3] = -M[i + 1]; r += 1
            # u_{i+1}(z_i - beta_{i+1}) = u_i(z_i)
            zs = hi - B[i + 1]
            A[r][a] = -hi ** 2; A[r][b] = -hi; A[r][c] = Fraction(-1)
            A[r][a + 3] = zs ** 2; A[r][b + 3] = zs; A[r][c + 3] = Fraction(1); r += 1
        else:
            # u_N'(z_N) = 0 (mu_{N+1} = 0)
            A[r][a] = 2 * hi; A[r][b] = Fraction(1); r += 1
    assert r == m
    for col in range(m):  # exact Gauss-Jordan
        piv = next(rr for rr in range(col, m) if A[rr][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        inv = 1 / A[col][col]
        A[col] = [v * inv for v in A[col]]
        for rr in range(m):
            if rr != col and A[rr][col] != 0:
                f = A[rr][col]
                A[rr] = [x - f * y for x, y in zip(A[rr], A[col])]
    return np.array([float(2 * M[i] * H[i] * A[3 * i][m]) for i in range(n)])


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_friction_exact_rational(oracle_mod, n):
    rng = np.random.default_rng(500 + n)
    for _ in range(20):
        h = rng.uniform(0.1, 3.0, size=n)
        mu = 10 ** rng.uniform(-4, -2, size=n)
        q = rng.normal(size=n) * 1e-3
        got = oracle_mod.friction(h, mu, q)
        want = exact_friction_global(h, mu, q)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_friction_exact_rational_slip(oracle_mod, n):
    """Slip lengths at the substrate and at every liquid-liquid interface
    (Eq. no_slip with beta_i > 0), against the exact solve of the printed
    global-coordinate conditions; slip only at the substrate, only at an
    upper interface, and everywhere."""
    rng = np.random.default_rng(520 + n)
    for trial in range(24):
        h = rng.uniform(0.1, 3.0, size=n)
        mu = 10 ** rng.uniform(-4, -2, size=n)
        q = rng.normal(size=n) * 1e-3
        slip = rng.uniform(0.0, 1.5, size=n)
        if trial % 3 == 0:
            slip[1:] = 0.0
        elif trial % 3 == 1 and n > 1:
            slip[:] = 0.0
            slip[rng.integers(1, n)] = rng.uniform(0.05, 1.5)
        got = oracle_mod.friction(h, mu, q, slip=slip)
        want = exact_friction_global(h, mu, q, slip)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), (slip, got, want)


def test_friction_slip_limits(oracle_mod):
    """Two layers: a slip length at the liquid-liquid interface lowers the
    friction's magnitude on a lone moving top layer (the layer below resists
    less), and beta -> 0 recovers the no-slip solve continuously."""
    h, mu, q = np.array([0.8, 0.5]), np.array([2e-3, 3e-3]), np.array([0.0, 1e-3])
    f0 = oracle_mod.friction(h, mu, q)
    prev = abs(f0[1])
    for be in (1e-3, 0.1, 0.5, 2.0):
        f = oracle_mod.friction(h, mu, q, slip=[0.0, be])
        assert abs(f[1]) < prev
        prev = abs(f[1])
    f_small = oracle_mod.friction(h, mu, q, slip=[0.0, 1e-12])
    assert np.abs(f_small - f0).max() <= 1e-9 * np.abs(f0).max()


def test_friction_single_layer_closed_form(oracle_mod):
    """One layer, no slip: a Poiseuille half-profile gives -3 mu q / h^2
    (the mobility h^3/(3 mu) of the single-layer TFE)."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        h, mu, q = rng.uniform(0.05, 5), 10 ** rng.uniform(-4, 0), rng.normal()
        fr = oracle_mod.friction([h], [mu], [q])[0]
        assert abs(fr - (-3 * mu * q / h ** 2)) <= 1e-14 * abs(fr)


def test_friction_single_layer_slip(oracle_mod):
    """Slip condition of Eq. (no_slip), u(-beta) = 0 for one layer: the
    profile u = a s^2 + b s + c with u'(h) = 0 and flux q gives
    2 mu h a = -3 mu q / (h^2 + 3 beta h + 3 beta^2 / 2)."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        h, mu, q, be = rng.uniform(0.1, 3), 10 ** rng.uniform(-4, -1), rng.normal(), rng.uniform(0, 1)
        fr = oracle_mod.friction([h], [mu], [q], slip=[be])[0]
        want = -3 * mu * q / (h * h + 3 * be * h + 1.5 * be * be)
        assert abs(fr - want) <= 1e-13 * abs(want)


def mobility(oracle_mod, h, mu):
    """M = -K^{-1} T with friction = K q and T_ij = h_i (j >= i): the mobility
    of Eq. (thin_film_equation_n) with mass flowing down the pressure
    gradient, from the Stokes balance of Eq. (thin_sheet_matrix_2)."""
    n = len(h)
    K = np.stack([oracle_mod.friction(h, mu, np.eye(n)[j]) for j in range(n)], axis=1)
    T = np.triu(np.tile(np.asarray(h)[:, None], (1, n)))
    return -np.linalg.solve(K, T)


def test_two_layer_mobility_printed(oracle_mod):
    forms = dict(read_forms("mobility_2layer.txt"))
    rng = np.random.default_rng(8)
    for _ in range(20):
        h = rng.uniform(0.1, 3.0, size=2)
        mu = 10 ** rng.uniform(-3, -1, size=2)
        M = mobility(oracle_mod, h, mu)
        ns = {"z1": h[0], "z2": h[0] + h[1], "mu1": mu[0], "mu2": mu[1]}
        want = np.array([[evaluate(forms["M11"], ns), evaluate(forms["M12"], ns)],
                         [evaluate(forms["M21"], ns), evaluate(forms["M22"], ns)]])
        assert np.abs(M - want).max() <= 1e-12 * np.abs(want).max()
        Mt = np.array([[1, 0], [1, 1]]) @ M
        want_t = np.array([[evaluate(forms["Mt11"], ns), evaluate(forms["Mt12"], ns)],
                           [evaluate(forms["Mt21"], ns), evaluate(forms["Mt22"], ns)]])
        assert np.abs(Mt - want_t).max() <= 1e-12 * np.abs(want_t).max()
    M1 = mobility(oracle_mod, [0.7], [0.02])
    assert abs(M1[0, 0] - evaluate(forms["M1"], {"z1": 0.7, "mu1": 0.02})) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4])
def test_mobility_onsager_symmetry(oracle_mod, n):
    """In interface variables the mobility P M (P lower-triangular ones) is
    symmetric positive definite for every N (Onsager reciprocity, Sec. II.B)."""
    rng = np.random.default_rng(900 + n)
    P = np.tril(np.ones((n, n)))
    for _ in range(20):
        h = rng.uniform(0.1, 3.0, size=n)
        mu = 10 ** rng.uniform(-3, -1, size=n)
        Mz = P @ mobility(oracle_mod, h, mu)
        assert np.abs(Mz - Mz.T).max() <= 1e-12 * np.abs(Mz).max()
        assert np.linalg.eigvalsh(0.5 * (Mz + Mz.T)).min() > 0
