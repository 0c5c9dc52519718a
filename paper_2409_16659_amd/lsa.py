"""Linear stability of a flat N-layer film (host tool; no GPU needed).

Linearising the N-layer thin-film equation (Sec. III) about flat layers of
thicknesses hbar, a Fourier mode exp(i q x) of the thickness perturbation
evolves as d h^/dt = A(q) h^ with A = -q^2 M E:

* E is the Jacobian of the layer pressures Delta_i (Eq. pressure) with
  respect to the thicknesses: the Laplace terms give
  (gamma_i + sum_k S_ik phi_k(Z_{i+k} - Z_i)) q^2 on the interface z_i, the
  wetting terms S_lk phi_k'' on the difference of the two interfaces they
  couple; interfaces are prefix sums of the thicknesses (z = P h, P lower
  triangular ones).
* M is the mobility, q = -M grad(Delta): the friction balances the pressure
  force layer by layer, K q = T grad(Delta), with K the friction matrix of
  the velocity profiles (Eqs. no_slip .. friction_force, slip lengths
  included) and T_ij = hbar_i for j >= i (p_i = sum_{j >= i} Delta_j), so
  M = -K^-1 T.  K comes from the library's host routine, the one that also
  checks the explicit-friction stability.

For N = 2 this is the printed two-layer analysis (Sec. IV.A).  Without
slip the eigenvalues are real: P M is symmetric positive definite and E P^-1
is symmetric (the Hessian of the free energy in interface coordinates).

The lattice Boltzmann step solves this equation only when friction
dominates.  The "lattice" model keeps what the tau-scheme adds at linear
order: the flux has inertia (each step adds the force to the layer's flux,
d q/dt = F) and the populations' non-equilibrium part gives the flux of a
longitudinal mode a viscous damping (tau - 1/2) q^2 (the second moment of
the shallow-water equilibrium without gravity carries no pressure, so the
damping comes from the third lattice moment alone).  For a mode with
thicknesses h^ cos(q x) and fluxes w sin(q x) the state (h^, w) obeys

    d/dt [h^; w] = [[0, -q I], [q T E, K - (tau - 1/2) q^2 I]] [h^; w],

whose slow eigenvalues tend to those of -q^2 M E as friction grows.
"""
import math

import numpy as np

from . import mlfilm


def phi_derivatives(k, d, hstar, a=9, b=3):
    """phi_k(d), phi_k'(d), phi_k''(d) of the wetting function
    phi_k(d) = (a r^b - b r^a) / (a - b), r = k h* / d."""
    r = k * hstar / d
    phi = (a * r ** b - b * r ** a) / (a - b)
    d1 = a * b * (r ** a - r ** b) / ((a - b) * d)
    d2 = a * b * ((b + 1) * r ** b - (a + 1) * r ** a) / ((a - b) * d * d)
    return phi, d1, d2


def _spread(film, l, k):
    return float(film["spread"].get((l, k), 0.0))


def pressure_jacobian(film, hbar, q):
    """E[i][j] = d Delta_i / d h_j at the flat state, for wavenumber q."""
    n = int(film["n_layers"])
    hs, a, b = float(film["hstar"]), int(film.get("exp_a", 9)), int(film.get("exp_b", 3))
    gam = [float(g) for g in film["gamma"]]
    Z = np.concatenate([[0.0], np.cumsum(hbar)])      # Z_0 = 0 (substrate) .. Z_N
    Ez = np.zeros((n, n + 1))                         # d Delta_i / d z_j, j = 0..N
    for i in range(1, n + 1):
        lap = gam[i - 1]
        for k in range(1, n - i + 1):                 # pairs (i, k) above z_i
            S = _spread(film, i, k)
            phi, _, d2 = phi_derivatives(k, Z[i + k] - Z[i], hs, a, b)
            lap += S * phi
            Ez[i - 1, i + k] -= S * d2
            Ez[i - 1, i] += S * d2
        Ez[i - 1, i] += lap * q * q
        for l in range(i):                            # pairs (l, i - l) below z_i
            S = _spread(film, l, i - l)
            _, _, d2 = phi_derivatives(i - l, Z[i] - Z[l], hs, a, b)
            Ez[i - 1, i] += S * d2
            Ez[i - 1, l] -= S * d2
    P = np.tril(np.ones((n, n)))                      # z_j = sum_{m <= j} h_m
    return Ez[:, 1:] @ P                              # z_0 is fixed


def mobility(film, hbar):
    """M = -K^-1 T (flux = -M grad Delta) at thicknesses hbar."""
    n = int(film["n_layers"])
    T = np.triu(np.ones((n, n))) * np.asarray(hbar, dtype=np.float64)[:, None]
    return -np.linalg.solve(friction(film, hbar), T)


def friction(film, hbar):
    """Friction matrix K (friction = K q) of the flat film, slip included."""
    n = int(film["n_layers"])
    slip = film.get("slip")
    K, _ = mlfilm.friction_matrix(hbar, film["mu"][:n], None if slip is None or not any(slip) else slip[:n])
    return K


def growth_matrix(film, hbar, q, model="lubrication"):
    """A(q) = -q^2 M E (N x N, state h^) for the thin-film equation, or the
    2N x 2N matrix of the lattice model (state (h^, w))."""
    E = pressure_jacobian(film, hbar, q)
    if model == "lubrication":
        return -q * q * mobility(film, hbar) @ E
    if model != "lattice":
        raise ValueError(f"unknown model {model!r}")
    n = int(film["n_layers"])
    T = np.triu(np.ones((n, n))) * np.asarray(hbar, dtype=np.float64)[:, None]
    damp = (float(film.get("tau", 1.0)) - 0.5) * q * q
    return np.block([[np.zeros((n, n)), -q * np.eye(n)],
                     [q * T @ E, friction(film, hbar) - damp * np.eye(n)]])


def growth_rates(film, hbar, q, model="lubrication"):
    """Eigenvalues of the growth matrix, largest real part first."""
    ev = np.linalg.eigvals(growth_matrix(film, hbar, q, model))
    return ev[np.argsort(-ev.real)]


def leading_mode(film, hbar, q, model="lubrication"):
    """(rate, dh, flux) of the fastest eigenmode: thickness amplitudes dh
    [N] (largest magnitude 1) and, for the lattice model, the flux
    amplitudes w [N] (flux w_i sin(q x) with thickness dh_i cos(q x))
    (zeros for the lubrication model, where the flux follows the heights)."""
    n = int(film["n_layers"])
    ev, V = np.linalg.eig(growth_matrix(film, hbar, q, model))
    j = int(np.argmax(ev.real))
    v = V[:, j].real
    v = v / v[np.argmax(np.abs(v[:n]))]
    w = v[n:] if model == "lattice" else np.zeros(n)
    return float(ev[j].real), v[:n], w


def mode_rates(film, hbar, length, model="lubrication"):
    """Largest growth rate of each periodic mode m = 1 .. length // 2 of a
    box of the given length (lattice units): array [m - 1]."""
    return np.array([growth_rates(film, hbar, 2 * math.pi * m / length, model)[0].real
                     for m in range(1, length // 2 + 1)])


def fastest_mode(film, hbar, length, model="lubrication"):
    """(m, rate) of the fastest-growing periodic mode, and the number of
    unstable modes."""
    eta = mode_rates(film, hbar, length, model)
    m = int(np.argmax(eta))
    return m + 1, float(eta[m]), int((eta > 0).sum())
