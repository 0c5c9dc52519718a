"""The surrogate's restart and judge arithmetic on the GPU.

* mlf_stokes_velocity against the FP64 oracle: the velocities must make
  the total force of the step vanish, -h_i grad p_i + friction_i(h U) = 0,
  with the oracle's pressures, its friction solve and independently
  written gradient stencils; N = 1 against the closed form
  U = -h^2 d p / (3 mu); every N against a direct solve K q = h grad p with
  K built column by column from the oracle's friction.
* A judge restarted from the solver's own heights with the velocities of
  an earlier solver state follows the solver far closer than one
  restarted at rest (the Stokes-limit velocities do worse than rest).
* mlf_nop_errors against the same norms in NumPy (FP64), and
  mlf_convert_heights (FP32 <-> FP64) against NumPy's rounding.
"""
import numpy as np
import pytest

from paper_2409_16659_amd import inputs
from tests.test_oracle_pressure_friction import grad9, smooth_heights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mlf(torch_cuda):
    from paper_2409_16659_amd import mlfilm

    mlfilm.load_library()
    return mlfilm


def _film(n, nx, ny, seed):
    rng = np.random.default_rng(seed)
    gam = list(rng.uniform(0.5e-2, 1.5e-2, size=n))
    spread = {(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(n)}
    for l in range(n):
        for k in range(2, n - l + 1):
            spread[(l, k)] = rng.uniform(-2e-3, 2e-3)
    mu = list(10 ** rng.uniform(-3, -2, size=n))
    return inputs.film_params(n, nx, ny, gamma=gam, mu=mu, hstar=0.15, spread=spread)


def _stokes_gpu(mlf, torch, film, h):
    p = mlf.make_params(film, "f64")
    hd = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    ux, uy = torch.empty_like(hd), torch.empty_like(hd)
    import ctypes as C

    rc = mlf.load_library().mlf_stokes_velocity(C.byref(p), C.c_void_p(hd.data_ptr()), C.c_void_p(ux.data_ptr()),
                                                C.c_void_p(uy.data_ptr()), None)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return ux.cpu().numpy(), uy.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_stokes_velocity_balances_the_forces(mlf, torch_cuda, oracle_mod, n):
    film = _film(n, 24, 20, 40 + n)
    h = smooth_heights(n, 24, 20, [0.9, 0.7, 0.5, 0.4][:n], 0.05, 50 + n)
    ux, uy = _stokes_gpu(mlf, torch_cuda, film, h)
    pres, _ = oracle_mod.pressure(film, h)
    gpx = np.stack([grad9(pres[i])[0] for i in range(n)])
    gpy = np.stack([grad9(pres[i])[1] for i in range(n)])
    # errors relative to the field's largest driving force (the pressure
    # gradient is a difference of nearby pressures: both sides round it
    # differently at ~1e-12 of its own size)
    drive_max = max(np.abs(h * gpx).max(), np.abs(h * gpy).max())
    u_max = max(np.abs(ux).max(), np.abs(uy).max())
    worst = worst_u = 0.0
    for y in range(20):
        for x in range(24):
            hn = h[:, y, x]
            for u, gp in ((ux, gpx), (uy, gpy)):
                drive = hn * gp[:, y, x]
                fr = oracle_mod.friction(hn, film["mu"], hn * u[:, y, x])
                worst = max(worst, np.abs(fr - drive).max() / drive_max)
                if n == 1:
                    want = -hn[0] ** 2 * gp[0, y, x] / (3 * film["mu"][0])
                    worst_u = max(worst_u, abs(u[0, y, x] - want) / u_max)
    print(f"N={n}: worst |friction - h grad p| / max|h grad p| = {worst:.2e}; N = 1 closed form {worst_u:.2e}",
          flush=True)
    assert worst <= 1e-11
    assert worst_u <= 1e-11


def test_stokes_velocity_is_the_direct_solve(mlf, torch_cuda, oracle_mod):
    n = 3
    film = _film(n, 16, 12, 61)
    h = smooth_heights(n, 16, 12, [1.0, 0.8, 0.6], 0.08, 62)
    ux, uy = _stokes_gpu(mlf, torch_cuda, film, h)
    pres, _ = oracle_mod.pressure(film, h)
    qmax = max(np.abs(h * ux).max(), np.abs(h * uy).max())
    for y in range(0, 12, 3):
        for x in range(0, 16, 3):
            hn = h[:, y, x]
            K = np.stack([oracle_mod.friction(hn, film["mu"], np.eye(n)[j]) for j in range(n)], axis=1)
            for u, comp in ((ux, 0), (uy, 1)):
                gp = np.array([grad9(pres[i])[comp][y, x] for i in range(n)])
                q = np.linalg.solve(K, hn * gp)
                assert np.abs(hn * u[:, y, x] - q).max() <= 1e-11 * qmax


def test_stokes_velocity_rejects_slip_and_bad_arguments(mlf, torch_cuda):
    import ctypes as C

    film = _film(2, 8, 8, 70)
    film["slip"] = [0.0, 0.1]
    p = mlf.make_params(film, "f64")
    t = torch_cuda.ones((2, 8, 8), dtype=torch_cuda.float64, device="cuda")
    lib = mlf.load_library()
    ptr = C.c_void_p(t.data_ptr())
    assert lib.mlf_stokes_velocity(C.byref(p), ptr, ptr, ptr, None) == -2
    film["slip"] = [0.0, 0.0]
    p = mlf.make_params(film, "f64")
    assert lib.mlf_stokes_velocity(C.byref(p), None, ptr, ptr, None) == -1


def test_restart_from_the_solver_state(mlf, torch_cuda):
    """Three films of the surrogate's workload at t = 6e4, restarted from
    the solver's own heights and run one 100-step window: populations at
    equilibrium with the velocities the solver had 700 steps earlier (the
    judge's restart) stay far closer to the continuing solver than a
    restart at rest; with the exact current velocities the restart is the
    solver itself (at tau = 1 heights and fluxes fix the state).  The
    Stokes-limit velocities do worse than rest on these films (their
    grid-scale noise carries Stokes fluxes that the scheme's lattice
    viscosity damps): reported, not gated."""
    torch = torch_cuda
    from paper_2409_16659_amd import surrogate as S

    films = S.films(3, seed0=5100)
    ref = mlf.Batch([f for f, _ in films], "f64")
    for i, (_, h0) in enumerate(films):
        ref.init(i, h0)
    ref.step(59300)
    shape = (3, 3, 256, 256)
    f64 = dict(dtype=torch.float64, device="cuda")
    h_old, ux_old, uy_old = (torch.empty(shape, **f64) for _ in range(3))
    ref.read_all_hu(h_old, ux_old, uy_old)
    ref.step(700)
    h, ux_now, uy_now = (torch.empty(shape, **f64) for _ in range(3))
    ref.read_all_hu(h, ux_now, uy_now)
    ref.step(100)
    truth = ref.read_all().cpu().numpy()
    ux, uy = torch.empty(shape, **f64), torch.empty(shape, **f64)
    errs = {}
    for mode in ("rest", "stokes", "carried", "exact"):
        b = mlf.Batch([f for f, _ in films], "f64")
        if mode == "stokes":
            b.stokes_velocity(h, ux, uy)
            b.init_all(h, ux, uy)
        elif mode == "carried":
            b.init_all(h, ux_old, uy_old)
        elif mode == "exact":
            b.init_all(h, ux_now, uy_now)
        else:
            b.init_all(h)
        b.step(100)
        got = b.read_all().cpu().numpy()
        d = np.linalg.norm((got - truth).reshape(3, -1), axis=1)
        pert = np.linalg.norm((truth - truth.mean(axis=(2, 3), keepdims=True)).reshape(3, -1), axis=1)
        errs[mode] = (d / np.linalg.norm(truth.reshape(3, -1), axis=1)).max(), (d / pert).max()
        print(f"restart {mode}: rel L2 {errs[mode][0]:.2e}, perturbation-relative {errs[mode][1]:.2e}", flush=True)
        del b
    assert errs["carried"][0] <= 0.25 * errs["rest"][0]
    assert errs["exact"][0] <= 1e-13
    assert errs["carried"][0] <= 1e-5


def test_judge_errors_and_conversions(mlf, torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(80)
    b = (0.8 + 1e-2 * rng.normal(size=(5, 3, 16, 256))).astype(np.float32)
    a = (b + 1e-4 * rng.normal(size=b.shape)).astype(np.float32)
    s = mlf.Surrogate(3, 256, 16, width=64, blocks=1, batch=8, scale=1e-2)
    got = s.errors(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    d = np.linalg.norm((a64 - b64).reshape(5, -1), axis=1)
    want0 = d / np.linalg.norm(b64.reshape(5, -1), axis=1)
    want1 = d / np.linalg.norm((b64 - b64.mean(axis=(2, 3), keepdims=True)).reshape(5, -1), axis=1)
    assert np.abs(got[:, 0] - want0).max() <= 1e-12 * want0.max()
    assert np.abs(got[:, 1] - want1).max() <= 1e-12 * want1.max()
    x64 = torch.from_numpy(rng.normal(size=(2, 3, 5, 7))).cuda()
    x32 = torch.empty(x64.shape, dtype=torch.float32, device="cuda")
    mlf.convert_heights(x64, x32)
    back = torch.empty_like(x64)
    mlf.convert_heights(x32, back)
    torch.cuda.synchronize()
    assert np.array_equal(x32.cpu().numpy(), x64.cpu().numpy().astype(np.float32))
    assert np.array_equal(back.cpu().numpy(), x32.cpu().numpy().astype(np.float64))
