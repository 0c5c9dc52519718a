"""D1Q3 films (pseudo-1D, ny == 1) on the GPU against the oracle's D1Q3
path: the resident kernels, which hold the film in LDS for many steps per
launch (one workgroup for up to 128 nodes; tiles of 32 nodes with 48-node
halos, 16 steps per launch, for longer films), and batches of strips.

Gates as for D2Q9: FP64 e_h <= 1e-12, e_U <= 1e-10, FP32 e_h <= 1e-5,
e_U <= 1e-4; populations against the oracle's; results independent of how
the steps are split into launches (bit for bit); D1Q3 equals D2Q9 on a film
one row high to FP64 rounding; mass conserved to 1e-12.
"""
import sys

import numpy as np
import pytest

from paper_2409_16659_amd import inputs

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def strip(n, nx, seed, tau=1.0, exps=(9, 3), slip=None):
    rng = np.random.default_rng(seed)
    gam = list(rng.uniform(0.5e-2, 1.5e-2, size=n))
    spread = {(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(n)}
    for l in range(n):
        for k in range(2, n - l + 1):
            spread[(l, k)] = rng.uniform(-2e-3, 2e-3)
    film = inputs.film_params(n, nx, 1, gamma=gam, mu=list(rng.uniform(1e-3, 2.5e-3, size=n)), hstar=0.15,
                              spread=spread, tau=tau, exp_a=exps[0], exp_b=exps[1], slip=slip)
    h0 = np.stack([(1.0 - 0.15 * i) + 1e-2 * rng.uniform(-1, 1, size=(1, nx)) for i in range(n)])
    return film, h0


def pair(mlf, oracle_mod, film, h0, steps, prec="f64", ux=None):
    say(f"case N={film['n_layers']} nx={film['nx']} {prec} steps={steps} tau={film.get('tau', 1.0)}")
    g = mlf.Film(film, prec, lattice="d1q3")
    g.init(h0, ux)
    o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    o.init(h0, ux)
    g.step(steps)
    o.step(steps)
    return g, o


def check(g, o, tol_h, tol_u):
    hg, ug, _ = g.read()
    ho, uo, _ = o.read()
    eh, eu = err(hg, ho), err(ug, uo)
    say(f"   e_h={eh:.2e} e_U={eu:.2e}")
    assert eh <= tol_h and eu <= tol_u


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("nx", [1, 2, 3, 7, 64, 128, 129, 333, 700])
def test_fp64_against_oracle(mlf, oracle_mod, n, nx):
    film, h0 = strip(n, nx, seed=10 * n + nx)
    g, o = pair(mlf, oracle_mod, film, h0, 300)
    check(g, o, 1e-12, 1e-10)
    fo = o.get_f()
    assert fo.shape == (n, 3, 1, nx)
    assert np.abs(g.populations() - fo).max() <= 1e-12 * np.abs(fo).max()


@pytest.mark.parametrize("n", [2, 4])
def test_fp64_long_strip_tiled(mlf, oracle_mod, n):
    """A long strip: 94 tiles of 32 nodes with a ragged last one (25)."""
    film, h0 = strip(n, 3001, seed=5 + n)
    g, o = pair(mlf, oracle_mod, film, h0, 120)
    check(g, o, 1e-12, 1e-10)


def test_fp64_general_tau_exponents_slip_velocity(mlf, oracle_mod):
    film, h0 = strip(3, 150, seed=1, tau=0.8, exps=(4, 3), slip=[0.3, 0.0, 1.0])
    rng = np.random.default_rng(2)
    ux = 1e-3 * rng.uniform(-1, 1, size=h0.shape)
    g, o = pair(mlf, oracle_mod, film, h0, 400, ux=ux)
    check(g, o, 1e-12, 1e-10)
    film, h0 = strip(2, 1500, seed=3, tau=1.3)
    g, o = pair(mlf, oracle_mod, film, h0, 100)
    check(g, o, 1e-12, 1e-10)


@pytest.mark.parametrize("nx", [96, 1024, 2000])
def test_fp32_against_oracle(mlf, oracle_mod, nx):
    film, h0 = strip(3, nx, seed=nx)
    g, o = pair(mlf, oracle_mod, film, h0, 300, prec="f32")
    check(g, o, 1e-5, 1e-4)


def test_two_layer_workload_full_length(mlf, oracle_mod):
    """The 2-layer pseudo-1D workload over its 10^4 steps on D1Q3 (resident
    kernel), against the oracle's D1Q3 and D2Q9 runs and the GPU's D2Q9
    path: the lattices agree in exact arithmetic."""
    film, h0, _ = inputs.workload("film2_pseudo1d_512")
    g = mlf.Film(film, "f64", lattice="d1q3")
    g.init(h0)
    m0 = g.mass()
    g.step(10_000)
    o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    o.init(h0)
    o.step(10_000)
    check(g, o, 1e-12, 1e-10)
    assert np.abs(g.mass() - m0).max() <= 1e-12 * m0.max()
    d = mlf.Film(film, "f64")
    d.init(h0)
    d.step(10_000)
    hd, ud, _ = d.read()
    hg, ug, _ = g.read()
    say(f"   D1Q3 vs D2Q9 on the GPU: e_h={err(hg, hd):.2e} e_U={err(ug, ud):.2e}")
    assert err(hg, hd) <= 1e-12 and err(ug, ud) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_launch_split_independence(mlf, prec):
    film, h0 = strip(3, 400, seed=4)
    a = mlf.Film(film, prec, lattice="d1q3")
    b = mlf.Film(film, prec, lattice="d1q3", check_every=7)
    for g in (a, b):
        g.init(h0)
    a.step(500)
    for chunk in (1, 2, 97, 400):
        b.step(chunk)
    assert a.steps_done == b.steps_done == 500
    assert np.array_equal(a.read()[0], b.read()[0]) and np.array_equal(a.read()[1], b.read()[1])


def test_diagnostics_and_checkpoint(mlf):
    film, h0 = strip(2, 300, seed=6)
    g = mlf.Film(film, "f64", lattice="d1q3")
    g.init(h0)
    g.step(50)
    h = g.read()[0]
    assert np.array_equal(g.layer_min(), h.reshape(2, -1).min(axis=1))
    blob = g.save()
    ref = g.read()[0]
    g.step(30)
    g.load(blob)
    assert g.steps_done == 50 and np.array_equal(g.read()[0], ref)
    f = g.populations()
    g.set_populations(f)
    assert np.abs(g.read()[0] - ref).max() <= 1e-15


def test_guard_and_unsupported(mlf):
    film, h0 = strip(2, 128, seed=7)
    bad = dict(film, mu=[3.0, 3.0])
    g = mlf.Film(bad, "f64", lattice="d1q3", allow_unstable=True)
    g.init(h0)
    with pytest.raises(mlf.MlfError) as e:
        g.step(2000)
    assert e.value.status in ("ENONPOSITIVE", "ENONFINITE")
    g = mlf.Film(film, "f64", lattice="d1q3")
    g.init(h0)
    with pytest.raises(mlf.MlfError) as e:
        g.capture(8)
    assert e.value.status == "EUNSUPPORTED"


@pytest.mark.parametrize("col", [0, 31, 32, 399])
def test_tiled_guard_at_tile_edges(mlf, col):
    """A non-positive height at the first or last node of a tile, or at the
    strip's wrap-around edge, trips the guard of the tiled kernel; the
    healthy strip runs on without a false alarm from the halos."""
    film, h0 = strip(2, 400, seed=8)
    g = mlf.Film(film, "f64", lattice="d1q3", check_every=20)
    g.init(h0)
    g.step(20)
    f = g.populations()
    f[0, 0, 0, col] = -5.0
    g.set_populations(f)
    with pytest.raises(mlf.MlfError) as e:
        g.step(20)
    assert e.value.status in ("ENONPOSITIVE", "ENONFINITE")
    ok = mlf.Film(film, "f64", lattice="d1q3", check_every=20)
    ok.init(h0)
    ok.step(200)


BATCH_STRIPS = [(1, 64), (2, 333), (3, 500), (4, 96), (2, 5), (4, 400), (3, 1)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_matches_single_films(mlf, prec):
    """A batch of D1Q3 strips (one workgroup per film, each held in LDS)
    gives every film bit for bit what the single-film resident kernel gives,
    with the steps split into launches differently."""
    films = [strip(n, nx, seed=300 + 7 * n + nx) for n, nx in BATCH_STRIPS]
    b = mlf.Batch([f for f, _ in films], prec, lattice="d1q3")
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    b.step(300)
    b.step(477)
    assert b.steps_done == 777
    mins = b.layer_min_all()
    for i, (film, h0) in enumerate(films):
        g = mlf.Film(film, prec, lattice="d1q3")
        g.init(h0)
        g.step(777)
        hb, ub, _ = b.read(i)
        hs, us, _ = g.read()
        assert np.array_equal(hb, hs) and np.array_equal(ub, us), i
        assert np.array_equal(mins[i, :film["n_layers"]], hb.reshape(film["n_layers"], -1).min(axis=1))


def test_batch_against_oracle(mlf, oracle_mod):
    films = [strip(n, nx, seed=400 + n) for n, nx in [(2, 200), (4, 150), (1, 77)]]
    b = mlf.Batch([f for f, _ in films], "f64", lattice="d1q3")
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    b.step(400)
    for i, (film, h0) in enumerate(films):
        o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
        o.init(h0)
        o.step(400)
        hb, ub, _ = b.read(i)
        ho, uo, _ = o.read()
        say(f"   batch film {i}: e_h={err(hb, ho):.2e} e_U={err(ub, uo):.2e}")
        assert err(hb, ho) <= 1e-12 and err(ub, uo) <= 1e-10
    with pytest.raises(mlf.MlfError) as e:
        b.capture(8)
    assert e.value.status == "EUNSUPPORTED"


def test_batch_guard_names_the_failing_film(mlf):
    films = [strip(2, 128, seed=500 + j) for j in range(3)]
    film, h0 = films[1]
    films[1] = (dict(film, mu=[3.0, 3.0]), h0)
    b = mlf.Batch([f for f, _ in films], "f64", lattice="d1q3", allow_unstable=True)
    for i, (_, h) in enumerate(films):
        b.init(i, h)
    with pytest.raises(mlf.MlfError) as e:
        b.step(2000)
    assert e.value.status in ("ENONPOSITIVE", "ENONFINITE")
    assert b.failed_film == 1


def test_rupture_detection_on_d1q3(mlf, oracle_mod):
    """Rupture of the four-layer strip on D1Q3: the single film (resident
    kernel) stops at the oracle's D1Q3 check, and a batch of strips reports
    for each film the step it gives alone."""
    films = []
    for j, amp in enumerate((1e-2, 2e-2, 5e-3)):
        film = inputs._film4(192, 1)
        films.append((film, inputs.initial_heights(film, (1.0, 0.8, 0.6, 0.4), "uniform", 11 + j, amp)))
    film, h0 = films[0]
    g = mlf.Film(film, "f64", lattice="d1q3")
    g.init(h0)
    steps, layer = g.step_until(60_000, 100)
    o = oracle_mod.Oracle(film, oracle_mod.D1Q3)
    o.init(h0)
    thr = mlf.rupture_threshold(film)
    while o.steps_done < 60_000:
        o.step(100)
        if (o.read()[0].reshape(4, -1).min(axis=1) <= thr).any():
            break
    say(f"   D1Q3 rupture: GPU {steps} (layer {layer}), oracle {o.steps_done}")
    assert steps == o.steps_done and layer == 3
    b = mlf.Batch([f for f, _ in films], "f64", lattice="d1q3")
    for i, (_, h) in enumerate(films):
        b.init(i, h)
    t_hit, lay, _ = b.step_until(60_000, 100)
    for i, (f, h) in enumerate(films):
        s = mlf.Film(f, "f64", lattice="d1q3")
        s.init(h)
        assert s.step_until(60_000, 100) == (t_hit[i], lay[i]), i
