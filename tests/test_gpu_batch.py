"""Batched films (one launch per step over a work list of (film, tile)
items, per-film constants in a device table, optional HIP graph of the step
loop) against single-film runs and the FP64 oracle.

Gate: every film of a batch is bit-identical to the same film stepped alone
through the single-film entry point with the same launch shape (that path
is pinned to the oracle elsewhere), for both launch modes (one workgroup
per item, persistent workgroups) and with graph replays; FP64 films also
meet the oracle tolerance directly.
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


def scan(count, seed, side_max=160):
    films = inputs.batch_scan(count=count, seed=seed, side_min=64, side_max=side_max)
    # ragged and tiny films next to the scan's multiples of 16
    extra = [(3, 37, 5), (2, 70, 1), (4, 101, 29), (1, 9, 9)]
    rng = np.random.default_rng(seed)
    for n, nx, ny in extra:
        gam = list(rng.uniform(0.5e-2, 1.5e-2, size=n))
        film = inputs.film_params(n, nx, ny, gamma=gam, mu=[1.5e-3] * n, hstar=0.15,
                                  spread={(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(n)})
        h0 = np.stack([(1.0 - 0.2 * i) + 1e-3 * rng.uniform(-1, 1, size=(ny, nx)) for i in range(n)])
        films.append((film, h0))
    return films


def single(mlf, film, h0, prec, launch, steps):
    g = mlf.Film(film, prec)
    g.set_launch(*launch)
    g.init(h0)
    g.step(steps)
    return g.read()


@pytest.mark.parametrize("prec", ["f32", "f64", "f16mix"])
@pytest.mark.parametrize("persistent", [0, 1])
def test_batch_matches_single_films(mlf, prec, persistent):
    films = scan(10, seed=5)
    launch = (128, 6)
    b = mlf.Batch([f for f, _ in films], prec)
    b.set_launch(*launch, persistent)
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    steps = 37
    b.step(steps)
    assert b.steps_done == steps
    say(f"batch {prec} persistent={persistent}: {len(films)} films, launch {b.get_launch()}")
    for i, (film, h0) in enumerate(films):
        hb, uxb, uyb = b.read(i)
        hs, uxs, uys = single(mlf, film, h0, prec, launch, steps)
        assert np.array_equal(hb, hs), i
        assert np.array_equal(uxb, uxs) and np.array_equal(uyb, uys), i


@pytest.mark.parametrize("prec", ["f32", "f16mix"])
@pytest.mark.parametrize("persistent", [0, 1])
def test_batch_two_rows_ahead_matches_single_films(mlf, prec, persistent):
    """Two rows in flight in the batch kernel (tall segments, where it
    pays) give every film the populations of its single-film run with one
    row in flight."""
    films = scan(8, seed=11)
    launch = (192, 24)
    b = mlf.Batch([f for f, _ in films], prec)
    b.set_launch(*launch, persistent)
    b.set_prefetch(2)
    assert b.get_prefetch() == 2
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    steps = 21
    b.step(steps)
    say(f"batch {prec} persistent={persistent} two rows ahead: {len(films)} films")
    for i, (film, h0) in enumerate(films):
        hb, uxb, uyb = b.read(i)
        hs, uxs, uys = single(mlf, film, h0, prec, launch, steps)
        assert np.array_equal(hb, hs), i
        assert np.array_equal(uxb, uxs) and np.array_equal(uyb, uys), i


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_batch_stochastic_rounding_matches_single_films(mlf, prec):
    """Stochastic rounding of the rest plane draws on each film's node
    index, layer and step count: every film of a batch is bit-identical to
    the same film stepped alone with stochastic rounding (and differs from
    round-to-nearest); a batch with it refuses graph capture."""
    films = scan(6, seed=17)
    launch = (128, 6)
    b = mlf.Batch([f for f, _ in films], prec)
    r = mlf.Batch([f for f, _ in films], prec)
    for bb in (b, r):
        bb.set_launch(*launch, 0)
        for i, (_, h0) in enumerate(films):
            bb.init(i, h0)
    assert not b.get_rounding()
    b.set_rounding(True)
    assert b.get_rounding() and not r.get_rounding()
    steps = 29
    b.step(steps)
    r.step(steps)
    say(f"batch {prec} stochastic rounding: {len(films)} films, launch {b.get_launch()}")
    differs = 0
    for i, (film, h0) in enumerate(films):
        g = mlf.Film(film, prec)
        g.set_launch(*launch)
        g.set_rounding(True)
        g.init(h0)
        g.step(steps)
        hs, uxs, uys = g.read()
        hb, uxb, uyb = b.read(i)
        assert np.array_equal(hb, hs), i
        assert np.array_equal(uxb, uxs) and np.array_equal(uyb, uys), i
        differs += not np.array_equal(hb, r.read(i)[0])
    assert differs == len(films)
    with pytest.raises(mlf.MlfError) as ex:
        b.capture(8)
    assert ex.value.status == "EUNSUPPORTED"
    b.set_rounding(False)
    b.capture(8)   # round-to-nearest batches capture again


def test_batch_fp64_against_oracle(mlf, oracle_mod):
    films = scan(3, seed=7, side_max=96)
    # one film with slip lengths next to no-slip films
    films[1] = (dict(films[1][0], slip=[0.5] * films[1][0]["n_layers"]), films[1][1])
    b = mlf.Batch([f for f, _ in films], "f64")
    b.set_launch(192, 5, 1)
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    steps = 60
    b.step(steps)
    for i, (film, h0) in enumerate(films):
        o = oracle_mod.Oracle(film)
        o.init(h0)
        o.step(steps)
        ho, uxo, uyo = o.read()
        hb, uxb, uyb = b.read(i)
        eh = np.abs(hb - ho).max() / np.abs(ho).max()
        us = max(np.abs(uxo).max(), np.abs(uyo).max(), 1e-300)
        eu = max(np.abs(uxb - uxo).max(), np.abs(uyb - uyo).max()) / us
        say(f"   film {i} N={film['n_layers']} {film['nx']}x{film['ny']}: e_h={eh:.2e} e_U={eu:.2e}")
        assert eh <= 1e-12 and eu <= 1e-10


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replays_match_eager_steps(mlf, persistent):
    """A captured 8-step graph, replayed several times with eager steps and
    synchronising read-backs in between, gives every time the state of a
    batch stepped eagerly."""
    films = scan(6, seed=9, side_max=128)
    launch = (192, 8, persistent)
    a = mlf.Batch([f for f, _ in films], "f32")
    e = mlf.Batch([f for f, _ in films], "f32")
    for bb in (a, e):
        bb.set_launch(*launch)
        for i, (_, h0) in enumerate(films):
            bb.init(i, h0)
    a.capture(8)
    for chunk in (8, 16, 3, 8, 13, 24):   # odd chunks: eager steps restore the parity
        a.step(chunk)
        e.step(chunk)
        assert a.steps_done == e.steps_done
        for i in (0, len(films) - 1, len(films) // 2):
            ha, _, _ = a.read(i)
            he, _, _ = e.read(i)
            assert np.array_equal(ha, he), (chunk, i)
    a.set_launch(*launch)   # a new launch shape drops the graph
    a.step(5)
    e.step(5)
    for i in range(len(films)):
        assert np.array_equal(a.read(i)[0], e.read(i)[0])


def test_graph_capture_rejects_odd_steps(mlf):
    films = scan(2, seed=11, side_max=64)
    b = mlf.Batch([f for f, _ in films], "f32")
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    with pytest.raises(mlf.MlfError) as ex:
        b.capture(3)
    assert ex.value.status == "EINVAL"


def test_batch_autotune_keeps_state(mlf):
    films = scan(8, seed=13)
    a = mlf.Batch([f for f, _ in films], "f32")
    for i, (_, h0) in enumerate(films):
        a.init(i, h0)
    a.step(4)
    before = [a.read(i)[0] for i in range(len(films))]
    bw, sh, pers = a.autotune(reps=1)
    say(f"   batch autotune: {bw}x{sh} persistent={pers} rows ahead {a.get_prefetch()}")
    assert (bw, sh, pers) == a.get_launch()
    assert a.get_prefetch() in (1, 2)
    assert a.steps_done == 4
    for i in range(len(films)):
        assert np.array_equal(a.read(i)[0], before[i])
    a.step(6)
    for i, (film, h0) in enumerate(films):
        hs, _, _ = single(mlf, film, h0, "f32", (bw, sh), 10)
        assert np.array_equal(a.read(i)[0], hs), i


def test_batch_mass_conservation(mlf):
    films = scan(5, seed=15)
    b = mlf.Batch([f for f, _ in films], "f64")
    for i, (_, h0) in enumerate(films):
        b.init(i, h0)
    m0 = [b.mass(i) for i in range(len(films))]
    b.step(200)
    for i in range(len(films)):
        m1 = b.mass(i)
        assert np.abs(m1 - m0[i]).max() <= 1e-12 * np.abs(m0[i]).max(), i


def test_batch_guard_names_the_failing_film(mlf):
    """One film with an explicitly unstable friction (accepted with
    allow_unstable) blows up; the guard reports that film."""
    films = scan(4, seed=17, side_max=64)
    bad = 2
    film, h0 = films[bad]
    film = dict(film)
    film["mu"] = [3.0] * film["n_layers"]
    films[bad] = (film, h0)
    b = mlf.Batch([f for f, _ in films], "f32", allow_unstable=True)
    for i, (_, h) in enumerate(films):
        b.init(i, h)
    with pytest.raises(mlf.MlfError) as ex:
        b.step(400)
    assert ex.value.status in ("ENONPOSITIVE", "ENONFINITE")
    assert b.failed_film == bad


def test_uninitialised_film_is_rejected(mlf):
    films = scan(3, seed=19, side_max=64)
    b = mlf.Batch([f for f, _ in films], "f32")
    b.init(0, films[0][1])
    with pytest.raises(mlf.MlfError) as ex:
        b.step(1)
    assert ex.value.status == "EINVAL"


def test_init_and_read_all_films_at_once(mlf, torch_cuda):
    """Batch-wide device init / read equal the per-film calls."""
    torch = torch_cuda
    rng = np.random.default_rng(21)
    films = []
    for j in range(3):
        gam = list(rng.uniform(0.5e-2, 1.5e-2, size=3))
        film = inputs.film_params(3, 96, 64, gamma=gam, mu=[1.5e-3] * 3, hstar=0.15,
                                  spread={(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(3)})
        films.append((film, np.stack([(1.0 - 0.2 * i) + 1e-3 * rng.uniform(-1, 1, (64, 96)) for i in range(3)])))
    hs = torch.from_numpy(np.stack([h for _, h in films])).cuda()
    a = mlf.Batch([f for f, _ in films], "f32")
    b = mlf.Batch([f for f, _ in films], "f32")
    a.init_all(hs)
    for i in range(len(films)):
        b.init(i, hs[i].contiguous())
    a.step(17)
    b.step(17)
    ra = a.read_all().cpu().numpy()
    for i in range(len(films)):
        assert np.array_equal(ra[i], b.read(i)[0]), i
