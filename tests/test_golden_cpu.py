"""Consistency of the oracle-written fixture the full-size parity test
compares against (tests/golden/film3_1024_t10k.npz, written by
tests/golden/make_film3_1024_t10k.py): shapes and row sets, finite positive
heights, the oracle's own per-layer mass conservation over the 10^4 steps,
and the state of the linear regime (the perturbation has neither vanished
nor grown to the film's scale)."""
import os

import numpy as np

from paper_2409_16659_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "film3_1024_t10k.npz")


def test_t10k_fixture_is_consistent():
    ref = np.load(GOLDEN)
    film, h0, _ = inputs.workload("film3_2d_1024")
    n, ny, nx = film["n_layers"], film["ny"], film["nx"]
    assert int(ref["steps"]) == 10_000
    assert np.array_equal(ref["rows_h"], np.arange(0, ny, 16))
    assert np.array_equal(ref["rows_u"], np.arange(0, ny, 64))
    assert ref["h"].shape == (n, ny // 16, nx)
    assert ref["ux"].shape == ref["uy"].shape == (n, ny // 64, nx)
    h = ref["h"]
    assert np.all(np.isfinite(h)) and np.all(h > film["hstar"])
    # the initial mass is the seeded input's own sum
    assert np.allclose(ref["mass0"], h0.sum(axis=(1, 2)), rtol=1e-14, atol=0)
    # the oracle conserves every layer's mass (FP64)
    assert np.abs(ref["mass"] - ref["mass0"]).max() <= 1e-12 * ref["mass0"].max()
    # layer means unchanged; perturbations small (linear regime) but alive
    hbar = np.array([1.0, 0.8, 0.6])
    assert np.abs(h.mean(axis=(1, 2)) - hbar).max() < 1e-4
    pert = np.abs(h - h.mean(axis=(1, 2), keepdims=True)).max()
    assert 1e-7 < pert < 1e-2
    assert np.abs(ref["ux"]).max() < 1e-3 and np.abs(ref["ux"]).max() > 0


LONG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "film4_512_long.npz")


def test_long_horizon_fixture_is_consistent():
    """tests/golden/film4_512_long.npz (the oracle's 4-layer 512^2 crop at
    10^4, 2 10^4 and 5 10^4 steps, every 8th row): shapes, finite positive
    heights, the oracle's per-layer mass conservation over
    5 10^4 steps, and a perturbation that grows between the checkpoints
    (the film is unstable on this horizon)."""
    ref = np.load(LONG)
    film, h0, _ = inputs.workload("film4_2d_512")
    n, ny, nx = film["n_layers"], film["ny"], film["nx"]
    assert list(ref["t"]) == [10_000, 20_000, 50_000]
    assert np.array_equal(ref["rows"], np.arange(0, ny, 8))
    assert ref["h"].shape == (3, n, ny // 8, nx)
    h = ref["h"]
    assert np.all(np.isfinite(h)) and np.all(h > 0)
    assert np.allclose(ref["mass0"], h0.sum(axis=(1, 2)), rtol=1e-14, atol=0)
    assert np.abs(ref["mass"] - ref["mass0"][None]).max() <= 1e-11 * ref["mass0"].max()
    pert = [float(np.linalg.norm(h[k] - h[k].mean(axis=(1, 2), keepdims=True))) for k in range(3)]
    assert pert[0] < pert[1] < pert[2]
