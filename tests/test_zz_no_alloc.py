"""The allocation-free per-layer mass (mlf_layer_mass_static) against
mlf_layer_mass through the C ABI: same kernels and summation order, so the
results must be bit-identical.  Two calls in a row on one GPU (they share
the library's fixed device array), the second on a smaller film."""
import ctypes as C

import numpy as np
import pytest

from paper_2409_16659_amd import inputs

pytestmark = pytest.mark.gpu


def _film(n, nx, ny, seed):
    gam = [1.0e-2, 0.8e-2, 0.6e-2, 0.5e-2][:n]
    spread = {(l, 1): inputs.young_spreading(gam[l], 20.0) for l in range(n)}
    film = inputs.film_params(n, nx, ny, gamma=gam, mu=[1e-3 * (1 + 0.5 * i) for i in range(n)], hstar=0.1,
                              spread=spread)
    h0 = inputs.initial_heights(film, (1.0, 0.8, 0.6, 0.4)[:n], "uniform", seed, 1e-3)
    return film, h0


def test_layer_mass_static_matches_layer_mass():
    import torch

    from paper_2409_16659_amd import mlfilm

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    lib = mlfilm.load_library()
    cases = [(4, 1031, 300, "f64", 11), (2, 64, 33, "f32", 12)]  # the second call on a smaller film
    for n, nx, ny, prec, seed in cases:
        print(f"case layer_mass_static N={n} {nx}x{ny} {prec}", flush=True)
        film, h0 = _film(n, nx, ny, seed)
        g = mlfilm.Film(film, prec)
        g.init(h0)
        g.step(9)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device=g.device)
        rc = lib.mlf_layer_mass_static(g.h, C.c_void_p(out.data_ptr()))
        assert rc == 0, rc
        g.stream.synchronize()
        got = out.cpu().numpy()
        ref = g.mass()
        assert np.array_equal(got, ref), (got, ref)
        # a second call on the same film after more steps: the array keeps the
        # previous call's partials, which must not leak into the result
        g.step(3)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        assert lib.mlf_layer_mass_static(g.h, C.c_void_p(out.data_ptr())) == 0
        g.stream.synchronize()
        assert np.array_equal(out.cpu().numpy(), g.mass())
        del g


def test_layer_mass_static_rejects_bad_arguments():
    import torch

    from paper_2409_16659_amd import mlfilm

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    lib = mlfilm.load_library()
    film, h0 = _film(2, 32, 8, 13)
    g = mlfilm.Film(film, "f32")
    out = torch.zeros(2, dtype=torch.float64, device=g.device)
    assert lib.mlf_layer_mass_static(g.h, C.c_void_p(out.data_ptr())) == -1  # before init
    g.init(h0)
    assert lib.mlf_layer_mass_static(g.h, None) == -1
    assert lib.mlf_layer_mass_static(None, C.c_void_p(out.data_ptr())) == -1
