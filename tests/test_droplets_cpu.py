"""Host side of the droplet sweep (paper_2409_16659_amd/droplets.py):
initial drops of every kind have the requested initial angle and volume
layout, the arc fit recovers exact caps, and every film passes the
library's parameter validation (no GPU needed)."""
import math

import numpy as np
import pytest

from paper_2409_16659_amd import droplets, mlfilm


@pytest.mark.parametrize("theta", [4.0, 17.3, 33.0, 44.0])
def test_fit_recovers_exact_caps(theta):
    x = np.arange(256) + 0.5
    d = droplets.cap(x, 128.0, 60.0, math.radians(theta))
    ang, e_best, err = droplets.fit_arc(d)
    assert abs(ang - theta) <= 0.5 and e_best < 0.02   # peak sampled half a node off
    assert err(math.radians(theta)) < 0.02 and err(math.radians(1.3 * theta)) > 0.05


def test_model_angle_small_slope_form():
    # tan(theta_eq) = 2 sin(theta / 2): 9.89 and 19.15 degrees for 10 and 20
    assert abs(droplets.model_angle(10.0) - 9.89) < 0.01
    assert abs(droplets.model_angle(20.0) - 19.15) < 0.01
    assert abs(droplets.model_angle(45.0) - 37.43) < 0.01


@pytest.mark.parametrize("kind", droplets.KINDS)
def test_initial_drops(kind):
    for th, th0 in ((20.0, 20.0), (20.0, 40.0), (10.0, 5.0)):
        film, h0 = droplets.drop(kind, th, th0)
        assert h0.shape == (film["n_layers"], 1, film["nx"]) and h0.min() > 0
        mlfilm.query_sizes(mlfilm.make_params(film, "f32"))   # valid and stable
        for face, d in droplets.profiles(kind, h0).items():
            ang, e_best, _ = droplets.fit_arc(d)
            assert abs(ang - th0) <= 0.5 and e_best < 0.02, (face, ang)
    # the spreading coefficient sits on the pair that holds the contact line
    film, _ = droplets.drop(kind, 20.0, 20.0)
    key = {"sessile": (0, 1), "type1": (0, 1), "type3": (0, 2), "lens": (1, 1)}[kind]
    nonzero = [k for k, v in film["spread"].items() if v != 0.0]
    assert nonzero == [key]


def test_paper_cases():
    cases = droplets.paper_cases()
    assert len(cases) == 4 * 5 * 3
    assert ("sessile", 30.0, 45.0) in cases and ("lens", 10.0, 5.0) in cases
