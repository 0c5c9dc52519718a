"""Long-horizon accuracy of the storage formats on the 4-layer 512^2 crop
(the [0:512, 0:512] window of the 4-layer workload's seeded fields, its own
periodic domain) against the FP64 oracle's heights stored at 10^4, 2 10^4
and 5 10^4 steps (tests/golden/film4_512_long.npz, every 8th row, written
by tests/golden/make_film4_512_long.py, which calls only the oracle).

Over this horizon the films go unstable and dewet, so any rounding
difference grows with the instability (by up to exp(eta T)): the GPU's
FP64 path, which rounds in another order, drifts from the oracle as well.
The errors are measured over the kept rows, max over layers: relative
L2 ||h - h_ref|| / ||h_ref|| and relative to the height perturbation,
||h - h_ref|| / ||h_ref - mean h_ref||, plus the relative change of each
layer's mass since t = 0.  Measured on MI355X (perturbation-relative at
10^4 / 2 10^4 / 5 10^4 steps): FP64 6.5e-9 / 7.1e-9 / 1.8e-10 (relative
L2 8.7e-11 at 5 10^4, mass unchanged); FP32 2.4e-5 / 4.0e-5 / 1.2e-4;
FP32 rest with IEEE-half moving planes 8.3e-4 / 3.8e-3 / 2.5e-3; with
bfloat16 moving planes 1.5e-2 / 5.6e-2 / 0.14.  The bars are about ten
times these (a regression check: in this unstable regime a different but
equally valid rounding order moves the errors by factors, not orders of
magnitude).  The all-16-bit formats, whose height increments round away,
are the documented failure: their films do not dewet, so at 5 10^4 steps
they are checked to stay a whole perturbation off the oracle; with the rest
population rounded stochastically (mlf_set_rounding) they follow it.
"""
import os

import numpy as np
import pytest

from paper_2409_16659_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "film4_512_long.npz")


@pytest.fixture(scope="module")
def mlf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_16659_amd import mlfilm

    mlfilm.load_library()
    return mlfilm


@pytest.fixture(scope="module")
def gold():
    return np.load(GOLDEN)


def run(mlf, gold, prec, stochastic=False):
    film, h0, _ = inputs.workload("film4_2d_512")
    g = mlf.Film(film, prec, check_every=-1)
    if stochastic:
        g.set_rounding(True)
    g.init(h0)
    m0 = g.mass()
    rows = gold["rows"]
    out = []
    t = 0
    for k, tc in enumerate(gold["t"]):
        g.step(int(tc) - t)
        t = int(tc)
        h, _, _ = g.read()
        ref = gold["h"][k]
        hs = h[:, rows]
        e_pert = max(float(np.linalg.norm(hs[i] - ref[i]) / np.linalg.norm(ref[i] - ref[i].mean()))
                     for i in range(ref.shape[0]))
        e_l2 = max(float(np.linalg.norm(hs[i] - ref[i]) / np.linalg.norm(ref[i])) for i in range(ref.shape[0]))
        m = g.mass()
        drift = float(np.max(np.abs(m - m0) / m0))
        out.append((t, e_l2, e_pert, drift))
        print(f"{prec} {'stochastic ' if stochastic else ''}t={t}: rel L2 {e_l2:.3e}, "
              f"vs perturbation {e_pert:.3e}, mass drift {drift:.2e}", flush=True)
    return out


# per format: (rel L2, perturbation-relative, mass drift) bars at 10^4, 2 10^4, 5 10^4 steps
BARS = {
    "f64": [(1e-11, 1e-7, 1e-12), (1e-11, 1e-7, 1e-12), (1e-9, 1e-8, 1e-12)],
    "f32": [(1e-7, 2e-4, 1e-8), (1e-6, 4e-4, 1e-7), (4e-4, 1e-3, 1e-4)],
    "f16mix": [(2e-6, 1e-2, 1e-8), (2e-5, 4e-2, 1e-7), (1e-2, 3e-2, 1e-4)],
    "bf16mix": [(3e-5, 0.15, 1e-8), (6e-4, 0.5, 1e-7), (0.3, 0.6, 2e-4)],
}


@pytest.mark.parametrize("prec", list(BARS))
def test_long_horizon_vs_stored_oracle(mlf, gold, prec):
    res = run(mlf, gold, prec)
    for (t, e_l2, e_pert, drift), (b_l2, b_pert, b_m) in zip(res, BARS[prec]):
        assert e_l2 <= b_l2, (t, e_l2, b_l2)
        assert e_pert <= b_pert, (t, e_pert, b_pert)
        assert drift <= b_m, (t, drift, b_m)


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_all_16_bit_formats_stall(mlf, gold, prec):
    """At 5 10^4 steps the oracle's film has dewetted while the all-16-bit
    ones have barely moved: the error is a whole perturbation."""
    res = run(mlf, gold, prec)
    t, e_l2, e_pert, drift = res[-1]
    assert e_pert >= 0.5, (t, e_pert)
    assert drift <= 1e-5


# all-16-bit storage with the rest population rounded stochastically: per
# format (rel L2, perturbation-relative, mass drift) bars at 10^4, 2 10^4,
# 5 10^4 steps, about three to five times the measured values (f16 4.9e-6 /
# 9.8e-3 / 1.3e-8, 2.2e-5 / 1.2e-2 / 4.4e-8, 1.4e-2 / 2.9e-2 / 4.8e-6; bf16
# 2.4e-5 / 4.7e-2 / 1.2e-7, 1.0e-4 / 5.2e-2 / 1.1e-7, 7.9e-2 / 0.18 / 3.0e-5)
SR_BARS = {
    "f16": [(3e-5, 5e-2, 1e-7), (1e-4, 5e-2, 2e-7), (5e-2, 0.1, 2e-5)],
    "bf16": [(1e-4, 0.2, 5e-7), (5e-4, 0.2, 5e-7), (0.3, 0.5, 1e-4)],
}


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_stochastic_rest_rounding_follows_the_oracle(mlf, gold, prec):
    """With the rest population rounded stochastically the all-16-bit films
    dewet with the oracle's: at 5 10^4 steps the height error is a small
    fraction of the perturbation instead of all of it; the mass drifts by
    the random walk of the roundings only."""
    for (t, e_l2, e_pert, drift), (b_l2, b_pert, b_m) in zip(run(mlf, gold, prec, stochastic=True), SR_BARS[prec]):
        assert e_l2 <= b_l2, (t, e_l2)
        assert e_pert <= b_pert, (t, e_pert)
        assert drift <= b_m, (t, drift)


def test_stochastic_rounding_is_reproducible(mlf):
    """The draws depend on node, layer and step only: three launch shapes
    and ways of splitting the steps give the same populations bit for bit;
    round-to-nearest films differ from them, and a film with stochastic
    rounding refuses graph capture."""
    import torch

    film, h0, _ = inputs.workload("film4_2d_512")
    res = []
    for launch, chunks in [((64, 5), [300]), ((256, 10), [7, 93, 200]), ((512, 37), [150, 150])]:
        g = mlf.Film(film, "f16", check_every=-1)
        g.set_rounding(True)
        assert g.get_rounding()
        g.set_launch(*launch)
        g.init(h0)
        for c in chunks:
            g.step(c)
        res.append(g.populations())
    assert all(np.array_equal(res[0], r) for r in res[1:])
    n = mlf.Film(film, "f16", check_every=-1)
    n.init(h0)
    n.step(300)
    assert not np.array_equal(n.populations(), res[0])
    c = mlf.Film(film, "f16", stream=torch.cuda.Stream())
    c.set_rounding(True)
    c.init(h0)
    with pytest.raises(mlf.MlfError) as e:
        c.capture(4)
    assert e.value.status == "EUNSUPPORTED"
