"""CPU checks of the C-ABI library: it loads without a GPU, exports every
function include/mlfilm.h declares, its host helpers agree with the oracle,
and argument/failure handling returns the documented codes before any
device work.  No compute kernel runs here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2409_16659_amd import inputs, mlfilm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", hdr)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mlf_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = mlfilm.load_library()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert lib.mlf_version().startswith(b"mlfilm")


def test_params_struct_layout_matches_header():
    # offsets of the ABI struct as the C compiler lays it out
    p = mlfilm.Params
    assert p.tau.offset == 16 and p.hstar.offset == 24
    assert p.gamma.offset == 40 and p.mu.offset == 72 and p.slip.offset == 104
    assert p.spread.offset == 136 and p.check_every.offset == 216
    assert p.allow_unstable.offset == 220 and p.lattice.offset == 224
    assert C.sizeof(p) == 232


def _tension_table(n, rng):
    g = np.zeros((n + 2, n + 2))
    for i in range(n + 2):
        for j in range(i + 1, n + 2):
            g[i, j] = g[j, i] = rng.uniform(0.5, 2.0)
    return g


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_spreading_helper_matches_oracle(oracle_mod, n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        g = _tension_table(n, rng)
        a = mlfilm.spreading_from_tensions(n, g)
        b = oracle_mod.spreading_from_tensions(n, g)
        assert a.keys() == b.keys()
        for k in a:
            assert a[k] == b[k]


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_friction_matrix_matches_oracle(oracle_mod, n):
    """The library's interface-velocity tridiagonal solve against the
    oracle's elimination of the full boundary-condition system."""
    rng = np.random.default_rng(40 + n)
    for _ in range(20):
        h = rng.uniform(0.05, 3.0, size=n)
        mu = 10 ** rng.uniform(-4, -1, size=n)
        K, rate = mlfilm.friction_matrix(h, mu)
        Ko = np.stack([oracle_mod.friction(h, mu, np.eye(n)[j]) for j in range(n)], axis=1)
        assert np.abs(K - Ko).max() <= 1e-13 * np.abs(Ko).max()
        assert abs(rate - np.linalg.eigvals(-Ko).real.max()) <= 1e-9 * rate


def test_query_sizes_and_validation():
    film, _, _ = inputs.workload("film3_2d_1024")
    p = mlfilm.make_params(film, "f32")
    pop, scratch = mlfilm.query_sizes(p)
    assert pop == 1024 * 1024 * 9 * 3 * 4 and scratch >= 16 << 20
    assert mlfilm.query_pitch(p) == 1024
    p64 = mlfilm.make_params(inputs.film_params(2, 100, 3, gamma=[1, 1], mu=[1, 1], hstar=0.1), "f64")
    assert mlfilm.query_pitch(p64) == 128
    assert mlfilm.query_sizes(p64)[0] == 128 * 3 * 9 * 2 * 8
    # per layer: the rest plane, then eight moving planes of that plane type
    for prec, (rb, mb) in [("f16", (2, 2)), ("bf16", (2, 2)), ("f16mix", (4, 2)), ("bf16mix", (4, 2))]:
        q = mlfilm.make_params(film, prec)
        assert mlfilm.query_sizes(q)[0] == 1024 * 1024 * 3 * (rb + 8 * mb)
        assert mlfilm.bytes_per_update(prec) == 2 * (rb + 8 * mb)
    q = mlfilm.make_params(film, "f32")
    q.precision = 6
    with pytest.raises(mlfilm.MlfError):
        mlfilm.query_sizes(q)
    # each group of three planes must fit a 2 GiB buffer descriptor
    big = inputs.film_params(1, 16384, 10922, gamma=[1], mu=[1], hstar=0.1)
    assert mlfilm.query_sizes(mlfilm.make_params(big, "f32"))[0] == 16384 * 10922 * 9 * 4
    assert 16384 * 10922 * 3 * 4 <= 2 ** 31
    big["ny"] = 10923
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.query_sizes(mlfilm.make_params(big, "f32"))
    assert e.value.status == "EUNSUPPORTED"
    for field, val in [("n_layers", 0), ("n_layers", 5), ("nx", 0), ("tau", 0.5), ("hstar", 0.0),
                       ("exp_b", 9)]:
        q = mlfilm.make_params(film, "f32")
        setattr(q, field, val)
        with pytest.raises(mlfilm.MlfError) as e:
            mlfilm.query_sizes(q)
        assert e.value.status == "EINVAL"
    q = mlfilm.make_params(film, "f32")
    q.slip[0] = 0.1
    mlfilm.query_sizes(q)  # slip lengths >= 0 are supported
    q.slip[0] = -0.1
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.query_sizes(q)
    assert e.value.status == "EINVAL"


def _fake_handle(film, precision="f64", allow_unstable=False):
    """A handle bound to aligned dummy addresses: valid for the host-side
    checks of mlf_init, which run before any device access."""
    lib = mlfilm.load_library()
    p = mlfilm.make_params(film, precision, allow_unstable=allow_unstable)
    h = C.c_void_p()
    assert lib.mlf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20),
                          None, C.byref(h)) == 0
    return lib, h


def test_create_rejects_bad_buffers():
    lib = mlfilm.load_library()
    film = inputs.film_params(1, 8, 8, gamma=[0.01], mu=[0.01], hstar=0.1)
    p = mlfilm.make_params(film)
    h = C.c_void_p()
    assert lib.mlf_create(C.byref(p), None, C.c_void_p(512), C.c_void_p(1024), None, C.byref(h)) == -1
    assert lib.mlf_create(C.byref(p), C.c_void_p(512), C.c_void_p(512), C.c_void_p(1024), None, C.byref(h)) == -1
    assert lib.mlf_create(C.byref(p), C.c_void_p(513), C.c_void_p(1024), C.c_void_p(2048), None, C.byref(h)) == -1


def test_init_failure_paths_on_host():
    film = inputs.film_params(2, 6, 5, gamma=[0.01, 0.01], mu=[0.01, 0.01], hstar=0.1)
    lib, h = _fake_handle(film)
    D = C.POINTER(C.c_double)
    try:
        a = np.ones((2, 5, 6))
        a[1, 2, 3] = 0.0
        assert lib.mlf_init(h, a.ctypes.data_as(D), None, None) == -5
        a[1, 2, 3] = np.nan
        assert lib.mlf_init(h, a.ctypes.data_as(D), None, None) == -4
        assert b"not finite" in lib.mlf_last_error(h)
        assert lib.mlf_step(h, 1) == -1  # not initialised
    finally:
        lib.mlf_destroy(h)
    # viscosity far above the explicit-friction bound at h*
    stiff = inputs.film_params(1, 6, 5, gamma=[0.01], mu=[1.0], hstar=0.1)
    lib, h = _fake_handle(stiff)
    try:
        a = np.ones((1, 5, 6))
        assert lib.mlf_init(h, a.ctypes.data_as(D), None, None) == -6
        assert b"unstable" in lib.mlf_last_error(h)
    finally:
        lib.mlf_destroy(h)


def test_set_launch_validation():
    film = inputs.film_params(1, 300, 40, gamma=[0.01], mu=[0.01], hstar=0.1)
    lib, h = _fake_handle(film)
    try:
        a, b = C.c_int32(), C.c_int32()
        assert lib.mlf_get_launch(h, C.byref(a), C.byref(b)) == 0
        assert a.value == 256 and 1 <= b.value <= 40
        assert lib.mlf_set_launch(h, 96, 4) == -1
        assert lib.mlf_set_launch(h, 64, 0) == 0
        assert lib.mlf_set_launch(h, 0, 1000) == 0
        lib.mlf_get_launch(h, C.byref(a), C.byref(b))
        assert b.value == 40
    finally:
        lib.mlf_destroy(h)


def test_set_launch_512_lanes():
    """512-lane strips are accepted for every format except FP64 films of
    four layers, whose step kernel is compiled for at most 256 lanes."""
    for prec, n, ok in [("f32", 4, True), ("f64", 3, True), ("f16mix", 4, True), ("f64", 4, False)]:
        film = inputs.film_params(n, 300, 40, gamma=[0.01] * n, mu=[0.01] * n, hstar=0.1)
        lib, h = _fake_handle(film, prec)
        try:
            rc = lib.mlf_set_launch(h, 512, 8)
            assert (rc == 0) == ok, (prec, n)
            a, b = C.c_int32(), C.c_int32()
            lib.mlf_get_launch(h, C.byref(a), C.byref(b))
            if ok:
                assert (a.value, b.value) == (512, 8)
            else:
                assert b"512" in lib.mlf_last_error(h)
                assert a.value != 512
        finally:
            lib.mlf_destroy(h)


def test_set_prefetch_validation():
    """Two rows in flight need a D2Q9 film with tau = 1 and non-FP64
    storage; 0 selects the default of one row; other values are refused."""
    cases = [("f32", 1.0, 2, True), ("f16mix", 1.0, 2, True), ("f64", 1.0, 2, False), ("f32", 0.8, 2, False),
             ("f64", 0.8, 1, True), ("f32", 1.0, 3, False), ("f32", 1.0, -1, False)]
    for prec, tau, rows, ok in cases:
        film = inputs.film_params(2, 64, 16, gamma=[0.01] * 2, mu=[0.01] * 2, hstar=0.1, tau=tau)
        lib, h = _fake_handle(film, prec)
        try:
            v = C.c_int32()
            assert lib.mlf_get_prefetch(h, C.byref(v)) == 0 and v.value == 1
            rc = lib.mlf_set_prefetch(h, rows)
            assert (rc == 0) == ok, (prec, tau, rows)
            lib.mlf_get_prefetch(h, C.byref(v))
            assert v.value == (rows if ok else 1)
            if not ok:
                assert lib.mlf_last_error(h)
            assert lib.mlf_set_prefetch(h, 0) == 0
            lib.mlf_get_prefetch(h, C.byref(v))
            assert v.value == 1
        finally:
            lib.mlf_destroy(h)
    assert lib.mlf_get_prefetch(None, C.byref(C.c_int32())) != 0


def test_set_rounding_validation():
    """Stochastic rounding of the rest plane is for D2Q9 films with f16 or
    bf16 storage only; other modes are refused; 0 restores the default."""
    for prec, ok in [("f16", True), ("bf16", True), ("f16mix", False), ("f32", False), ("f64", False)]:
        film = inputs.film_params(2, 64, 16, gamma=[0.01] * 2, mu=[0.01] * 2, hstar=0.1)
        lib, h = _fake_handle(film, prec)
        try:
            v = C.c_int32()
            assert lib.mlf_get_rounding(h, C.byref(v)) == 0 and v.value == 0
            assert (lib.mlf_set_rounding(h, 1) == 0) == ok, prec
            lib.mlf_get_rounding(h, C.byref(v))
            assert v.value == (1 if ok else 0)
            assert lib.mlf_set_rounding(h, 2) != 0
            assert lib.mlf_set_rounding(h, 0) == 0
            lib.mlf_get_rounding(h, C.byref(v))
            assert v.value == 0
        finally:
            lib.mlf_destroy(h)


def test_batch_set_rounding_validation():
    """The batch form of the rounding mode: f16 / bf16 D2Q9 batches only,
    unknown modes refused, 0 restores the default (no device access)."""
    film = inputs.film_params(2, 64, 16, gamma=[0.01] * 2, mu=[0.01] * 2, hstar=0.1)
    lib = mlfilm.load_library()
    for prec, ok in [("f16", True), ("bf16", True), ("f16mix", False), ("f32", False)]:
        ps = (mlfilm.Params * 2)(*[mlfilm.make_params(film, prec)] * 2)
        b = C.c_void_p()
        assert lib.mlf_batch_create(ps, 2, C.c_void_p(1 << 20), C.c_void_p(1 << 28), C.c_void_p(1 << 29),
                                    None, C.byref(b)) == 0
        try:
            v = C.c_int32()
            assert lib.mlf_batch_get_rounding(b, C.byref(v)) == 0 and v.value == 0
            assert (lib.mlf_batch_set_rounding(b, 1) == 0) == ok, prec
            lib.mlf_batch_get_rounding(b, C.byref(v))
            assert v.value == (1 if ok else 0)
            assert lib.mlf_batch_set_rounding(b, 3) != 0
            assert lib.mlf_batch_set_rounding(b, 0) == 0
            lib.mlf_batch_get_rounding(b, C.byref(v))
            assert v.value == 0
            assert lib.mlf_batch_get_rounding(b, None) != 0
        finally:
            lib.mlf_batch_destroy(b)
    assert lib.mlf_batch_set_rounding(None, 1) != 0


def test_surrogate_sizes_and_validation():
    from oracle import nop

    p = mlfilm.NopParams(3, 256, 256, 128, 3, 64, 1e-2)
    n, w = C.c_size_t(), C.c_size_t()
    lib = mlfilm.load_library()
    assert lib.mlf_nop_query_sizes(C.byref(p), C.byref(n), C.byref(w)) == 0
    assert n.value == nop.layout(3, 128, 3)[1]
    assert 800_000 < n.value < 1_100_000  # about one million parameters
    for field, val in [("nx", 200), ("ny", 250), ("n_layers", 5), ("batch", 0), ("blocks", -1), ("scale", 0.0)]:
        q = mlfilm.NopParams(3, 256, 256, 128, 3, 64, 1e-2)
        setattr(q, field, val)
        assert lib.mlf_nop_query_sizes(C.byref(q), C.byref(n), C.byref(w)) == -1, field
    q = mlfilm.NopParams(3, 256, 256, 96, 3, 64, 1e-2)
    assert lib.mlf_nop_query_sizes(C.byref(q), C.byref(n), C.byref(w)) == -2
    # one latent image must index in 32 bits: (ny/4)(nx/4) C < 2^31
    q = mlfilm.NopParams(1, 16384, 16384, 128, 1, 1, 1e-2)
    assert lib.mlf_nop_query_sizes(C.byref(q), C.byref(n), C.byref(w)) == -1
    q = mlfilm.NopParams(1, 16384, 16380, 128, 1, 1, 1e-2)
    assert lib.mlf_nop_query_sizes(C.byref(q), C.byref(n), C.byref(w)) == -1   # ny % 16
    q = mlfilm.NopParams(1, 16384, 16368, 128, 1, 1, 1e-2)
    assert lib.mlf_nop_query_sizes(C.byref(q), C.byref(n), C.byref(w)) == 0


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_friction_matrix_with_slip_matches_oracle(oracle_mod, n):
    """Interface-velocity form with slip lengths against the oracle's
    3N x 3N elimination of the same boundary conditions."""
    rng = np.random.default_rng(40 + n)
    for _ in range(20):
        h = rng.uniform(0.05, 2.0, n)
        mu = rng.uniform(1e-3, 1e-1, n)
        slip = rng.uniform(0.0, 1.0, n) * (rng.uniform(size=n) < 0.7)
        K, rate = mlfilm.friction_matrix(h, mu, slip)
        Ko = np.stack([oracle_mod.friction(h, mu, np.eye(n)[j], slip) for j in range(n)], axis=1)
        assert np.abs(K - Ko).max() <= 1e-12 * np.abs(Ko).max()
        # with slip the spectrum of -K may hold complex pairs: the rate is the largest modulus
        assert abs(rate - np.abs(np.linalg.eigvals(-Ko)).max()) <= 1e-9 * rate
        # zero slip is the no-slip matrix
        K0, _ = mlfilm.friction_matrix(h, mu, np.zeros(n))
        assert np.array_equal(K0, mlfilm.friction_matrix(h, mu)[0])


def test_single_layer_slip_closed_form():
    """One layer: the profile u(s) = a s^2 + b s + c with u(-beta) = 0,
    u'(h) = 0 and mean U gives friction 2 mu h a = -2 mu h U / (2h^2/3 + 2h beta + beta^2)."""
    for h, mu, beta in [(1.0, 0.1, 0.0), (0.3, 0.02, 0.1), (2.0, 1.0, 5.0)]:
        K, _ = mlfilm.friction_matrix([h], [mu], [beta])
        want = -2 * mu * h / (2 * h * h / 3 + 2 * h * beta + beta * beta) / h  # per unit flux q = h U
        assert abs(K[0, 0] - want) <= 1e-13 * abs(want)


def test_d1q3_validation_and_sizes():
    film = inputs.film_params(2, 100, 1, gamma=[0.01, 0.01], mu=[0.01, 0.01], hstar=0.3)
    q9 = mlfilm.make_params(film, "f64")
    q3 = mlfilm.make_params(film, "f64", lattice="d1q3")
    b9, _ = mlfilm.query_sizes(q9)
    b3, _ = mlfilm.query_sizes(q3)
    assert b9 == 3 * b3 == 9 * mlfilm.query_pitch(q3) * 2 * 8   # three planes instead of nine
    for prec in ("f16", "bf16", "f16mix", "bf16mix"):
        with pytest.raises(mlfilm.MlfError) as e:
            mlfilm.query_sizes(mlfilm.make_params(film, prec, lattice="d1q3"))
        assert e.value.status == "EUNSUPPORTED"
    two_rows = inputs.film_params(2, 100, 2, gamma=[0.01, 0.01], mu=[0.01, 0.01], hstar=0.3)
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.query_sizes(mlfilm.make_params(two_rows, "f64", lattice="d1q3"))
    assert e.value.status == "EINVAL"
    q3.lattice = 7
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.query_sizes(q3)
    assert e.value.status == "EINVAL"
    # batches: one lattice per batch; D1Q3 films must fit one workgroup's LDS
    mlfilm.batch_query_sizes([mlfilm.make_params(film, "f64", lattice="d1q3")] * 3)
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.batch_query_sizes([mlfilm.make_params(film, "f64", lattice="d1q3"), mlfilm.make_params(film, "f64")])
    assert e.value.status == "EUNSUPPORTED"
    long_strip = inputs.film_params(2, 1100, 1, gamma=[0.01, 0.01], mu=[0.01, 0.01], hstar=0.3)
    mlfilm.query_sizes(mlfilm.make_params(long_strip, "f64", lattice="d1q3"))  # single film: one-step kernel
    with pytest.raises(mlfilm.MlfError) as e:
        mlfilm.batch_query_sizes([mlfilm.make_params(long_strip, "f32", lattice="d1q3")])
    assert e.value.status == "EUNSUPPORTED"
