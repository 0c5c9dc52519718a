"""ctypes binding of the FP64 CPU oracle (``oracle/mlf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle exists to check the HIP implementation.
Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module; the product package never does.

Parameters arrive as a plain mapping (see ``paper_2409_16659_amd.inputs``) and
are copied into the oracle's own struct; nothing here is shared with the HIP
binding.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same source (the sanitizer build)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
MAX_LAYERS = 4
D2Q9, D1Q3 = 0, 1
OK, ENONPOSITIVE, ENONFINITE, EINVAL = 0, 1, 2, 3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("lattice", C.c_int),
        ("tau", C.c_double), ("hstar", C.c_double),
        ("exp_a", C.c_int), ("exp_b", C.c_int),
        ("gamma", C.c_double * MAX_LAYERS), ("mu", C.c_double * MAX_LAYERS),
        ("slip", C.c_double * MAX_LAYERS),
        ("spread", (C.c_double * MAX_LAYERS) * MAX_LAYERS),
    ]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER(_Params)
    sig = {
        "orc_create": (C.c_void_p, [P]),
        "orc_destroy": (None, [C.c_void_p]),
        "orc_init": (C.c_int, [C.c_void_p, _D, _D, _D]),
        "orc_step": (C.c_int, [C.c_void_p, C.c_long]),
        "orc_steps_done": (C.c_long, [C.c_void_p]),
        "orc_read": (None, [C.c_void_p, _D, _D, _D]),
        "orc_mass": (None, [C.c_void_p, _D]),
        "orc_get_f": (None, [C.c_void_p, _D]),
        "orc_set_f": (None, [C.c_void_p, _D]),
        "orc_set_threads": (None, [C.c_int]),
        "orc_get_threads": (C.c_int, []),
        "orc_lattice": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _D]),
        "orc_phi": (C.c_double, [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int]),
        "orc_dphi": (C.c_double, [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int]),
        "orc_spreading_from_tensions": (None, [C.c_int, _D, C.c_void_p]),
        "orc_grad": (None, [C.c_int, C.c_int, C.c_int, _D, _D, _D]),
        "orc_lap": (None, [C.c_int, C.c_int, C.c_int, _D, _D]),
        "orc_pressure": (C.c_int, [P, _D, _D, _D]),
        "orc_friction": (C.c_int, [C.c_int, _D, _D, _D, _D, _D]),
        "orc_equilibrium": (None, [C.c_int, C.c_double, C.c_double, C.c_double, _D]),
        "orc_forcing": (None, [C.c_int, C.c_double, C.c_double, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(film, lattice: int = D2Q9) -> _Params:
    """Copy a film parameter mapping into the oracle's struct."""
    p = _Params()
    n = int(film["n_layers"])
    p.n_layers = n
    p.nx, p.ny = int(film["nx"]), int(film["ny"])
    p.lattice = lattice
    p.tau = float(film.get("tau", 1.0))
    p.hstar = float(film["hstar"])
    p.exp_a, p.exp_b = int(film.get("exp_a", 9)), int(film.get("exp_b", 3))
    for i in range(n):
        p.gamma[i] = float(film["gamma"][i])
        p.mu[i] = float(film["mu"][i])
        p.slip[i] = float(film.get("slip", [0.0] * n)[i])
    for (l, k), v in dict(film.get("spread", {})).items():
        if not (0 <= l < n and 1 <= k <= n - l):
            raise ValueError(f"spreading coefficient S_{l}{k} out of range for N={n}")
        p.spread[l][k - 1] = float(v)
    return p


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def lattice(lat: int = D2Q9):
    lib = _load()
    cx = (C.c_int * 9)()
    cy = (C.c_int * 9)()
    w = (C.c_double * 9)()
    q = lib.orc_lattice(lat, cx, cy, w)
    return np.array(cx[:q]), np.array(cy[:q]), np.array(w[:q])


def phi(k, d, hstar, a=9, b=3):
    return _load().orc_phi(int(k), float(d), float(hstar), int(a), int(b))


def dphi(k, d, hstar, a=9, b=3):
    return _load().orc_dphi(int(k), float(d), float(hstar), int(a), int(b))


def spreading_from_tensions(n: int, g) -> dict:
    """S_lk from a full symmetric (N+2)x(N+2) tension table, as {(l, k): S}."""
    g = _f64(g)
    assert g.shape == (n + 2, n + 2)
    out = ((C.c_double * MAX_LAYERS) * MAX_LAYERS)()
    _load().orc_spreading_from_tensions(n, _ptr(g), C.byref(out))
    return {(l, k): out[l][k - 1] for l in range(n) for k in range(1, n - l + 1)}


def grad(f, lat: int = D2Q9):
    f = _f64(f)
    ny, nx = f.shape
    gx = np.empty_like(f)
    gy = np.empty_like(f)
    _load().orc_grad(lat, nx, ny, _ptr(f), _ptr(gx), _ptr(gy))
    return gx, gy


def lap(f, lat: int = D2Q9):
    f = _f64(f)
    ny, nx = f.shape
    out = np.empty_like(f)
    _load().orc_lap(lat, nx, ny, _ptr(f), _ptr(out))
    return out


def pressure(film, h, lat: int = D2Q9):
    """(p_i - p_atm, Delta_i) for heights h[N][ny][nx]."""
    p = make_params(film, lat)
    h = _f64(h)
    pres = np.empty_like(h)
    jump = np.empty_like(h)
    rc = _load().orc_pressure(C.byref(p), _ptr(h), _ptr(pres), _ptr(jump))
    if rc:
        raise OracleError(rc, "pressure")
    return pres, jump


def friction(h, mu, q, slip=None):
    h, mu, q = _f64(h), _f64(mu), _f64(q)
    n = h.shape[0]
    slip = _f64(np.zeros(n) if slip is None else slip)
    fr = np.empty(n)
    rc = _load().orc_friction(n, _ptr(h), _ptr(mu), _ptr(slip), _ptr(q), _ptr(fr))
    if rc:
        raise OracleError(rc, "friction")
    return fr


def equilibrium(h, ux, uy=0.0, lat: int = D2Q9):
    q = 3 if lat == D1Q3 else 9
    out = np.empty(q)
    _load().orc_equilibrium(lat, float(h), float(ux), float(uy), _ptr(out))
    return out


def forcing(fx, fy=0.0, lat: int = D2Q9):
    q = 3 if lat == D1Q3 else 9
    out = np.empty(q)
    _load().orc_forcing(lat, float(fx), float(fy), _ptr(out))
    return out


class Oracle:
    """One oracle film: populations f[N][Q][ny][nx] in FP64 host memory."""

    def __init__(self, film, lattice: int = D2Q9):
        self.lib = _load()
        self.film = dict(film)
        self.params = make_params(film, lattice)
        self.n = self.params.n_layers
        self.nx, self.ny = self.params.nx, self.params.ny
        self.q = 3 if lattice == D1Q3 else 9
        h = self.lib.orc_create(C.byref(self.params))
        if not h:
            raise OracleError(EINVAL, "create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_destroy(self.h)
            self.h = None

    def init(self, h, ux=None, uy=None):
        h = _f64(h)
        assert h.shape == (self.n, self.ny, self.nx)
        ux = None if ux is None else _f64(ux)
        uy = None if uy is None else _f64(uy)
        rc = self.lib.orc_init(self.h, _ptr(h), _ptr(ux), _ptr(uy))
        if rc:
            raise OracleError(rc, "init")

    def step(self, n: int = 1):
        rc = self.lib.orc_step(self.h, int(n))
        if rc:
            raise OracleError(rc, "step")

    @property
    def steps_done(self) -> int:
        return int(self.lib.orc_steps_done(self.h))

    def read(self):
        shape = (self.n, self.ny, self.nx)
        h, ux, uy = np.empty(shape), np.empty(shape), np.empty(shape)
        self.lib.orc_read(self.h, _ptr(h), _ptr(ux), _ptr(uy))
        return h, ux, uy

    def mass(self):
        m = np.empty(self.n)
        self.lib.orc_mass(self.h, _ptr(m))
        return m

    def get_f(self):
        f = np.empty((self.n, self.q, self.ny, self.nx))
        self.lib.orc_get_f(self.h, _ptr(f))
        return f

    def set_f(self, f):
        f = _f64(f)
        assert f.shape == (self.n, self.q, self.ny, self.nx)
        self.lib.orc_set_f(self.h, _ptr(f))
