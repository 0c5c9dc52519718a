"""ctypes binding of ``libmlfilm.so`` (C ABI in ``include/mlfilm.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies the device buffers (caller-owned, as the ABI requires) and
the stream.  If the library has not been built this module raises; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

MAX_LAYERS = 4
MAX_PAIRS = MAX_LAYERS * (MAX_LAYERS + 1) // 2
F64, F32, F16, BF16, F16_MIX, BF16_MIX = 0, 1, 2, 3, 4, 5
PRECISIONS = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "f16dev": F16, "bf16dev": BF16,
              "f16mix": F16_MIX, "bf16mix": BF16_MIX}
# bytes of (rest plane, one moving plane) per node
PLANE_BYTES = {F64: (8, 8), F32: (4, 4), F16: (2, 2), BF16: (2, 2), F16_MIX: (4, 2), BF16_MIX: (4, 2)}


def bytes_per_update(precision) -> int:
    """Algorithmic bytes per layer-node update: every population read once
    and written once."""
    code = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    r, m = PLANE_BYTES[code]
    return 2 * (r + 8 * m)
STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EDEVICE", -4: "ENONFINITE",
          -5: "ENONPOSITIVE", -6: "EUNSTABLE"}


class NopParams(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("width", C.c_int32),
                ("blocks", C.c_int32), ("batch", C.c_int32), ("scale", C.c_double)]


class MlfError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        super().__init__(f"{what} failed: {STATUS.get(code, code)}" + (f" ({detail})" if detail else ""))
        self.code = code
        self.status = STATUS.get(code, str(code))


class Params(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32),
        ("tau", C.c_double), ("hstar", C.c_double), ("exp_a", C.c_int32), ("exp_b", C.c_int32),
        ("gamma", C.c_double * MAX_LAYERS), ("mu", C.c_double * MAX_LAYERS),
        ("slip", C.c_double * MAX_LAYERS), ("spread", C.c_double * MAX_PAIRS),
        ("check_every", C.c_int32), ("allow_unstable", C.c_int32), ("lattice", C.c_int32),
    ]


_D = C.POINTER(C.c_double)
_lib = None


def load_library():
    """Load the built library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_2409_16659_amd.build")
    # torch ships its own HIP runtime under the soname the library links
    # against; loading torch first makes the library bind to that copy, so
    # that one runtime owns the device memory torch allocates for us.
    import torch  # noqa: F401

    lib = C.CDLL(path)
    P = C.POINTER(Params)
    H = C.c_void_p
    st = C.c_int
    sig = {
        "mlf_query_sizes": (st, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "mlf_query_pitch": (st, [P, C.POINTER(C.c_int32)]),
        "mlf_create": (st, [P, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(H)]),
        "mlf_init": (st, [H, _D, _D, _D]),
        "mlf_init_device": (st, [H, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_step": (st, [H, C.c_int64]),
        "mlf_read": (st, [H, _D, _D, _D]),
        "mlf_read_device": (st, [H, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_layer_mass": (st, [H, _D]),
        "mlf_layer_min": (st, [H, _D]),
        "mlf_layer_mass_static": (st, [H, C.c_void_p]),
        "mlf_step_until": (st, [H, C.c_int64, C.c_int32, _D, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
        "mlf_read_populations": (st, [H, _D]),
        "mlf_write_populations": (st, [H, _D]),
        "mlf_save": (st, [H, C.c_void_p, C.POINTER(C.c_size_t)]),
        "mlf_load": (st, [H, C.c_void_p, C.c_size_t]),
        "mlf_set_launch": (st, [H, C.c_int32, C.c_int32]),
        "mlf_set_prefetch": (st, [H, C.c_int32]),
        "mlf_get_prefetch": (st, [H, C.POINTER(C.c_int32)]),
        "mlf_set_rounding": (st, [H, C.c_int32]),
        "mlf_get_rounding": (st, [H, C.POINTER(C.c_int32)]),
        "mlf_get_launch": (st, [H, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "mlf_autotune": (st, [H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "mlf_capture": (st, [H, C.c_int32]),
        "mlf_steps_done": (C.c_int64, [H]),
        "mlf_last_error": (C.c_char_p, [H]),
        "mlf_destroy": (st, [H]),
        "mlf_batch_query_sizes": (st, [P, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "mlf_batch_create": (st, [P, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(H)]),
        "mlf_batch_init": (st, [H, C.c_int32, _D, _D, _D]),
        "mlf_batch_step": (st, [H, C.c_int64]),
        "mlf_batch_capture": (st, [H, C.c_int32]),
        "mlf_batch_read": (st, [H, C.c_int32, _D, _D, _D]),
        "mlf_batch_layer_mass": (st, [H, C.c_int32, _D]),
        "mlf_batch_layer_min": (st, [H, C.c_int32, _D]),
        "mlf_batch_layer_min_all": (st, [H, _D]),
        "mlf_batch_step_until": (st, [H, C.c_int64, C.c_int32, _D, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64)]),
        "mlf_batch_read_device": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_batch_init_device": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_batch_init_device_all": (st, [H, C.POINTER(C.c_void_p)]),
        "mlf_batch_init_device_all_u": (st, [H, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_void_p)]),
        "mlf_batch_read_device_all": (st, [H, C.POINTER(C.c_void_p)]),
        "mlf_batch_set_launch": (st, [H, C.c_int32, C.c_int32, C.c_int32]),
        "mlf_batch_set_prefetch": (st, [H, C.c_int32]),
        "mlf_batch_get_prefetch": (st, [H, C.POINTER(C.c_int32)]),
        "mlf_batch_set_rounding": (st, [H, C.c_int32]),
        "mlf_batch_get_rounding": (st, [H, C.POINTER(C.c_int32)]),
        "mlf_batch_get_launch": (st, [H, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "mlf_batch_autotune": (st, [H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
        "mlf_batch_steps_done": (C.c_int64, [H]),
        "mlf_batch_failed_film": (C.c_int32, [H]),
        "mlf_batch_last_error": (C.c_char_p, [H]),
        "mlf_batch_destroy": (st, [H]),
        "mlf_nop_query_sizes": (st, [C.POINTER(NopParams), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "mlf_nop_create": (st, [C.POINTER(NopParams), C.c_void_p, C.c_void_p, C.POINTER(H)]),
        "mlf_nop_set_params": (st, [H, C.POINTER(C.c_float)]),
        "mlf_nop_get_params": (st, [H, C.POINTER(C.c_float)]),
        "mlf_nop_predict": (st, [H, C.c_int32, C.c_void_p, C.c_void_p]),
        "mlf_nop_loss": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
        "mlf_nop_gradient": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_float),
                                  C.POINTER(C.c_double)]),
        "mlf_nop_train_step": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_float, C.POINTER(C.c_double)]),
        "mlf_nop_time_conv": (st, [H, C.c_int32, C.c_int32, C.POINTER(C.c_float)]),
        "mlf_nop_errors": (st, [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_convert_heights": (st, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
        "mlf_stokes_velocity": (st, [P, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
        "mlf_nop_steps_done": (C.c_int32, [H]),
        "mlf_nop_last_error": (C.c_char_p, [H]),
        "mlf_nop_destroy": (st, [H]),
        "mlf_spreading_from_tensions": (st, [C.c_int32, _D, _D]),
        "mlf_friction_matrix": (st, [C.c_int32, _D, _D, _D, _D]),
        "mlf_friction_matrix_slip": (st, [C.c_int32, _D, _D, _D, _D, _D]),
        "mlf_version": (C.c_char_p, []),
        "mlf_stream_probe": (st, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64,
                                  C.c_int32, C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


LATTICES = {"d2q9": 0, "d1q3": 1}


def make_params(film, precision="f64", check_every=0, allow_unstable=False, lattice="d2q9") -> Params:
    """Copy a film parameter mapping (see ``inputs``) into the ABI struct."""
    p = Params()
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    n = int(film["n_layers"])
    p.n_layers, p.nx, p.ny = n, int(film["nx"]), int(film["ny"])
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.tau = float(film.get("tau", 1.0))
    p.hstar = float(film["hstar"])
    p.exp_a, p.exp_b = int(film.get("exp_a", 9)), int(film.get("exp_b", 3))
    for i in range(n):
        p.gamma[i] = float(film["gamma"][i])
        p.mu[i] = float(film["mu"][i])
        p.slip[i] = float(film.get("slip", [0.0] * n)[i])
    idx = 0
    spread = dict(film.get("spread", {}))
    for l in range(n):
        for k in range(1, n - l + 1):
            p.spread[idx] = float(spread.get((l, k), 0.0))
            idx += 1
    for key in spread:
        l, k = key
        if not (0 <= l < n and 1 <= k <= n - l):
            raise ValueError(f"spreading coefficient S_{l}{k} out of range for N={n}")
    p.check_every = int(check_every)
    p.allow_unstable = 1 if allow_unstable else 0
    return p


def query_sizes(params: Params):
    lib = load_library()
    a, b = C.c_size_t(), C.c_size_t()
    rc = lib.mlf_query_sizes(C.byref(params), C.byref(a), C.byref(b))
    if rc:
        raise MlfError(rc, "mlf_query_sizes")
    return a.value, b.value


def query_pitch(params: Params) -> int:
    lib = load_library()
    v = C.c_int32()
    rc = lib.mlf_query_pitch(C.byref(params), C.byref(v))
    if rc:
        raise MlfError(rc, "mlf_query_pitch")
    return v.value


def spreading_from_tensions(n: int, g) -> dict:
    lib = load_library()
    g = _f64(g)
    out = np.zeros(MAX_PAIRS)
    rc = lib.mlf_spreading_from_tensions(int(n), _dp(g), _dp(out))
    if rc:
        raise MlfError(rc, "mlf_spreading_from_tensions")
    res, idx = {}, 0
    for l in range(n):
        for k in range(1, n - l + 1):
            res[(l, k)] = out[idx]
            idx += 1
    return res


def friction_matrix(h, mu, slip=None):
    """Friction matrix K (friction = K q) of one node and the largest
    eigenvalue of -K; slip lengths optional."""
    lib = load_library()
    h, mu = _f64(h), _f64(mu)
    n = h.shape[0]
    K = np.zeros((n, n))
    rate = C.c_double()
    if slip is None:
        rc = lib.mlf_friction_matrix(n, _dp(h), _dp(mu), _dp(K), C.byref(rate))
    else:
        rc = lib.mlf_friction_matrix_slip(n, _dp(h), _dp(mu), _dp(_f64(slip)), _dp(K), C.byref(rate))
    if rc:
        raise MlfError(rc, "mlf_friction_matrix")
    return K, rate.value


STREAM_MODES = {"read": 0, "write": 1, "copy": 2}
STREAM_SCHEDULES = {"chunked": 0, "grid": 1}


def stream_probe(mode, src, dst, nbytes, schedule="chunked", nontemporal=False, blocks=0, stream=None):
    """One pass of the library's streaming probe (``mlf_stream_probe``) over
    ``nbytes`` of the device tensors ``src``/``dst``; asynchronous on
    ``stream`` (default: torch's current stream)."""
    import torch

    lib = load_library()
    nbytes = int(nbytes)
    for t in (src, dst):
        if t is not None and t.numel() * t.element_size() < nbytes:
            raise ValueError("buffer smaller than nbytes")
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.mlf_stream_probe(STREAM_MODES[mode], STREAM_SCHEDULES[schedule], 1 if nontemporal else 0,
                              C.c_void_p(src.data_ptr() if src is not None else 0), C.c_void_p(dst.data_ptr()),
                              nbytes, int(blocks), C.c_void_p(s.cuda_stream))
    if rc:
        raise MlfError(rc, "mlf_stream_probe")


def convert_heights(src, dst, stream=None):
    """Copy heights between FP64 and FP32 device tensors of one shape
    (mlf_convert_heights) on `stream` (default: torch's current stream);
    returns dst."""
    import torch

    lib = load_library()
    assert src.is_contiguous() and dst.is_contiguous() and src.shape == dst.shape
    if src.dtype == torch.float64 and dst.dtype == torch.float32:
        to32 = 1
    elif src.dtype == torch.float32 and dst.dtype == torch.float64:
        to32 = 0
    else:
        raise ValueError("convert_heights needs FP64 -> FP32 or FP32 -> FP64")
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.mlf_convert_heights(C.c_void_p(src.data_ptr()), to32, C.c_void_p(dst.data_ptr()), src.numel(),
                                 C.c_void_p(s.cuda_stream))
    if rc:
        raise MlfError(rc, "mlf_convert_heights")
    return dst


def rupture_threshold(film):
    """Height at or below which a layer counts as ruptured (its first
    hole): 1.5 h*, the same for every layer."""
    return np.full(int(film["n_layers"]), 1.5 * float(film["hstar"]))


class Film:
    """One film on the current CUDA/HIP device.

    Device buffers are torch uint8 tensors owned by this object; the stream is
    torch's current stream at construction unless one is given.
    """

    def __init__(self, film, precision="f64", check_every=0, allow_unstable=False,
                 stream=None, device=None, lattice="d2q9"):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.film = dict(film)
        self.params = make_params(film, precision, check_every, allow_unstable, lattice)
        self.nq = 3 if self.params.lattice == LATTICES["d1q3"] else 9
        self.n, self.nx, self.ny = self.params.n_layers, self.params.nx, self.params.ny
        pop_bytes, scratch_bytes = query_sizes(self.params)
        self.pop_bytes, self.scratch_bytes = pop_bytes, scratch_bytes
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev
        self.pop_a = torch.empty(pop_bytes, dtype=torch.uint8, device=dev)
        self.pop_b = torch.empty(pop_bytes, dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._own_stream = stream is not None
        if self._own_stream:
            # the buffers come from torch's allocator on the current stream
            torch.cuda.current_stream(dev).synchronize()
        h = C.c_void_p()
        rc = self.lib.mlf_create(C.byref(self.params), C.c_void_p(self.pop_a.data_ptr()),
                                 C.c_void_p(self.pop_b.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise MlfError(rc, "mlf_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            if getattr(self, "_own_stream", False):
                self.stream.synchronize()  # the buffers are freed on torch's stream after this
            self.lib.mlf_destroy(self.h)
            self.h = None

    def _check(self, rc, what):
        if rc:
            detail = self.lib.mlf_last_error(self.h)
            raise MlfError(rc, what, detail.decode() if detail else "")

    def init(self, h, ux=None, uy=None):
        t = self.torch
        if isinstance(h, t.Tensor):
            if self._own_stream:
                t.cuda.current_stream(self.device).synchronize()
            args = [None if a is None else C.c_void_p(a.data_ptr()) for a in (h, ux, uy)]
            for a in (h, ux, uy):
                if a is not None:
                    assert a.dtype == t.float64 and a.is_contiguous() and a.device.type == "cuda"
                    assert tuple(a.shape) == (self.n, self.ny, self.nx)
            self._check(self.lib.mlf_init_device(self.h, *args), "mlf_init_device")
            return
        h = _f64(h)
        assert h.shape == (self.n, self.ny, self.nx)
        ux = None if ux is None else _f64(ux)
        uy = None if uy is None else _f64(uy)
        self._check(self.lib.mlf_init(self.h, _dp(h), _dp(ux), _dp(uy)), "mlf_init")

    def step(self, n=1):
        self._check(self.lib.mlf_step(self.h, int(n)), "mlf_step")

    def capture(self, steps):
        """Replay `steps` (even) step launches from a HIP graph; 0 drops it.
        Needs a non-default stream (pass stream=torch.cuda.Stream())."""
        self._check(self.lib.mlf_capture(self.h, int(steps)), "mlf_capture")

    @property
    def steps_done(self) -> int:
        return int(self.lib.mlf_steps_done(self.h))

    def read(self):
        shape = (self.n, self.ny, self.nx)
        h, ux, uy = np.empty(shape), np.empty(shape), np.empty(shape)
        self._check(self.lib.mlf_read(self.h, _dp(h), _dp(ux), _dp(uy)), "mlf_read")
        return h, ux, uy

    def read_device(self, out=None):
        t = self.torch
        shape = (self.n, self.ny, self.nx)
        if out is None:
            out = tuple(t.empty(shape, dtype=t.float64, device=self.device) for _ in range(3))
        ptrs = [None if a is None else C.c_void_p(a.data_ptr()) for a in out]
        self._check(self.lib.mlf_read_device(self.h, *ptrs), "mlf_read_device")
        return out

    def mass(self):
        m = np.empty(self.n)
        self._check(self.lib.mlf_layer_mass(self.h, _dp(m)), "mlf_layer_mass")
        return m

    def layer_min(self):
        """Per-layer minimum height (the heights read() returns)."""
        m = np.empty(self.n)
        self._check(self.lib.mlf_layer_min(self.h, _dp(m)), "mlf_layer_min")
        return m

    def step_until(self, max_steps, check_every=100, threshold=None):
        """Step until some layer's minimum height reaches its threshold
        (default: the rupture criterion, 1.5 h*), checked every check_every
        steps.  Returns (steps taken, layer or -1)."""
        thr = rupture_threshold(self.film) if threshold is None else _f64(threshold)
        taken, layer = C.c_int64(), C.c_int32()
        self._check(self.lib.mlf_step_until(self.h, int(max_steps), int(check_every), _dp(thr),
                                            C.byref(taken), C.byref(layer)), "mlf_step_until")
        return taken.value, layer.value

    def populations(self):
        f = np.empty((self.n, self.nq, self.ny, self.nx))
        self._check(self.lib.mlf_read_populations(self.h, _dp(f)), "mlf_read_populations")
        return f

    def set_populations(self, f):
        f = _f64(f)
        assert f.shape == (self.n, self.nq, self.ny, self.nx)
        self._check(self.lib.mlf_write_populations(self.h, _dp(f)), "mlf_write_populations")

    def save(self) -> bytes:
        n = C.c_size_t()
        self._check(self.lib.mlf_save(self.h, None, C.byref(n)), "mlf_save")
        buf = C.create_string_buffer(n.value)
        self._check(self.lib.mlf_save(self.h, buf, C.byref(n)), "mlf_save")
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.lib.mlf_load(self.h, buf, len(blob)), "mlf_load")

    def set_launch(self, block_w=0, seg_h=0):
        self._check(self.lib.mlf_set_launch(self.h, int(block_w), int(seg_h)), "mlf_set_launch")

    def set_prefetch(self, rows=0):
        self._check(self.lib.mlf_set_prefetch(self.h, int(rows)), "mlf_set_prefetch")

    def get_prefetch(self) -> int:
        v = C.c_int32()
        self._check(self.lib.mlf_get_prefetch(self.h, C.byref(v)), "mlf_get_prefetch")
        return v.value

    def set_rounding(self, stochastic: bool):
        """Stochastic rounding of the rest population (f16 / bf16 storage)."""
        self._check(self.lib.mlf_set_rounding(self.h, 1 if stochastic else 0), "mlf_set_rounding")

    def get_rounding(self) -> bool:
        v = C.c_int32()
        self._check(self.lib.mlf_get_rounding(self.h, C.byref(v)), "mlf_get_rounding")
        return v.value == 1

    def autotune(self, reps=5):
        """Pick the fastest launch shape on the current state (unchanged)."""
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.mlf_autotune(self.h, int(reps), C.byref(a), C.byref(b)), "mlf_autotune")
        return a.value, b.value

    def get_launch(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.mlf_get_launch(self.h, C.byref(a), C.byref(b)), "mlf_get_launch")
        return a.value, b.value


def batch_query_sizes(params_list):
    """(pop_bytes, scratch_bytes) of a batch of films (list of Params)."""
    lib = load_library()
    arr = (Params * len(params_list))(*params_list)
    a, b = C.c_size_t(), C.c_size_t()
    rc = lib.mlf_batch_query_sizes(arr, len(params_list), C.byref(a), C.byref(b))
    if rc:
        raise MlfError(rc, "mlf_batch_query_sizes")
    return a.value, b.value


class Batch:
    """Many independent films advanced by one launch per step (C ABI
    mlf_batch_*).  Films share the storage precision, tau and exponents.
    Buffers are torch uint8 tensors owned by this object; the batch runs on
    its own (default-priority) stream so that its step loop can be
    captured into a HIP graph."""

    def __init__(self, films, precision="f32", allow_unstable=False, stream=None, device=None, lattice="d2q9"):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.films = [dict(f) for f in films]
        self.params = [make_params(f, precision, 0, allow_unstable, lattice) for f in films]
        self.n = len(films)
        arr = (Params * self.n)(*self.params)
        pop_bytes, scratch_bytes = batch_query_sizes(self.params)
        self.pop_bytes, self.scratch_bytes = pop_bytes, scratch_bytes
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev
        self.pop_a = torch.empty(pop_bytes, dtype=torch.uint8, device=dev)
        self.pop_b = torch.empty(pop_bytes, dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        h = C.c_void_p()
        rc = self.lib.mlf_batch_create(arr, self.n, C.c_void_p(self.pop_a.data_ptr()),
                                       C.c_void_p(self.pop_b.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise MlfError(rc, "mlf_batch_create")
        # buffers allocated on the current stream are used on the batch's stream
        torch.cuda.current_stream(dev).synchronize()
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.stream.synchronize()  # the buffers are freed on torch's stream after this
            self.lib.mlf_batch_destroy(self.h)
            self.h = None

    def _check(self, rc, what):
        if rc:
            detail = self.lib.mlf_batch_last_error(self.h)
            raise MlfError(rc, what, detail.decode() if detail else "")

    def init(self, f, h, ux=None, uy=None):
        p = self.params[f]
        t = self.torch
        if isinstance(h, t.Tensor):
            assert h.dtype == t.float64 and h.is_cuda and h.is_contiguous()
            assert tuple(h.shape) == (p.n_layers, p.ny, p.nx) and ux is None and uy is None
            # h comes from torch's stream; the batch reads it on its own
            t.cuda.current_stream(self.device).synchronize()
            self._check(self.lib.mlf_batch_init_device(self.h, int(f), C.c_void_p(h.data_ptr()), None, None),
                        "mlf_batch_init_device")
            return
        h = _f64(h)
        assert h.shape == (p.n_layers, p.ny, p.nx)
        ux = None if ux is None else _f64(ux)
        uy = None if uy is None else _f64(uy)
        self._check(self.lib.mlf_batch_init(self.h, int(f), _dp(h), _dp(ux), _dp(uy)), "mlf_batch_init")

    def step(self, n=1):
        self._check(self.lib.mlf_batch_step(self.h, int(n)), "mlf_batch_step")

    def capture(self, steps):
        self._check(self.lib.mlf_batch_capture(self.h, int(steps)), "mlf_batch_capture")

    def read(self, f):
        p = self.params[f]
        shape = (p.n_layers, p.ny, p.nx)
        h, ux, uy = np.empty(shape), np.empty(shape), np.empty(shape)
        self._check(self.lib.mlf_batch_read(self.h, int(f), _dp(h), _dp(ux), _dp(uy)), "mlf_batch_read")
        return h, ux, uy

    def read_device(self, f, out=None):
        """Heights of film f as a device FP64 tensor [N][ny][nx], written
        asynchronously on the batch's stream: synchronise that stream before
        using it on another one."""
        p = self.params[f]
        t = self.torch
        if out is None:
            out = t.empty((p.n_layers, p.ny, p.nx), dtype=t.float64, device=self.device)
        assert out.dtype == t.float64 and out.is_contiguous() and tuple(out.shape) == (p.n_layers, p.ny, p.nx)
        self._check(self.lib.mlf_batch_read_device(self.h, int(f), C.c_void_p(out.data_ptr()), None, None),
                    "mlf_batch_read_device")
        return out

    def _ptrs(self, t):
        """Device pointers of the per-film slices of a [films][N][ny][nx] FP64 tensor."""
        p0 = self.params[0]
        T = self.torch
        assert all((p.n_layers, p.ny, p.nx) == (p0.n_layers, p0.ny, p0.nx) for p in self.params)
        assert t.dtype == T.float64 and t.is_cuda and t.is_contiguous()
        assert tuple(t.shape) == (self.n, p0.n_layers, p0.ny, p0.nx)
        step = t[0].numel() * 8
        return (C.c_void_p * self.n)(*[t.data_ptr() + f * step for f in range(self.n)])

    def init_all(self, h, ux=None, uy=None):
        """Initialise every film (all of one shape) from a device FP64 tensor
        [films][N][ny][nx] (and optional velocities of the same shape), with
        one synchronisation."""
        ptrs = self._ptrs(h)
        self.torch.cuda.current_stream(self.device).synchronize()
        if ux is None and uy is None:
            self._check(self.lib.mlf_batch_init_device_all(self.h, ptrs), "mlf_batch_init_device_all")
            return
        self._check(self.lib.mlf_batch_init_device_all_u(self.h, ptrs, self._ptrs(ux), self._ptrs(uy)),
                    "mlf_batch_init_device_all_u")

    def stokes_velocity(self, h, ux, uy):
        """Stokes-limit velocities (mlf_stokes_velocity) of every film's
        heights h into ux, uy (device FP64 tensors [films][N][ny][nx]), on the
        batch's stream."""
        hp, xp, yp = self._ptrs(h), self._ptrs(ux), self._ptrs(uy)
        # h may come from torch's stream; the batch reads it on its own
        self.torch.cuda.current_stream(self.device).synchronize()
        for f in range(self.n):
            rc = self.lib.mlf_stokes_velocity(C.byref(self.params[f]), hp[f], xp[f], yp[f],
                                              C.c_void_p(self.stream.cuda_stream))
            if rc:
                raise MlfError(rc, "mlf_stokes_velocity")

    def read_all(self, out=None):
        """Heights of every film (all of one shape) as a device FP64 tensor
        [films][N][ny][nx]; the batch's stream is synchronised before return."""
        p0 = self.params[0]
        if out is None:
            out = self.torch.empty((self.n, p0.n_layers, p0.ny, p0.nx), dtype=self.torch.float64,
                                   device=self.device)
        self._check(self.lib.mlf_batch_read_device_all(self.h, self._ptrs(out)), "mlf_batch_read_device_all")
        self.stream.synchronize()
        return out

    def read_all_hu(self, h, ux, uy):
        """Heights and velocities of every film (all of one shape) into device
        FP64 tensors [films][N][ny][nx]; the batch's stream is synchronised
        before return."""
        hp, xp, yp = self._ptrs(h), self._ptrs(ux), self._ptrs(uy)
        for f in range(self.n):
            self._check(self.lib.mlf_batch_read_device(self.h, f, hp[f], xp[f], yp[f]), "mlf_batch_read_device")
        self.stream.synchronize()
        return h, ux, uy

    def mass(self, f):
        m = np.empty(self.params[f].n_layers)
        self._check(self.lib.mlf_batch_layer_mass(self.h, int(f), _dp(m)), "mlf_batch_layer_mass")
        return m

    def layer_min(self, f):
        m = np.empty(self.params[f].n_layers)
        self._check(self.lib.mlf_batch_layer_min(self.h, int(f), _dp(m)), "mlf_batch_layer_min")
        return m

    def layer_min_all(self):
        """Minimum heights of every film, [n][MAX_LAYERS] (+inf past a
        film's layers), from one pass over the batch."""
        m = np.empty((self.n, MAX_LAYERS))
        self._check(self.lib.mlf_batch_layer_min_all(self.h, _dp(m)), "mlf_batch_layer_min_all")
        return m

    def step_until(self, max_steps, check_every=100, threshold=None):
        """Step the batch until every film has some layer at or below its
        threshold (default 1.5 h* per film) or max_steps have run.  Returns
        (t_hit, layer_hit, steps taken): t_hit[f] is the batch step count at
        the end of the chunk in which film f first got there (-1: never)."""
        thr = np.full((self.n, MAX_LAYERS), -np.inf)
        for f, film in enumerate(self.films):
            t = rupture_threshold(film) if threshold is None else _f64(threshold[f])
            thr[f, :len(t)] = t
        t_hit = np.empty(self.n, dtype=np.int64)
        layer = np.empty(self.n, dtype=np.int32)
        taken = C.c_int64()
        self._check(self.lib.mlf_batch_step_until(
            self.h, int(max_steps), int(check_every), _dp(thr),
            t_hit.ctypes.data_as(C.POINTER(C.c_int64)), layer.ctypes.data_as(C.POINTER(C.c_int32)),
            C.byref(taken)), "mlf_batch_step_until")
        return t_hit, layer, taken.value

    def set_launch(self, block_w=0, seg_h=0, persistent=0):
        self._check(self.lib.mlf_batch_set_launch(self.h, int(block_w), int(seg_h), int(persistent)),
                    "mlf_batch_set_launch")

    def set_prefetch(self, rows=0):
        self._check(self.lib.mlf_batch_set_prefetch(self.h, int(rows)), "mlf_batch_set_prefetch")

    def get_prefetch(self) -> int:
        v = C.c_int32()
        self._check(self.lib.mlf_batch_get_prefetch(self.h, C.byref(v)), "mlf_batch_get_prefetch")
        return v.value

    def set_rounding(self, stochastic: bool):
        """Stochastic rounding of every film's rest population (f16 / bf16
        storage); a film draws as it would stepped alone."""
        self._check(self.lib.mlf_batch_set_rounding(self.h, 1 if stochastic else 0), "mlf_batch_set_rounding")

    def get_rounding(self) -> bool:
        v = C.c_int32()
        self._check(self.lib.mlf_batch_get_rounding(self.h, C.byref(v)), "mlf_batch_get_rounding")
        return v.value == 1

    def get_launch(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.mlf_batch_get_launch(self.h, C.byref(a), C.byref(b), C.byref(c)),
                    "mlf_batch_get_launch")
        return a.value, b.value, c.value

    def autotune(self, reps=3):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.mlf_batch_autotune(self.h, int(reps), C.byref(a), C.byref(b), C.byref(c)),
                    "mlf_batch_autotune")
        return a.value, b.value, c.value

    @property
    def steps_done(self) -> int:
        return int(self.lib.mlf_batch_steps_done(self.h))

    @property
    def failed_film(self) -> int:
        return int(self.lib.mlf_batch_failed_film(self.h))


class Surrogate:
    """The learned surrogate (C ABI mlf_nop_*): a convolutional neural
    operator advancing layer heights by one window.  Heights are torch
    float32 CUDA tensors [batch][N][ny][nx]; parameters are a float32 numpy
    vector in the ABI's packing order."""

    def __init__(self, n_layers, nx, ny, width=128, blocks=3, batch=64, scale=1e-2, stream=None, device=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.p = NopParams(int(n_layers), int(nx), int(ny), int(width), int(blocks), int(batch), float(scale))
        n, w = C.c_size_t(), C.c_size_t()
        rc = self.lib.mlf_nop_query_sizes(C.byref(self.p), C.byref(n), C.byref(w))
        if rc:
            raise MlfError(rc, "mlf_nop_query_sizes")
        self.param_count, self.workspace_bytes = n.value, w.value
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = C.c_void_p()
        rc = self.lib.mlf_nop_create(C.byref(self.p), C.c_void_p(self.ws.data_ptr()),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise MlfError(rc, "mlf_nop_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.mlf_nop_destroy(self.h)
            self.h = None

    def _check(self, rc, what):
        if rc:
            d = self.lib.mlf_nop_last_error(self.h)
            raise MlfError(rc, what, d.decode() if d else "")

    def _dev(self, t):
        t = self.torch.as_tensor(t)
        assert t.dtype == self.torch.float32 and t.is_cuda and t.is_contiguous()
        assert t.dim() == 4 and tuple(t.shape[1:]) == (self.p.n_layers, self.p.ny, self.p.nx)
        return t

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.param_count
        self._check(self.lib.mlf_nop_set_params(self.h, v.ctypes.data_as(C.POINTER(C.c_float))), "mlf_nop_set_params")

    def get_params(self):
        v = np.empty(self.param_count, dtype=np.float32)
        self._check(self.lib.mlf_nop_get_params(self.h, v.ctypes.data_as(C.POINTER(C.c_float))), "mlf_nop_get_params")
        return v

    def predict(self, h, out=None):
        h = self._dev(h)
        out = self.torch.empty_like(h) if out is None else out
        self._check(self.lib.mlf_nop_predict(self.h, h.shape[0], C.c_void_p(h.data_ptr()), C.c_void_p(out.data_ptr())),
                    "mlf_nop_predict")
        return out

    def loss(self, h0, h1):
        h0, h1 = self._dev(h0), self._dev(h1)
        v = C.c_double()
        self._check(self.lib.mlf_nop_loss(self.h, h0.shape[0], C.c_void_p(h0.data_ptr()), C.c_void_p(h1.data_ptr()),
                                          C.byref(v)), "mlf_nop_loss")
        return v.value

    def gradient(self, h0, h1):
        h0, h1 = self._dev(h0), self._dev(h1)
        g = np.empty(self.param_count, dtype=np.float32)
        v = C.c_double()
        self._check(self.lib.mlf_nop_gradient(self.h, h0.shape[0], C.c_void_p(h0.data_ptr()),
                                              C.c_void_p(h1.data_ptr()), g.ctypes.data_as(C.POINTER(C.c_float)),
                                              C.byref(v)), "mlf_nop_gradient")
        return v.value, g

    def errors(self, a, b):
        """Per-sample (relative L2, perturbation-relative L2) errors of the
        FP32 height tensors a against the reference b (mlf_nop_errors, FP64
        reduction on the device), returned as a host array [S][2]."""
        a, b = self._dev(a), self._dev(b)
        assert a.shape == b.shape
        out = self.torch.empty((a.shape[0], 2), dtype=self.torch.float64, device=self.device)
        self._check(self.lib.mlf_nop_errors(self.h, a.shape[0], C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                            C.c_void_p(out.data_ptr())), "mlf_nop_errors")
        self.stream.synchronize()
        return out.cpu().numpy()

    def time_conv(self, batch, reps=20):
        """Average ms of one MFMA 3x3 convolution: forward with the plain,
        GELU and residual epilogues, and the weight gradient."""
        ms = (C.c_float * 4)()
        self._check(self.lib.mlf_nop_time_conv(self.h, int(batch), int(reps), ms), "mlf_nop_time_conv")
        return dict(zip(("fwd", "fwd_gelu", "fwd_resid", "wgrad"), list(ms)))

    def conv_flops(self, batch):
        """Multiply-add flops of one 3x3 convolution on `batch` samples."""
        return 2.0 * batch * (self.p.ny // 4) * (self.p.nx // 4) * 9 * self.p.width ** 2

    def train_step(self, h0, h1, lr):
        h0, h1 = self._dev(h0), self._dev(h1)
        v = C.c_double()
        self._check(self.lib.mlf_nop_train_step(self.h, h0.shape[0], C.c_void_p(h0.data_ptr()),
                                                C.c_void_p(h1.data_ptr()), float(lr), C.byref(v)),
                    "mlf_nop_train_step")
        return v.value
