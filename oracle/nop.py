"""Reference of the learned surrogate's network (test infrastructure only:
loaded by tests, never by the library or the benchmark's timed path).

Plain NumPy in FP64, written from the network's definition (see
include/mlf_surrogate.h): forward, loss, backward by the chain rule, and
one Adam step.  With bf16=True the values that the GPU rounds to bfloat16
before a matrix-core product (the inputs of every 3x3 convolution and its
weights, in the forward and both backward products) are rounded the same
way here (round to nearest even), so that the GPU and the reference differ
only by FP32 versus FP64 accumulation.  Pins (tests/test_nop_reference.py):
finite-difference gradients of the unrounded network, exact mass
conservation of the increment, and equivariance under periodic shifts by
whole patches.
"""
import math

import numpy as np

PATCH = 4


def bf16(a):
    """Round to bfloat16 (nearest even) and return as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layout(n_layers, width, blocks):
    """Offsets of the packed parameter vector (same order as the C ABI)."""
    C, J = width, n_layers * PATCH * PATCH
    off = {}
    o = 0

    def take(name, size):
        nonlocal o
        off[name] = (o, size)
        o += size

    take("We", J * C)
    take("be", C)
    for l in range(blocks):
        take(f"W1_{l}", 9 * C * C)
        take(f"b1_{l}", C)
        take(f"W2_{l}", 9 * C * C)
        take(f"b2_{l}", C)
    take("Wd", J * C)
    take("bd", J)
    return off, o


def unpack(vec, n_layers, width, blocks):
    C, J = width, n_layers * PATCH * PATCH
    off, n = layout(n_layers, width, blocks)
    assert vec.size == n
    shapes = {"We": (J, C), "be": (C,), "Wd": (J, C), "bd": (J,)}
    out = {}
    for k, (o, s) in off.items():
        shp = shapes.get(k, (9, C, C) if k.startswith("W") else (C,))
        out[k] = np.asarray(vec[o:o + s], dtype=np.float64).reshape(shp)
    return out


def pack(p, n_layers, width, blocks):
    off, n = layout(n_layers, width, blocks)
    v = np.zeros(n)
    for k, (o, s) in off.items():
        v[o:o + s] = np.asarray(p[k]).ravel()
    return v


def init_params(rng, n_layers, width, blocks):
    """He-style random initial parameters; the last conv of each block and
    the decoder start small so that the network starts near zero."""
    C, J = width, n_layers * PATCH * PATCH
    p = {"We": rng.normal(0, 1 / math.sqrt(J), (J, C)), "be": np.zeros(C)}
    for l in range(blocks):
        p[f"W1_{l}"] = rng.normal(0, math.sqrt(2 / (9 * C)), (9, C, C))
        p[f"b1_{l}"] = np.zeros(C)
        p[f"W2_{l}"] = rng.normal(0, 0.1 * math.sqrt(1 / (9 * C)), (9, C, C))
        p[f"b2_{l}"] = np.zeros(C)
    p["Wd"] = rng.normal(0, 0.1 / math.sqrt(C), (J, C))
    p["bd"] = np.zeros(J)
    return pack(p, n_layers, width, blocks)


def offsets9():
    """(dy, dx) of offset o = 3 (dy + 1) + (dx + 1)."""
    return [(o // 3 - 1, o % 3 - 1) for o in range(9)]


def shift(X, dy, dx):
    """Xs[b, y, x] = X[b, y + dy, x + dx], periodic."""
    return np.roll(X, (-dy, -dx), axis=(1, 2))


def conv3x3(X, W):
    """out[b, y, x, co] = sum_{o, ci} W[o, co, ci] X[b, y + dy_o, x + dx_o, ci]."""
    out = np.zeros(X.shape[:3] + (W.shape[1],))
    for o, (dy, dx) in enumerate(offsets9()):
        out += shift(X, dy, dx) @ W[o].T
    return out


def conv3x3_input_grad(dY, W):
    """Adjoint of conv3x3 w.r.t. X: dX[p, ci] = sum_{o, co} W[o, co, ci] dY[p - off_o, co]."""
    out = np.zeros(dY.shape[:3] + (W.shape[2],))
    for o, (dy, dx) in enumerate(offsets9()):
        out += shift(dY, -dy, -dx) @ W[o]
    return out


def conv3x3_weight_grad(X, dY):
    """dW[o, co, ci] = sum_p dY[p, co] X[p + off_o, ci]."""
    C_out, C_in = dY.shape[3], X.shape[3]
    dW = np.zeros((9, C_out, C_in))
    for o, (dy, dx) in enumerate(offsets9()):
        Xs = shift(X, dy, dx)
        dW[o] = dY.reshape(-1, C_out).T @ Xs.reshape(-1, C_in)
    return dW


GELU_K0 = math.sqrt(2.0 / math.pi)
GELU_K1 = 0.044715


def gelu(a):
    return 0.5 * a * (1 + np.tanh(GELU_K0 * (a + GELU_K1 * a ** 3)))


def gelu_grad(a):
    th = np.tanh(GELU_K0 * (a + GELU_K1 * a ** 3))
    return 0.5 * (1 + th) + 0.5 * a * (1 - th * th) * GELU_K0 * (1 + 3 * GELU_K1 * a * a)


def patches(x):
    """[B, N, ny, nx] -> [B, gy, gx, 16N], index j = (i * 4 + u) * 4 + v."""
    B, N, ny, nx = x.shape
    gy, gx = ny // PATCH, nx // PATCH
    return x.reshape(B, N, gy, PATCH, gx, PATCH).transpose(0, 2, 4, 1, 3, 5).reshape(B, gy, gx, N * PATCH * PATCH)


def unpatch(P, N):
    """Inverse of patches (pixel shuffle)."""
    B, gy, gx, _ = P.shape
    return P.reshape(B, gy, gx, N, PATCH, PATCH).transpose(0, 3, 1, 4, 2, 5).reshape(B, N, gy * PATCH, gx * PATCH)


class Net:
    def __init__(self, n_layers, width, blocks, scale, use_bf16=True):
        self.N, self.C, self.L, self.s = n_layers, width, blocks, float(scale)
        self.rnd = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))

    def forward(self, vec, h):
        """Projected increment Delta and the activations for backward."""
        p = unpack(vec, self.N, self.C, self.L)
        R = self.rnd
        h = np.asarray(h, dtype=np.float64)
        x = (h - h.mean(axis=(2, 3), keepdims=True)) / self.s
        P = patches(x)
        r = P @ p["We"] + p["be"]
        acts = []
        for l in range(self.L):
            rb = R(r)
            a = conv3x3(rb, R(p[f"W1_{l}"])) + p[f"b1_{l}"]
            gb = R(gelu(a))
            c = conv3x3(gb, R(p[f"W2_{l}"])) + p[f"b2_{l}"]
            acts.append((rb, a, gb))
            r = r + c
        Dl = r @ p["Wd"].T + p["bd"]
        D = unpatch(Dl, self.N)
        delta = D - D.mean(axis=(2, 3), keepdims=True)
        return delta, dict(P=P, acts=acts, rL=r, p=p)

    def predict(self, vec, h):
        delta, _ = self.forward(vec, h)
        return np.asarray(h, dtype=np.float64) + self.s * delta

    def loss(self, vec, h0, h1):
        delta, cache = self.forward(vec, h0)
        t = (np.asarray(h1, np.float64) - np.asarray(h0, np.float64)) / self.s
        return float(np.mean((delta - t) ** 2)), delta, t, cache

    def gradient(self, vec, h0, h1):
        L0, delta, t, cache = self.loss(vec, h0, h1)
        R = self.rnd
        p = cache["p"]
        g = {}
        dd = 2 * (delta - t) / delta.size
        dD = dd - dd.mean(axis=(2, 3), keepdims=True)      # adjoint of the projection
        dDl = patches(dD)
        rL = cache["rL"]
        g["Wd"] = dDl.reshape(-1, dDl.shape[-1]).T @ rL.reshape(-1, self.C)
        g["bd"] = dDl.reshape(-1, dDl.shape[-1]).sum(axis=0)
        dr = dDl @ p["Wd"]
        for l in reversed(range(self.L)):
            rb, a, gb = cache["acts"][l]
            dcb = R(dr)
            g[f"b2_{l}"] = dr.reshape(-1, self.C).sum(axis=0)
            g[f"W2_{l}"] = conv3x3_weight_grad(gb, dcb)
            dg = conv3x3_input_grad(dcb, R(p[f"W2_{l}"]))
            da = dg * gelu_grad(a)
            dab = R(da)
            g[f"b1_{l}"] = da.reshape(-1, self.C).sum(axis=0)
            g[f"W1_{l}"] = conv3x3_weight_grad(rb, dab)
            dr = dr + conv3x3_input_grad(dab, R(p[f"W1_{l}"]))
        P = cache["P"]
        g["We"] = P.reshape(-1, P.shape[-1]).T @ dr.reshape(-1, self.C)
        g["be"] = dr.reshape(-1, self.C).sum(axis=0)
        return L0, pack(g, self.N, self.C, self.L)


def adam_step(vec, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (vec, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return vec - lr * mh / (np.sqrt(vh) + eps), m, v
